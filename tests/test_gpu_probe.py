"""The streaming bandwidth probe through the C ABI (measurement support): both load
and store forms run and report a positive rate, and arguments outside the
documented ranges are refused without a launch."""
import pytest

pytest.importorskip("torch")

from paper_1904_07497_amd import respca as rp  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nontemporal", [False, True])
@pytest.mark.parametrize("reads,writes", [(1, 0), (3, 2), (4, 3)])
def test_probe_reports_a_rate(reads, writes, nontemporal):
    print(f"probe {reads}r{writes}w nontemporal={nontemporal}", flush=True)
    gbps, ms = rp.bandwidth_probe(reads, writes, 16 << 20, reps=2, nontemporal=nontemporal)
    assert ms > 0.0
    assert 0.0 < gbps < 1e5   # GB/s: positive and below any plausible memory rate


@pytest.mark.parametrize("reads,writes,nbytes", [(0, 1, 1 << 20), (5, 0, 1 << 20), (1, 4, 1 << 20),
                                                  (1, 1, 1000)])
def test_probe_rejects_bad_arguments(reads, writes, nbytes):
    with pytest.raises(rp.RespcaError):
        rp.bandwidth_probe(reads, writes, nbytes, reps=1)
