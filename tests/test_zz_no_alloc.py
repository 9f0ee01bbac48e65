"""respca_iterate_noalloc (workspace from the library's fixed per-GPU scratch
array) against respca_iterate on the same states, through the C ABI.

Bars as in the other parity tests: relative Frobenius error <= 1e-10 (FP64) or
<= 1e-5 (FP32) on L, S and Theta/rho, labels and Lloyd counts equal.  Two calls
in a row, the second on a smaller problem, so the second reuses an array that
still holds the first call's contents.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1904_07497_amd import respca as rp  # noqa: E402
from paper_1904_07497_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda")


def _state(X, c, seed):
    st = synth.random_state(X, c, seed=seed, s_frac=0.2, s_amp=2.0)
    return {"L": _dev(st["L"]), "S": _dev(st["S"]), "Theta": _dev(st["Theta"]),
            "labels": torch.from_numpy(st["labels"].copy()).to("cuda"), "C": _dev(st["C"]),
            "rho": 0.05}


def _clone(st):
    return {k: (v.clone() if torch.is_tensor(v) else v) for k, v in st.items()}


def _rel(a, b):
    a = a.double().cpu().numpy()
    b = b.double().cpu().numpy()
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


# (d, n, c, dtype, precision, sparse_norm): the second case of each pair is smaller
CALLS = [
    [(2051, 1333, 40, np.float32, rp.BF16GEMM_F32, 0), (517, 300, 7, np.float32, rp.F32, 0)],
    [(1037, 777, 9, np.float64, rp.F64, 0), (300, 211, 5, np.float64, rp.F64, 1)],
    [(1500, 1200, 100, np.float32, rp.F32, 1), (96, 80, 3, np.float32, rp.BF16GEMM_F32, 0)],
]


@pytest.mark.parametrize("calls", CALLS)
def test_noalloc_iterate_matches_iterate(calls):
    for i, (d, n, c, dtype, prec, norm) in enumerate(calls):
        print(f"noalloc call {i}: d={d} n={n} c={c} {np.dtype(dtype).name} precision={prec} "
              f"sparse_norm={norm}", flush=True)
        X, _, _, _ = synth.clustered(d, n, c, seed=31 + i, sep=3.0, noise=1.0, frac=0.1,
                                     amp=10.0, dtype=dtype)
        Xd = _dev(X)
        ref = _state(X, c, seed=7 + i)
        got = _clone(ref)
        kw = dict(iters=3, lam=0.8, max_lloyd=100, precision=prec, sparse_norm=norm)
        n_ref, i_ref = rp.iterate(Xd, ref, **kw)
        n_got, i_got = rp.iterate(Xd, got, noalloc=True, **kw)
        tol = 1e-10 if dtype == np.float64 else 1e-5
        assert torch.equal(got["labels"], ref["labels"])
        assert i_got["lloyd_steps"] == i_ref["lloyd_steps"] and i_got["iters"] == 3
        assert got["rho"] == ref["rho"]
        for k in ("L", "S", "C"):
            assert _rel(got[k], ref[k]) <= tol, k
        assert _rel(got["Theta"] / ref["rho"], ref["Theta"] / ref["rho"]) <= tol
        np.testing.assert_allclose(n_got, n_ref, rtol=tol)


def test_noalloc_rejects_a_problem_beyond_the_scratch_size_before_any_work():
    """d = 2 * 10^6 rows, n = 64 columns, c = 4: the group partial sums alone need
    (1 + 4) * d doubles = 80 MB, more than the 64 MiB array; the call fails with
    RESPCA_ERR_UNSUPPORTED and leaves the state untouched, and a normal call on the
    same handle still works afterwards."""
    d, n, c = 2_000_000, 64, 4
    g = torch.Generator(device="cuda").manual_seed(3)

    def cm(t):   # column-major copy
        return t.T.contiguous().T

    X = torch.randn(n, d, device="cuda", generator=g).T
    st = {"L": torch.randn(n, d, device="cuda", generator=g).T,
          "S": torch.zeros(n, d, device="cuda").T, "Theta": torch.zeros(n, d, device="cuda").T,
          "labels": (torch.arange(n, device="cuda", dtype=torch.int32) % c),
          "C": rp.empty_colmajor(d, c, torch.float32, "cuda").zero_(), "rho": 0.1}
    before = _clone(st)
    with pytest.raises(rp.RespcaError) as e:
        rp.iterate(X, st, iters=1, lam=1.0, noalloc=True)
    assert e.value.status == rp.ERR_UNSUPPORTED
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    for k in ("L", "S", "Theta", "labels", "C"):
        assert torch.equal(st[k], before[k]), k
    assert st["rho"] == before["rho"]
    # the first 1000 rows (leading dimension 2 * 10^6): fits, and matches respca_iterate
    dd = 1000
    small = X[:dd]
    st2 = {"L": cm(st["L"][:dd]), "S": cm(st["S"][:dd]), "Theta": cm(st["Theta"][:dd]),
           "labels": st["labels"].clone(),
           "C": rp.empty_colmajor(dd, c, torch.float32, "cuda").zero_(), "rho": 0.1}
    ref = _clone(st2)
    rp.iterate(small, ref, iters=1, lam=1.0)
    rp.iterate(small, st2, iters=1, lam=1.0, noalloc=True)
    assert torch.equal(st2["labels"], ref["labels"])
    for k in ("L", "S", "C"):
        assert _rel(st2[k], ref[k]) <= 1e-5, k
