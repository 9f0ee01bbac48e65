"""Anomaly scores (Sec. 5.3: the l2 norms of the columns of the recovered S) on
the GPU against the FP64 oracle: the scores of given matrices (FP64 and FP32,
padded leading dimensions, ragged shapes, the empty cases and the argument
checks), and the scores of an l2,1 solve on data with planted outlier columns,
iteration-locked to the oracle's solve."""
import ctypes as ct

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1904_07497_amd import respca as rp  # noqa: E402
from tests.test_oracle_pins import _planted_outlier_columns  # noqa: E402

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


def padded(a, dtype, pad):
    """A (d, n) column-major device tensor with leading dimension d + pad."""
    d, n = a.shape
    buf = torch.full((n, d + pad), float("nan"), dtype=dtype, device="cuda")
    buf[:, :d] = torch.from_numpy(np.ascontiguousarray(a.T)).to(dtype)
    return buf.T[:d, :]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("d,n,pad", [(1037, 777, 3), (1, 5, 0), (4096, 3, 5), (300, 70000, 1)])
def test_column_norms_match_oracle(dtype, d, n, pad):
    say(f"column norms {dtype} {d}x{n} pad {pad}")
    rng = np.random.default_rng(d + n)
    a = rng.normal(size=(d, n)) * (rng.random((d, n)) < 0.3)   # sparse, with zero columns
    a[:, ::7] = 0.0
    if dtype == torch.float32:
        a = a.astype(np.float32).astype(np.float64)
    got = rp.column_norms(padded(a, dtype, pad)).cpu().numpy()
    want = oracle.column_norms(np.asfortranarray(a))
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=0.0)
    assert np.all(got[::7] == 0.0)


def test_column_norms_empty_cases_and_argument_checks():
    L = rp.lib()
    h = rp.handle(0)
    out = torch.full((5,), -1.0, dtype=torch.float64, device="cuda")
    # d = 0: every column is empty, its norm zero
    assert L.respca_column_norms(h._h, rp.F32, 0, 5, None, 1, out.data_ptr(), None) == rp.OK
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [0.0] * 5
    # n = 0: nothing to do, nothing read
    assert L.respca_column_norms(h._h, rp.F64, 4, 0, None, 4, None, None) == rp.OK
    S = torch.zeros((3, 4), dtype=torch.float32, device="cuda").T   # (4, 3) column-major, ld 4
    for prec, d, n, lds, sp, op in [(7, 4, 3, 4, S.data_ptr(), out.data_ptr()),      # precision
                                    (rp.F32, 4, 3, 3, S.data_ptr(), out.data_ptr()),  # lds < d
                                    (rp.F32, -1, 3, 4, S.data_ptr(), out.data_ptr()),  # d < 0
                                    (rp.F32, 4, 3, 4, None, out.data_ptr()),          # S null
                                    (rp.F32, 4, 3, 4, S.data_ptr(), None)]:           # out null
        assert L.respca_column_norms(h._h, prec, d, n, sp, lds, op, None) == rp.ERR_INVALID


@pytest.mark.parametrize("precision", [rp.F64, rp.F32])
def test_l21_solve_scores_flag_the_planted_outlier_columns(precision):
    """The Sec. 5.3 experiment in miniature on the GPU: both solves stop at the
    oracle's iteration; the ten largest scores are the planted outlier columns,
    the inlier scores are zero, and the score vector matches the oracle's."""
    X, out_idx, c = _planted_outlier_columns()
    dtype = np.float64 if precision == rp.F64 else np.float32
    Xd = X.astype(dtype)
    o = oracle.solve(Xd, oracle.make_params(c, lam=0.1, tol=1e-7, sparse_norm=1, seed=0))
    T = o["info"]["iters"]
    g = rp.solve(torch.from_numpy(np.asfortranarray(Xd)).cuda(), rank=c, lam=0.1, tol=0.0,
                 max_iter=T, seed=0, sparse_norm=1, precision=precision)
    assert g["info"]["iters"] == T
    sc = rp.column_norms(g["S"]).cpu().numpy()
    osc = oracle.column_norms(o["S"])
    say(f"scores: top {np.round(np.sort(sc)[::-1][:11], 3)}")
    np.testing.assert_array_equal(np.sort(np.argsort(-sc)[:10]), out_idx)
    inl = np.setdiff1d(np.arange(X.shape[1]), out_idx)
    assert np.all(sc[inl] == 0.0)
    tol = 1e-10 if precision == rp.F64 else 1e-5
    assert np.linalg.norm(sc - osc) <= tol * np.linalg.norm(osc)
