"""Column-wise (l2,1) sparse term on the GPU against the FP64 oracle.

The penalty is the alternative named after eq_obj (Sec. 3), with the norm of
eq_rpca_l21 (Sec. 2): the S-step shrinks each column of B = X - L + Theta/rho
by max(0, 1 - 1/(rho ||B_j||)).  Iteration-locked steps from a state where both
the zero band and the shrink branch occur, whole solves on data with corrupted
columns, a sampled check at 10^4 x 10^4, and the argument checks."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1904_07497_amd import respca as rp  # noqa: E402
from paper_1904_07497_amd import synth  # noqa: E402
from tests._trajectory import column_support_check, trajectory  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL, F32_TOL = 1e-10, 1e-5


def dev(a, dtype=None):
    a = np.asfortranarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return torch.from_numpy(a).to("cuda")


def host(t):
    return np.asfortranarray(t.detach().cpu().numpy().astype(np.float64))


def rel(a, b, scale):
    den = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (den if den > 0 else scale)


def say(msg):
    print(msg, flush=True)


def _mixed_state(X, c, seed, rho):
    """An arbitrary state whose Theta columns have norms in [0.2, 1.5], so that at a
    small rho some columns of B fall inside the zero band and some outside."""
    st = synth.random_state(X, c, seed=seed, s_frac=0.2, s_amp=2.0)
    T = np.asarray(st["Theta"], np.float64)
    u = np.random.default_rng(seed + 1).uniform(0.2, 1.5, X.shape[1])
    st["Theta"] = np.asfortranarray((T * (u / np.linalg.norm(T, axis=0))).astype(X.dtype))
    st["rho"] = rho
    return st


def _gpu_state(st, dtype):
    return {"L": dev(st["L"], dtype), "S": dev(st["S"], dtype), "Theta": dev(st["Theta"], dtype),
            "labels": torch.from_numpy(st["labels"].copy()).to("cuda"),
            "C": dev(st["C"], dtype), "rho": st["rho"]}


def _column_support_check(X, L_or, Th_prev, rho, S_gpu, S_or, eps):
    """Zero and non-zero columns agree wherever rho ||B_j|| is well away from 1."""
    B = X - L_or + Th_prev / rho
    nb = np.linalg.norm(B, axis=0)
    scale = np.linalg.norm(np.abs(X) + np.abs(L_or) + np.abs(Th_prev) / rho, axis=0)
    sep = np.abs(rho * nb - 1.0) > 64 * eps * rho * scale * np.sqrt(X.shape[0])
    gz = np.linalg.norm(S_gpu, axis=0) == 0
    oz = np.linalg.norm(S_or, axis=0) == 0
    assert np.array_equal(gz[sep], oz[sep])
    return sep.mean(), oz.mean()


@pytest.mark.parametrize("dtype,precision", [(np.float64, rp.F64), (np.float32, rp.F32),
                                             (np.float32, rp.BF16GEMM_F32)])
def test_l21_iterate_matches_oracle_steps(dtype, precision):
    d, n, c = 2051, 333, 7
    say(f"l21 iterate {d}x{n} c={c} precision={precision}")
    X, _, _, _ = synth.clustered(d, n, c, seed=99, sep=3.0, noise=1.0, frac=0.1, amp=10.0,
                                 dtype=dtype)
    st = _mixed_state(X, c, 5, 0.002)
    lam = 0.8
    gs = _gpu_state(st, dtype)
    ost = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype != np.int32 else v)
           for k, v in st.items()}
    p = oracle.make_params(c, lam=lam, max_lloyd=1, sparse_norm=1)
    tol = F64_TOL if dtype == np.float64 else F32_TOL
    eps = np.finfo(dtype).eps
    Xo = X.astype(np.float64)
    nX = np.linalg.norm(Xo)
    zero_seen = shrink_seen = False
    for t in range(3):
        th_prev = ost["Theta"].copy()
        rho_t = ost["rho"]
        norms, info = rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=1, precision=precision,
                                 sparse_norm=1)
        ost = oracle.step(p, Xo, ost)
        np.testing.assert_array_equal(gs["labels"].cpu().numpy(), ost["labels"])
        for k in ("L", "S"):
            assert rel(host(gs[k]), ost[k], nX) <= tol, (t, k)
        assert rel(host(gs["Theta"]) / rho_t, ost["Theta"] / rho_t, nX) <= tol
        np.testing.assert_allclose(norms[0], ost["norms"],
                                   rtol=1e-3 if dtype == np.float32 else 1e-9,
                                   atol=1e-6 * nX if dtype == np.float32 else 1e-12 * nX)
        sep, zfrac = _column_support_check(Xo, ost["L"], th_prev, rho_t, host(gs["S"]), ost["S"],
                                           eps)
        assert sep > 0.95
        zero_seen |= zfrac > 0
        shrink_seen |= zfrac < 1
        # multiplier columns stay in the unit ball (subgradient of the column norms)
        assert np.linalg.norm(host(gs["Theta"]), axis=0).max() <= 1 + 1e-4
    assert zero_seen and shrink_seen


def _column_outliers(d, n, c, seed, dtype):
    """Grouped data with 5 % of the columns replaced by large Gaussian noise: the
    column-sparse corruption the l2,1 penalty is meant for."""
    X, _, _, _ = synth.clustered(d, n, c, seed=seed, sep=4.0, noise=0.5, frac=0.0, amp=0.0,
                                 dtype=np.float64)
    rng = np.random.default_rng(seed + 7)
    bad = rng.choice(n, max(1, n // 20), replace=False)
    X[:, bad] = rng.normal(0, 20.0, (d, bad.size))
    return np.asfortranarray(X.astype(dtype)), bad


@pytest.mark.parametrize("shape,dtype,precision", [
    ((517, 300, 4), np.float64, rp.F64),
    ((1000, 257, 3), np.float64, rp.F64),   # even d: the two-wide FP64 vector path
    ((1037, 777, 5), np.float32, rp.F32),
    ((2051, 300, 40), np.float32, rp.BF16GEMM_F32)])
def test_l21_solve_iteration_locked(shape, dtype, precision):
    d, n, c = shape
    say(f"l21 solve {shape} precision={precision}")
    X, _ = _column_outliers(d, n, c, d + n, dtype)
    lam = 0.05
    o = oracle.solve(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=2, sparse_norm=1))
    assert o["status"] == 0
    T = o["info"]["iters"]
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=2, precision=precision,
                 sparse_norm=1)
    assert g["status"] == rp.NOT_CONVERGED and g["info"]["iters"] == T
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    nX = np.linalg.norm(X.astype(np.float64))
    tol = F64_TOL if dtype == np.float64 else F32_TOL
    assert rel(host(g["L"]), o["L"], nX) <= tol
    assert rel(host(g["S"]), o["S"], nX) <= tol
    st, th_prev, rho_t, _ = trajectory(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=2,
                                                             sparse_norm=1), T)
    sep, zfrac = column_support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(g["S"]),
                                      st["S"], np.finfo(dtype).eps)
    say(f"l21 column support: {sep:.4f} separated, {zfrac:.4f} zero")
    assert sep > 0.95 and 0 < zfrac < 1
    # free-running: same stopping iteration
    g2 = rp.solve(dev(X), rank=c, lam=lam, tol=1e-6, seed=2, precision=precision, sparse_norm=1)
    assert abs(g2["info"]["iters"] - T) <= 1


def test_l21_iterate_full_size_sampled_columns():
    """10^4 x 10^4, rank 100, 10 % corruptions, c = 100, FP32: one l2,1 iteration from
    an arbitrary state, checked at sampled columns (the factor of a column depends
    only on that column, the group means on all of them)."""
    d = n = 10000
    c = 100
    say("l21 full-size iterate: generating")
    X, _, _ = synth.config_large(1, np.float32)
    rho = 2e-4   # about 60 % of the sampled columns in the zero band
    st = _mixed_state(X, c, 8, rho)
    lam = 0.01
    gs = _gpu_state(st, np.float32)
    say("l21 full-size iterate: gpu")
    rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=1, sparse_norm=1)
    rng = np.random.default_rng(0)
    sel = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)]))
    say("l21 full-size iterate: oracle")
    o = oracle.step_columns(oracle.make_params(c, lam=lam, max_lloyd=1, sparse_norm=1), X, st, sel)
    Xo = X[:, sel].astype(np.float64)
    idx = torch.from_numpy(sel).cuda()
    for k in ("L", "S"):
        assert rel(host(gs[k][:, idx]), o[k], np.linalg.norm(Xo)) <= F32_TOL, k
    assert rel(host(gs["Theta"][:, idx]) / rho, o["Theta"] / rho, np.linalg.norm(Xo)) <= F32_TOL
    oz = np.linalg.norm(o["S"], axis=0) == 0
    assert oz.any() and not oz.all()


def test_l21_argument_checks():
    Xh = np.random.default_rng(3).normal(size=(40, 30)).astype(np.float32)
    X = dev(Xh)
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=3, sparse_norm=2)
    assert e.value.status == rp.ERR_INVALID
    Xs = [X, dev(Xh[:, :20])]
    params, _ = rp.batch_params([3, 2])
    params[1].sparse_norm = 1
    with pytest.raises(rp.RespcaError) as e:
        rp.solve_batched(Xs, params)
    assert e.value.status == rp.ERR_UNSUPPORTED
