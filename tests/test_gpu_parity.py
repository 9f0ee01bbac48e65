"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (relative Frobenius error, denominator the oracle's norm or ||X||_F when
that is zero): <= 1e-10 for FP64 runs, <= 1e-5 for FP32 runs.  Integer outputs
(labels, iteration and Lloyd counts) must match exactly wherever the decision
is well separated; the support of S must match on well-separated entries.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1904_07497_amd import respca as rp  # noqa: E402
from paper_1904_07497_amd import synth  # noqa: E402
from tests._trajectory import support_check, trajectory  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL, F32_TOL = 1e-10, 1e-5


def dev(a, dtype=None):
    a = np.asfortranarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return torch.from_numpy(a).to("cuda")


def host(t):
    return np.asfortranarray(t.detach().cpu().numpy().astype(np.float64))


def rel(a, b, scale_fallback):
    den = np.linalg.norm(b)
    if den == 0:
        den = scale_fallback
    return np.linalg.norm(np.asarray(a, np.float64) - b) / den


def say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ K-means

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape", [(300, 500, 6), (1037, 211, 9), (5, 64, 3)])
def test_kmeans_matches_oracle_on_grouped_data(dtype, shape):
    d, n, c = shape
    say(f"kmeans {dtype.__name__} {shape}")
    X, _, _, g = synth.clustered(d, n, c, seed=d + n, sep=3.0, noise=0.5, frac=0.02, amp=5.0,
                                 dtype=dtype)
    prec = rp.F64 if dtype == np.float64 else rp.F32
    for seed in (0, 7):
        lab, C, info = rp.kmeans(dev(X), c, seed=seed, precision=prec)
        ol, oC, osteps = oracle.kmeans(X, c, seed)
        np.testing.assert_array_equal(lab.cpu().numpy(), ol)
        assert info["init_lloyd"] == osteps
        tol = F64_TOL if dtype == np.float64 else F32_TOL
        assert rel(host(C), oC, 1.0) <= tol


def test_kmeans_f64_unstructured_small_config():
    X, _, _ = synth.config_small(0)
    lab, C, info = rp.kmeans(dev(X), 25, seed=0, precision=rp.F64)
    ol, oC, osteps = oracle.kmeans(X, 25, 0)
    np.testing.assert_array_equal(lab.cpu().numpy(), ol)
    assert info["init_lloyd"] == osteps
    assert rel(host(C), oC, 1.0) <= F64_TOL


# ------------------------------------------------------------ whole solves

@pytest.mark.parametrize("lam", [1 / np.sqrt(500), np.sqrt(500)])
def test_solve_f64_small_config(lam):
    """500 x 500, rank 25, 5 % corruptions in [-50, 50], c = 25, tol 1e-7, FP64."""
    X, _, _ = synth.config_small(0)
    say(f"solve f64 500x500 lam={lam}")
    g = rp.solve(dev(X), rank=25, lam=lam, tol=1e-7, seed=0, precision=rp.F64)
    o = oracle.solve(X, oracle.make_params(25, lam=lam, tol=1e-7, seed=0))
    gi, oi = g["info"], o["info"]
    assert g["status"] == rp.OK and o["status"] == 0
    assert (gi["iters"], gi["lloyd_steps"], gi["init_lloyd"]) == \
        (oi["iters"], oi["lloyd_steps"], oi["init_lloyd"])
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    nX = np.linalg.norm(X)
    assert rel(host(g["L"]), o["L"], nX) <= F64_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F64_TOL
    assert abs(gi["primal"] - oi["primal"]) <= 1e-9 * max(oi["primal"], 1e-12) + 1e-16
    st, th_prev, rho_t, _ = trajectory(X, oracle.make_params(25, lam=lam, tol=1e-7, seed=0),
                                       max_iter=oi["iters"])
    frac = support_check(X, st["L"], th_prev, rho_t, host(g["S"]), st["S"], np.finfo(np.float64).eps)
    say(f"S support: {frac:.4f} of entries separated")
    assert frac > 0.99


@pytest.mark.parametrize("shape,lam", [((1037, 777, 5), None), ((2051, 300, 7), 0.3),
                                       ((64, 1000, 4), None), ((4096, 130, 3), 2.0)])
def test_solve_f32_grouped_iteration_locked(shape, lam):
    """FP32 GPU vs FP64 oracle on data with the model's group structure, ragged
    tails in both dimensions; both run exactly the iteration count the oracle
    needs for tol 1e-6 (so a stop near the threshold cannot mask a mismatch)."""
    d, n, c = shape
    say(f"solve f32 {shape} lam={lam}")
    X, _, _, _ = synth.clustered(d, n, c, seed=d * 3 + n, sep=4.0, noise=0.5, frac=0.05, amp=10.0,
                                 dtype=np.float32)
    lam = float(np.sqrt(max(d, n))) if lam is None else lam
    o = oracle.solve(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=1))
    T = o["info"]["iters"]
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=1)
    assert g["status"] == rp.NOT_CONVERGED and g["info"]["iters"] == T
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F32_TOL
    st, th_prev, rho_t, _ = trajectory(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=1), T)
    frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(g["S"]), st["S"],
                         np.finfo(np.float32).eps)
    say(f"S support: {frac:.4f} of entries separated")
    assert frac > 0.5
    # free-running: same stopping iteration
    g2 = rp.solve(dev(X), rank=c, lam=lam, tol=1e-6, seed=1)
    assert abs(g2["info"]["iters"] - T) <= 1


@pytest.mark.parametrize("dtype,d,n", [(np.float64, 3000, 3000), (np.float32, 4096, 4200)])
def test_solve_above_the_nontemporal_size_iteration_locked(dtype, d, n):
    """Arrays of 64 MiB and more take the nontemporal forms of the sweep and the
    means passes (FP64: double2 loads and stores): six iterations, iteration-locked
    to the oracle, on grouped data; labels equal, L and S within the precision's bar,
    the support of S equal on well-separated entries."""
    c, T = 6, 6
    assert d * n * np.dtype(dtype).itemsize >= 64 << 20
    say(f"solve {np.dtype(dtype).name} {d}x{n} above the nontemporal size")
    X, _, _, _ = synth.clustered(d, n, c, seed=17, sep=4.0, noise=0.5, frac=0.05, amp=10.0,
                                 dtype=dtype)
    lam = float(np.sqrt(max(d, n)))
    prm = oracle.make_params(c, lam=lam, tol=0.0, max_iter=T, seed=2)
    o = oracle.solve(X, prm)
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=2,
                 precision=rp.F64 if dtype == np.float64 else rp.F32)
    assert g["info"]["iters"] == o["info"]["iters"] == T
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    tol = F64_TOL if dtype == np.float64 else F32_TOL
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= tol
    assert rel(host(g["S"]), o["S"], nX) <= tol
    st, th_prev, rho_t, _ = trajectory(X, prm, T)
    frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(g["S"]), st["S"],
                         np.finfo(dtype).eps)
    say(f"S support: {frac:.4f} of entries separated")
    assert frac > 0.5


@pytest.mark.parametrize("precision", [rp.F32, rp.BF16GEMM_F32])
def test_solve_single_lloyd_step_matches_oracle(precision):
    """p-step of one Lloyd assignment per outer iteration (max_lloyd = 1, also for
    the initial K-means): iteration-locked whole solve against the oracle run with
    the same option (labels, iteration and Lloyd counts, L and S)."""
    d, n, c = 1500, 900, 12
    X, _, _, _ = synth.clustered(d, n, c, seed=77, sep=3.0, noise=0.8, frac=0.05, amp=10.0,
                                 dtype=np.float32)
    lam = float(np.sqrt(max(d, n)))
    o = oracle.solve(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=3, max_lloyd=1))
    T = o["info"]["iters"]
    say(f"single-Lloyd-step solve T={T} precision={precision}")
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=3, max_lloyd=1,
                 precision=precision)
    assert g["info"]["iters"] == T
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    assert g["info"]["init_lloyd"] == o["info"]["init_lloyd"]
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F32_TOL
    st, th_prev, rho_t, _ = trajectory(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=3,
                                                             max_lloyd=1), T)
    frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(g["S"]), st["S"],
                         np.finfo(np.float32).eps)
    assert frac > 0.5


def test_solve_f32_video_clip_matches_oracle_and_table2_counts():
    """Synthetic 8-bit clip, lambda = sqrt(max(n, d)), tol 1e-3 (the Sec. 5.1
    setting): the GPU stops at the oracle's iteration (23, as in Table 2)."""
    X, _, _ = synth.video(n=200, h=48, w=64, seed=2, dtype=np.float32)
    d, n = X.shape
    lam = float(np.sqrt(max(d, n)))
    for c in (1, 2):
        o = oracle.solve(X, oracle.make_params(c, lam=lam, tol=1e-3))
        g = rp.solve(dev(X), rank=c, lam=lam, tol=1e-3)
        assert g["info"]["iters"] == o["info"]["iters"]
        assert 23 <= g["info"]["iters"] <= 25
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
        assert rel(host(g["S"]), o["S"], nX) <= F32_TOL


def test_warm_start_labels_match_oracle_from_same_init():
    X, _, _ = synth.config_small(1)
    init = np.random.default_rng(3).integers(0, 25, 500).astype(np.int32)
    g = rp.solve(dev(X), rank=25, lam=0.5, tol=1e-7, precision=rp.F64,
                 init_labels=torch.from_numpy(init))
    o = oracle.solve(X, oracle.make_params(25, lam=0.5, tol=1e-7), init_labels=init)
    assert g["info"]["iters"] == o["info"]["iters"] and g["info"]["init_lloyd"] == 0
    nX = np.linalg.norm(X)
    assert rel(host(g["L"]), o["L"], nX) <= F64_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F64_TOL


# -------------------------------------------------------- single iterations

def _gpu_state(st, dtype):
    return {"L": dev(st["L"], dtype), "S": dev(st["S"], dtype), "Theta": dev(st["Theta"], dtype),
            "labels": torch.from_numpy(st["labels"].copy()).to("cuda"),
            "C": dev(st["C"], dtype), "rho": st["rho"]}


def _support_check(X, L_or, Th_prev, rho, S_gpu, S_or, eps):
    """Support of S identical on entries where |B| is well away from 1/rho."""
    B = X - L_or + Th_prev / rho
    margin = np.abs(np.abs(B) - 1.0 / rho)
    bound = 64 * eps * (np.abs(X) + np.abs(L_or) + np.abs(Th_prev) / rho + 1.0 / rho)
    sep = margin > bound
    assert np.array_equal((S_gpu != 0)[sep], (S_or != 0)[sep])
    return sep.mean()


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("max_lloyd", [1, 100])
def test_iterate_matches_oracle_steps(dtype, max_lloyd):
    d, n, c = 2051, 333, 7
    X, _, _, _ = synth.clustered(d, n, c, seed=99, sep=3.0, noise=1.0, frac=0.1, amp=10.0,
                                 dtype=dtype)
    st = synth.random_state(X, c, seed=5, s_frac=0.2, s_amp=2.0)
    st["rho"] = 0.05
    lam = 0.8
    prec = rp.F64 if dtype == np.float64 else rp.F32
    gs = _gpu_state(st, dtype)
    ost = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype != np.int32 else v)
           for k, v in st.items()}
    p = oracle.make_params(c, lam=lam, max_lloyd=max_lloyd)
    tol = F64_TOL if dtype == np.float64 else F32_TOL
    eps = np.finfo(dtype).eps
    Xo = X.astype(np.float64)
    nX = np.linalg.norm(Xo)
    for t in range(3):
        th_prev = ost["Theta"].copy()
        rho_t = ost["rho"]
        norms, info = rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=max_lloyd, precision=prec)
        ost = oracle.step(p, Xo, ost)
        np.testing.assert_array_equal(gs["labels"].cpu().numpy(), ost["labels"])
        assert info["lloyd_steps"] == ost["lloyd"]
        assert gs["rho"] == pytest.approx(ost["rho"], rel=1e-15)
        for k in ("L", "S"):
            assert rel(host(gs[k]), ost[k], nX) <= tol, (t, k)
        # Theta is checked through what the method uses, Theta / rho
        assert rel(host(gs["Theta"]) / rho_t, ost["Theta"] / rho_t, nX) <= tol
        np.testing.assert_allclose(norms[0], ost["norms"], rtol=1e-3 if dtype == np.float32 else 1e-9,
                                   atol=1e-6 * nX if dtype == np.float32 else 1e-12 * nX)
        frac = _support_check(Xo, ost["L"], th_prev, rho_t, host(gs["S"]), ost["S"], eps)
        assert frac > 0.99


def test_iterate_full_size_sampled_columns():
    """10^4 x 10^4, rank 100, 10 % corruptions in [-100, 100], c = 100, FP32: one
    iteration from an arbitrary state, checked at sampled columns against the
    oracle (group means over all columns, then per-column outputs)."""
    d = n = 10000
    c = 100
    say("full-size iterate: generating")
    X, _, _ = synth.config_large(1, np.float32)
    st = synth.random_state(X, c, seed=8, s_frac=0.1, s_amp=20.0)
    st["rho"] = 0.3
    lam = 0.01
    gs = _gpu_state(st, np.float32)
    say("full-size iterate: gpu")
    rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=1)
    rng = np.random.default_rng(0)
    sel = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)]))
    say("full-size iterate: oracle")
    o = oracle.step_columns(oracle.make_params(c, lam=lam, max_lloyd=1), X, st, sel)
    Xo = X[:, sel].astype(np.float64)
    for k in ("L", "S"):
        got = host(gs[k][:, torch.from_numpy(sel).cuda()])
        assert rel(got, o[k], np.linalg.norm(Xo)) <= F32_TOL, k
    got_t = host(gs["Theta"][:, torch.from_numpy(sel).cuda()])
    assert rel(got_t / 0.3, o["Theta"] / 0.3, np.linalg.norm(Xo)) <= F32_TOL
    # labels: identical where the top-2 squared-distance gap is well separated
    lab = gs["labels"].cpu().numpy()[sel]
    mu = o["mu"]
    dist = ((o["L"][:, :, None] - mu[:, None, :]) ** 2).sum(axis=0)
    srt = np.sort(dist, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    cn = np.sqrt((mu ** 2).sum(axis=0)).max()
    ln = np.sqrt((o["L"] ** 2).sum(axis=0))
    # FP32 partial dot products over 1024-row slices: worst-case rounding bound
    bound = 1024 * np.finfo(np.float32).eps * (cn ** 2 + 2 * cn * ln)
    sep = gap > bound
    assert sep.mean() > 0.5
    np.testing.assert_array_equal(lab[sep], o["labels"][sep])


def test_gaussian_rank100_steps_along_the_oracle_trajectory():
    """2000 x 2000, rank 100 (U, V iid N(0, 1)), 10 % corruptions in [-100, 100],
    c = 100, lambda = 0.01 (the 10^4 x 10^4 workload's construction at a size the
    oracle solves in under a minute).  At t = 1, T/2 and T - 1 of the oracle's own
    trajectory (T its stop at tol 1e-6), one GPU iteration with the full p-step
    (up to 100 Lloyd passes), FP32 and bounded mode, from the oracle's state cast
    to FP32, against one oracle iteration from the same cast state: L, S and
    Theta/rho to the FP32 bar, labels on well-separated columns, S support."""
    d = n = 2000
    c = 100
    lam = 0.01
    X, _, _ = synth.low_rank_plus_sparse(d, n, c, 0.10, 100.0, seed=11, dtype=np.float32)
    Xo = X.astype(np.float64)
    p = oracle.make_params(c, lam=lam, tol=1e-6, seed=1)
    say("rank-100 trajectory: oracle")
    o = oracle.solve(X, p)
    T = o["info"]["iters"]
    stops = sorted({1, T // 2, T - 1})
    labels, C, _ = oracle.kmeans(Xo, c, 1, 100)
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.zeros((d, n), order="F"), "labels": labels, "C": C, "rho": p.rho0}
    nX = np.linalg.norm(Xo)
    eps = np.finfo(np.float32).eps
    for t in range(1, stops[-1] + 1):
        st = oracle.step(p, Xo, st)
        if t not in stops:
            continue
        # the state both sides start from: the oracle's iterate t, cast to FP32
        cast = {k: (v.astype(np.float32).astype(np.float64) if k in ("L", "S", "Theta", "C") else v)
                for k, v in st.items()}
        ref = oracle.step(p, Xo, cast)
        for prec in (rp.F32, rp.BF16GEMM_F32):
            gs = _gpu_state(cast, np.float32)
            _, info = rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=100, precision=prec)
            lab = gs["labels"].cpu().numpy()
            # labels: identical where the top-2 squared-distance gap of the oracle's
            # last assignment (its final L against its final centroids) is clear of
            # the FP32 rounding of the distances
            dist = ((ref["L"][:, :, None] - ref["C"][:, None, :]) ** 2).sum(axis=0)
            srt = np.sort(dist, axis=1)
            cn = np.sqrt((ref["C"] ** 2).sum(axis=0)).max()
            ln = np.sqrt((ref["L"] ** 2).sum(axis=0))
            sep = (srt[:, 1] - srt[:, 0]) > 2 * d * eps * (cn ** 2 + 2 * cn * ln + ln ** 2)
            flips = int((lab != ref["labels"]).sum())
            say(f"t={t}/{T} precision={prec}: Lloyd {info['lloyd_steps']}/{ref['lloyd']}, "
                f"label flips {flips}, separated {sep.mean():.3f}")
            np.testing.assert_array_equal(lab[sep], ref["labels"][sep])
            if flips == 0:
                assert info["lloyd_steps"] == ref["lloyd"]
            # L, S and Theta come before the p-step in the iteration (they use the
            # groups the state carries), so they are compared whatever the labels
            for k in ("L", "S"):
                assert rel(host(gs[k]), ref[k], nX) <= F32_TOL, (t, prec, k)
            # Theta / rho is a term of D = X - S + Theta / rho, so its error is measured
            # on the scale of X (for unsaturated entries Theta = rho B, and B = X - L +
            # Theta / rho carries the FP32 rounding of X - L)
            dth = np.linalg.norm(host(gs["Theta"]) / cast["rho"] - ref["Theta"] / cast["rho"]) / nX
            assert dth <= F32_TOL, (t, prec, dth)
            frac = support_check(Xo, ref["L"], cast["Theta"], cast["rho"], host(gs["S"]),
                                 ref["S"], eps)
            assert frac > 0.5


# ------------------------------------------------------------- full size

@pytest.mark.parametrize("precision", [rp.F32, rp.BF16GEMM_F32])
@pytest.mark.parametrize("rank", [100, 5])
def test_solve_full_size_properties(rank, precision):
    """10^4 x 10^4 FP32-data solve, true rank given (c = 100) and withheld (c = 5),
    FP32 and bounded distances: converges, X = L + S to the tolerance, finite
    outputs, labels in range."""
    say(f"full-size solve c={rank} precision={precision}: generating")
    X, _, _ = synth.config_large(1, np.float32)
    Xd = dev(X)
    say(f"full-size solve c={rank}: gpu")
    g = rp.solve(Xd, rank=rank, lam=0.01, tol=1e-6, seed=0, precision=precision)
    say(f"info {g['info']}")
    assert g["status"] == rp.OK
    L, S = g["L"].double(), g["S"].double()
    r = torch.linalg.norm(Xd.double() - L - S) / torch.linalg.norm(Xd.double())
    assert float(r) <= 1e-6 * 1.5
    assert torch.isfinite(L).all() and torch.isfinite(S).all()
    lab = g["labels"]
    assert int(lab.min()) >= 0 and int(lab.max()) < rank


# ------------------------------------------------------------- edge cases

def test_zero_input_and_error_paths():
    Z = torch.zeros((40, 30), dtype=torch.float32, device="cuda").T.contiguous().T
    g = rp.solve(Z, rank=3, lam=1.0)
    assert g["status"] == rp.OK and g["info"]["iters"] == 0
    assert not g["L"].any() and not g["S"].any() and not g["labels"].any()
    X = dev(np.random.default_rng(0).normal(size=(40, 30)), np.float32)
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=31, lam=1.0)
    assert e.value.status == rp.ERR_INVALID
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=3, lam=-1.0)
    assert e.value.status == rp.ERR_INVALID
    Xn = X.clone()
    Xn[3, 4] = float("nan")
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(Xn, rank=3, lam=1.0)
    assert e.value.status == rp.ERR_NONFINITE
    Xi = X.clone()
    Xi[0, 0] = float("inf")
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(Xi, rank=3, lam=1.0)
    assert e.value.status == rp.ERR_NONFINITE
    g = rp.solve(X, rank=3, lam=1.0, max_iter=1)
    assert g["status"] == rp.NOT_CONVERGED and g["info"]["iters"] == 1


def test_degenerate_cases_match_closed_forms():
    """c = n or lambda = 0: L = X, S = 0, stop at t = 2; d = n = 1."""
    X = np.random.default_rng(1).normal(size=(7, 40))
    for c, lam in [(40, 2.0), (3, 0.0)]:
        g = rp.solve(dev(X), rank=c, lam=lam, tol=1e-12, precision=rp.F64)
        assert g["info"]["iters"] == 2
        np.testing.assert_allclose(host(g["L"]), X, atol=1e-15)
        assert not g["S"].any()
    one = np.array([[3.5]])
    g = rp.solve(dev(one), rank=1, lam=1.0, tol=1e-12, precision=rp.F64)
    assert g["info"]["iters"] == 2 and float(g["L"][0, 0]) == 3.5


def test_padded_leading_dimension_and_determinism():
    d, n, c = 1001, 257, 4
    X, _, _, _ = synth.clustered(d, n, c, seed=4, sep=4.0, noise=0.5, dtype=np.float32)
    Xd = dev(X)
    pad = torch.zeros((n, d + 5), dtype=torch.float32, device="cuda")
    pad[:, :d] = Xd.T
    Xp = pad.T[:d]                       # stride (1, d + 5)
    assert Xp.stride() == (1, d + 5)
    a = rp.solve(Xd, rank=c, lam=0.7, tol=1e-6, seed=2)
    b = rp.solve(Xd, rank=c, lam=0.7, tol=1e-6, seed=2)
    assert torch.equal(a["L"], b["L"]) and torch.equal(a["S"], b["S"])
    assert torch.equal(a["labels"], b["labels"])
    p = rp.solve(Xp, rank=c, lam=0.7, tol=1e-6, seed=2)
    o = oracle.solve(X, oracle.make_params(c, lam=0.7, tol=1e-6, seed=2))
    nX = np.linalg.norm(X.astype(np.float64))
    assert p["info"]["iters"] == o["info"]["iters"]
    assert rel(host(p["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(p["S"]), o["S"], nX) <= F32_TOL


@pytest.mark.parametrize("dtype,precision", [(np.float64, rp.F64), (np.float32, rp.F32)])
def test_stopped_solve_returns_the_last_sparse_part_in_padded_outputs(dtype, precision):
    """A solve stopped by max_iter (not by the tolerance) returns the L and S of its
    last iteration (the whole solve keeps B = X - L + Theta/rho in S and turns it into
    soft(B, 1/rho) at the end); L and S in buffers with a padded leading dimension
    (d + 3): the padding rows keep their contents."""
    d, n, c = 203, 150, 4
    X, _, _, _ = synth.clustered(d, n, c, seed=9, sep=4.0, noise=0.5, frac=0.05, amp=8.0, dtype=dtype)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    bufL = torch.full((n, d + 3), 7.25, dtype=tdt, device="cuda")
    bufS = torch.full((n, d + 3), -3.5, dtype=tdt, device="cuda")
    L, S = bufL.T[:d], bufS.T[:d]
    assert L.stride() == (1, d + 3)
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    for T in (1, 4):
        g = rp.solve(dev(X), rank=c, lam=0.6, tol=1e-12, max_iter=T, seed=5, precision=precision,
                     out=(L, S, labels), history=True)
        o = oracle.solve(X, oracle.make_params(c, lam=0.6, tol=1e-12, max_iter=T, seed=5),
                         history=True)
        assert g["status"] == rp.NOT_CONVERGED and g["info"]["iters"] == T
        assert o["info"]["iters"] == T
        # the per-iteration criterion terms (primal, dL, dS relative to ||X||)
        assert g["history"].shape == o["history"].shape == (T, 3)
        np.testing.assert_allclose(g["history"], o["history"],
                                   rtol=1e-9 if dtype == np.float64 else 1e-4, atol=1e-12)
        nX = np.linalg.norm(X.astype(np.float64))
        tol = F64_TOL if dtype == np.float64 else F32_TOL
        assert rel(host(L), o["L"], nX) <= tol
        assert rel(host(S), o["S"], nX) <= tol
        np.testing.assert_array_equal(labels.cpu().numpy(), o["labels"])
        assert torch.all(bufL[:, d:] == 7.25) and torch.all(bufS[:, d:] == -3.5)


# ------------------------------------------------------ bf16 distance mode

@pytest.mark.parametrize("shape,lam", [((1037, 777, 5), None), ((2051, 300, 40), 0.3)])
def test_bf16_solve_matches_oracle(shape, lam):
    """Split-bf16 MFMA distances with exact refinement: same labels and the FP32
    bar against the FP64 oracle (iteration-locked), on grouped data."""
    d, n, c = shape
    X, _, _, _ = synth.clustered(d, n, c, seed=d * 3 + n, sep=4.0, noise=0.5, frac=0.05, amp=10.0,
                                 dtype=np.float32)
    lam = float(np.sqrt(max(d, n))) if lam is None else lam
    o = oracle.solve(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=1))
    T = o["info"]["iters"]
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=1, precision=rp.BF16GEMM_F32)
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    assert g["info"]["init_lloyd"] == o["info"]["init_lloyd"]
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F32_TOL
    st, th_prev, rho_t, _ = trajectory(X, oracle.make_params(c, lam=lam, tol=1e-6, seed=1), T)
    frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(g["S"]), st["S"],
                         np.finfo(np.float32).eps)
    assert frac > 0.5


def test_bf16_kmeans_matches_oracle():
    X, _, _, _ = synth.clustered(777, 900, 12, seed=5, sep=3.0, noise=0.7, dtype=np.float32)
    lab, C, info = rp.kmeans(dev(X), 12, seed=4, precision=rp.BF16GEMM_F32)
    ol, oC, osteps = oracle.kmeans(X, 12, 4)
    np.testing.assert_array_equal(lab.cpu().numpy(), ol)
    assert info["init_lloyd"] == osteps


@pytest.mark.parametrize("d,n,c,pad", [
    (1024, 900, 40, 0),     # direct tile, three group blocks (two workgroups per CU)
    (512, 1300, 70, 0),     # direct tile, five group blocks
    (1028, 700, 70, 0),     # direct tile, two stages in flight, ragged last stage
    (2340, 400, 100, 4),    # direct tile, seven group blocks, ragged last stage, padded ld
    (1020, 600, 20, 8),     # at most 32 groups: FP32 MFMA tile with bounds, padded ld
    (2048, 300, 130, 4),    # two group tiles (c > 128), padded ld
    (1000, 777, 5, 0),      # at most 16 groups: FP64 tile, 6 columns per lane group
    (1022, 513, 16, 6),     # FP64 tile, scalar loads (d % 4 != 0), padded ld
    (260, 1500, 9, 4),      # FP64 tile, 16-byte loads with ld > d
    (3000, 100, 1, 0),      # one group
    (7, 40, 3, 1),          # FP64 tile, fewer rows than one step, scalar loads
    (64, 9, 4, 0),          # FP64 tile, fewer columns than one lane group's share
])
def test_bf16_kmeans_tile_variants_match_oracle(d, n, c, pad):
    """Every bounded-distance tile variant (chosen by c and the column layout) gives
    the oracle's labels and Lloyd count on grouped data, also with ld > d."""
    X, _, _, _ = synth.clustered(d, n, c, seed=d + c, sep=3.0, noise=0.7, dtype=np.float32)
    buf = rp.empty_colmajor(d + pad, n, torch.float32, torch.device("cuda:0"))
    buf.zero_()
    Xv = buf[:d]
    Xv.copy_(torch.from_numpy(X))
    say(f"tile variant d={d} n={n} c={c} ld={Xv.stride(1)}")
    lab, C, info = rp.kmeans(Xv, c, seed=7, precision=rp.BF16GEMM_F32)
    ol, oC, osteps = oracle.kmeans(X, c, 7)
    np.testing.assert_array_equal(lab.cpu().numpy(), ol)
    assert info["init_lloyd"] == osteps


@pytest.mark.parametrize("d,n,c", [(1500, 1234, 5), (1023, 777, 16), (4096, 300, 1), (644, 2100, 9)])
def test_bounded_small_c_iterations_unstructured(d, n, c):
    """At most 16 groups the bounded mode sums its dot products in FP64: on data with
    no group structure, three iterations with up to 100 Lloyd passes each give the
    oracle's labels and Lloyd counts, and L, S to the FP32 bar."""
    rng = np.random.default_rng(d + c)
    X = np.asfortranarray(rng.standard_normal((d, n)).astype(np.float32))
    st = synth.random_state(X, c, seed=c, s_frac=0.1, s_amp=1.0)
    st["rho"] = 0.05
    lam = 0.5
    gs = _gpu_state(st, np.float32)
    ost = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype != np.int32 else v)
           for k, v in st.items()}
    p = oracle.make_params(c, lam=lam, max_lloyd=100)
    Xo = X.astype(np.float64)
    nX = np.linalg.norm(Xo)
    say(f"bounded small c d={d} n={n} c={c}")
    for t in range(3):
        _, info = rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=100, precision=rp.BF16GEMM_F32)
        ost = oracle.step(p, Xo, ost)
        np.testing.assert_array_equal(gs["labels"].cpu().numpy(), ost["labels"])
        assert info["lloyd_steps"] == ost["lloyd"]
        for k in ("L", "S"):
            assert rel(host(gs[k]), ost[k], nX) <= F32_TOL, (t, k)


@pytest.mark.parametrize("precision", [rp.F32, rp.BF16GEMM_F32])
def test_exact_ties_go_to_lowest_group(precision):
    """Two identical centroids (empty groups carried in the state) tie exactly for
    the columns nearest to them; the lower group must win, as in the oracle.
    lambda = 0 makes L = X, so the tie is exact in any precision."""
    d, n, c = 256, 200, 4
    rng = np.random.default_rng(11)
    e = np.zeros(d)
    e[0] = 10.0
    X = np.empty((d, n))
    X[:, :90] = e[:, None] + rng.normal(0, 0.1, (d, 90))
    X[:, 90:180] = -e[:, None] + rng.normal(0, 0.1, (d, 90))
    X[:, 180:] = rng.normal(0, 0.01, (d, 20))
    X = np.asfortranarray(X.astype(np.float32))
    st = synth.random_state(X, c, seed=3, s_frac=0.0)
    lab = np.zeros(n, dtype=np.int32)
    lab[90:180] = 3
    lab[190:] = 3                              # groups 1 and 2 are empty
    st["labels"] = lab
    st["C"][:, 1] = 0.0                        # identical centroids at the origin
    st["C"][:, 2] = 0.0
    st["Theta"][:] = 0.0
    st["rho"] = 1e-2
    gs = _gpu_state(st, np.float32)
    rp.iterate(dev(X), gs, iters=1, lam=0.0, max_lloyd=1, precision=precision)
    ost = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype != np.int32 else v)
           for k, v in st.items()}
    o = oracle.step(oracle.make_params(c, lam=0.0, max_lloyd=1), X.astype(np.float64), ost)
    assert np.all(o["labels"][180:] == 1)
    np.testing.assert_array_equal(gs["labels"].cpu().numpy(), o["labels"])


@pytest.mark.parametrize("c", [100, 5])
def test_bf16_iterate_full_size_sampled_columns(c):
    """Full-size one-iteration check of the bounded mode at 10^4 x 10^4: c = 100 on
    the split-bf16 direct tile, c = 5 on the FP64 tile."""
    d = n = 10000
    X, _, _ = synth.config_large(1, np.float32)
    st = synth.random_state(X, c, seed=8, s_frac=0.1, s_amp=20.0)
    st["rho"] = 0.3
    lam = 0.01
    gs = _gpu_state(st, np.float32)
    rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=1, precision=rp.BF16GEMM_F32)
    rng = np.random.default_rng(0)
    sel = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)]))
    o = oracle.step_columns(oracle.make_params(c, lam=lam, max_lloyd=1), X, st, sel)
    Xo = X[:, sel].astype(np.float64)
    idx = torch.from_numpy(sel).cuda()
    for k in ("L", "S"):
        assert rel(host(gs[k][:, idx]), o[k], np.linalg.norm(Xo)) <= F32_TOL, k
    lab = gs["labels"].cpu().numpy()[sel]
    mu = o["mu"]
    dist = ((o["L"][:, :, None] - mu[:, None, :]) ** 2).sum(axis=0)
    srt = np.sort(dist, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    cn = np.sqrt((mu ** 2).sum(axis=0)).max()
    ln = np.sqrt((o["L"] ** 2).sum(axis=0))
    # refined decisions are exact up to double rounding of FP32 inputs
    bound = 64 * np.finfo(np.float32).eps * (cn ** 2 + 2 * cn * ln)
    sep = gap > bound
    assert sep.mean() > 0.9
    np.testing.assert_array_equal(lab[sep], o["labels"][sep])


def test_bounded_iterate_clip_shape_sampled_columns():
    """The bounded mode's FP64 tile at the clip shape (76800 x 2000, c = 5: many row
    slices per column): one iteration from a random state, sampled columns against
    the oracle, labels equal wherever the two nearest distances are separated."""
    X, _, _ = synth.video(n=2000, h=240, w=320, seed=2, dtype=np.float32)
    d, n = X.shape
    c = 5
    st = synth.random_state(X, c, seed=9, s_frac=0.1, s_amp=20.0)
    st["rho"] = 0.05
    lam = float(np.sqrt(max(d, n)))
    say(f"bounded iterate clip shape d={d} n={n}")
    gs = _gpu_state(st, np.float32)
    rp.iterate(dev(X), gs, iters=1, lam=lam, max_lloyd=1, precision=rp.BF16GEMM_F32)
    rng = np.random.default_rng(1)
    sel = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 62, replace=False)]))
    o = oracle.step_columns(oracle.make_params(c, lam=lam, max_lloyd=1), X, st, sel)
    Xo = X[:, sel].astype(np.float64)
    idx = torch.from_numpy(sel).cuda()
    for k in ("L", "S"):
        assert rel(host(gs[k][:, idx]), o[k], np.linalg.norm(Xo)) <= F32_TOL, k
    lab = gs["labels"].cpu().numpy()[sel]
    mu = o["mu"]
    dist = ((o["L"][:, :, None] - mu[:, None, :]) ** 2).sum(axis=0)
    srt = np.sort(dist, axis=1)
    gap = srt[:, 1] - srt[:, 0]
    cn = np.sqrt((mu ** 2).sum(axis=0)).max()
    ln = np.sqrt((o["L"] ** 2).sum(axis=0))
    bound = 64 * np.finfo(np.float32).eps * (cn ** 2 + 2 * cn * ln)
    sep = gap > bound
    assert sep.mean() > 0.9
    np.testing.assert_array_equal(lab[sep], o["labels"][sep])


# ------------------------------------------------------------ batched solver

def _batch_mix(seed=7):
    """Grouped instances of uneven, ragged sizes (labels well separated)."""
    rng = np.random.default_rng(seed)
    shapes = [(37, 50, 3), (200, 333, 5), (513, 129, 7), (1030, 241, 4), (64, 700, 9),
              (255, 255, 6), (2049, 97, 3), (321, 1025, 12), (8, 40, 2), (1500, 600, 20)]
    Xs = []
    for i, (d, n, c) in enumerate(shapes):
        X, _, _, _ = synth.clustered(d, n, c, seed=int(rng.integers(1 << 30)), sep=4.0, noise=0.5,
                                     frac=0.05, amp=8.0, dtype=np.float32, min_size=2)
        Xs.append(X)
    return shapes, Xs


_BATCH_ORACLE = {}


def _batch_mix_oracle():
    """The ragged mix and, per instance, the oracle's trajectory to its stop at
    tol 1e-6 (computed once per test session)."""
    if not _BATCH_ORACLE:
        shapes, Xs = _batch_mix()
        lams = [0.5 if i % 3 == 0 else float(np.sqrt(max(s[0], s[1]))) for i, s in enumerate(shapes)]
        runs = []
        for i, (X, (d, n, c), lam) in enumerate(zip(Xs, shapes, lams)):
            p = oracle.make_params(c, lam=lam, tol=1e-6, seed=i)
            o = oracle.solve(X, p)
            runs.append((o, trajectory(X, p, o["info"]["iters"])))
        _BATCH_ORACLE.update(shapes=shapes, Xs=Xs, lams=lams, runs=runs)
    return _BATCH_ORACLE


# (jc, slice_rows, blocks_per_cu): the default, the tuner's corners and the shape
# the tuner picks for the 256-instance mix
BATCH_TILES = [(8, 1024, 2), (4, 512, 1), (32, 2048, 2), (4, 2048, 2), (32, 512, 1),
               (16, 1024, 2)]


@pytest.mark.parametrize("tile", BATCH_TILES)
def test_batched_matches_oracle_per_instance(tile):
    """Every instance of a ragged batch, solved in one persistent launch with the
    given tile shape, meets the FP32 bar against the oracle run on that instance
    alone (iteration-locked): labels, initial Lloyd count, L, S and the support
    of S on well-separated entries."""
    mix = _batch_mix_oracle()
    shapes, Xs, lams, runs = mix["shapes"], mix["Xs"], mix["lams"], mix["runs"]
    rp.set_batched_tile(*tile)
    assert rp.get_batched_tile() == tile
    plist, keep = rp.batch_params([s[2] for s in shapes], lams, tol=0.0,
                                  max_iter=0, seeds=list(range(len(shapes))))
    for p, (o, _) in zip(plist, runs):
        p.max_iter = o["info"]["iters"]
    Xd = [dev(X) for X in Xs]
    say(f"batched tile {tile}")
    try:
        outs, infos, status = rp.solve_batched(Xd, plist)
    finally:
        rp.set_batched_tile(8, 1024, 2)
    for i, (X, (o, (st, th_prev, rho_t, _))) in enumerate(zip(Xs, runs)):
        say(f"batched instance {i} {shapes[i]} iters {infos[i]['iters']} / {o['info']['iters']}")
        assert infos[i]["iters"] == o["info"]["iters"]
        assert infos[i]["init_lloyd"] == o["info"]["init_lloyd"]
        np.testing.assert_array_equal(outs[i][2].cpu().numpy(), o["labels"])
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(outs[i][0]), o["L"], nX) <= F32_TOL, i
        assert rel(host(outs[i][1]), o["S"], nX) <= F32_TOL, i
        frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(outs[i][1]),
                             st["S"], np.finfo(np.float32).eps)
        assert frac > 0.5, (i, frac)


# the eight smallest instances (by d n) of the 256-instance size mix, seeds 3 000 000 + i
CONFIG3_SMALLEST = [134, 192, 99, 123, 246, 199, 136, 142]


def test_batched_size_mix_instances_match_oracle():
    """Instances of the 256-instance size mix itself (Gaussian U V^T of rank 5-50,
    1-20 % corruptions in [-50, 50], c = rank, lambda = 1/sqrt(max(d, n))), solved
    together in one persistent launch, each iteration-locked to the oracle's stop
    at tol 1e-6 with the full p-step (up to 100 Lloyd passes): labels, initial
    Lloyd counts, L and S to the FP32 bar and the support of S on well-separated
    entries.  The data have no group structure, so K-means decisions can be close;
    every label that differs from the oracle's is printed."""
    Xs, ranks, lams, runs = [], [], [], []
    for k, i in enumerate(CONFIG3_SMALLEST):
        X, r, meta = synth.batch_instance(i)
        lam = 1.0 / np.sqrt(max(meta["d"], meta["n"]))
        p = oracle.make_params(r, lam=lam, tol=1e-6, seed=k)
        o = oracle.solve(X, p)
        assert o["status"] == 0
        Xs.append(X)
        ranks.append(r)
        lams.append(lam)
        runs.append((o, trajectory(X, p, o["info"]["iters"])))
    plist, _ = rp.batch_params(ranks, lams, tol=0.0, max_iter=0, seeds=list(range(len(Xs))))
    for p, (o, _) in zip(plist, runs):
        p.max_iter = o["info"]["iters"]
    outs, infos, _ = rp.solve_batched([dev(X) for X in Xs], plist)
    for k, (X, (o, (st, th_prev, rho_t, _))) in enumerate(zip(Xs, runs)):
        lab = outs[k][2].cpu().numpy()
        flips = np.flatnonzero(lab != o["labels"])
        say(f"size-mix instance {CONFIG3_SMALLEST[k]} {X.shape} c={ranks[k]}: iters "
            f"{infos[k]['iters']}/{o['info']['iters']}, init Lloyd {infos[k]['init_lloyd']}/"
            f"{o['info']['init_lloyd']}, label flips {flips.size} {flips[:10].tolist()}")
        assert infos[k]["iters"] == o["info"]["iters"]
        assert infos[k]["init_lloyd"] == o["info"]["init_lloyd"]
        assert flips.size == 0
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(outs[k][0]), o["L"], nX) <= F32_TOL, k
        assert rel(host(outs[k][1]), o["S"], nX) <= F32_TOL, k
        frac = support_check(X.astype(np.float64), st["L"], th_prev, rho_t, host(outs[k][1]),
                             st["S"], np.finfo(np.float32).eps)
        assert frac > 0.5, (k, frac)


def test_batched_tile_setter_and_tuned_cache(tmp_path):
    """Tile shapes outside the tuner's candidates are refused; the tuner's choice
    is written to the cache file, read back by a later call (same key), and a
    line with a shape outside the candidates is ignored (the tuner runs again)."""
    with pytest.raises(rp.RespcaError):
        rp.set_batched_tile(0, 1024, 2)
    with pytest.raises(rp.RespcaError):
        rp.set_batched_tile(8, 1000, 2)
    assert rp.get_batched_tile() == (8, 1024, 2)
    shapes, Xs = _batch_mix()
    lams = [1.0] * len(shapes)
    plist, _ = rp.batch_params([s[2] for s in shapes], lams, tol=1e-4, max_iter=5)
    Xd = [dev(X) for X in Xs]
    cache = tmp_path / "tune.txt"
    ms = rp.autotune_batched(Xd, plist, cache_path=str(cache))
    tuned = rp.get_batched_tile()
    lines = cache.read_text().split()
    assert len(lines) == 5 and tuple(int(v) for v in lines[1:4]) == tuned and ms > 0
    key = lines[0]
    assert "_k3_" in key
    rp.set_batched_tile(*(BATCH_TILES[1] if tuned != BATCH_TILES[1] else BATCH_TILES[2]))
    assert rp.autotune_batched(Xd, plist, cache_path=str(cache)) == pytest.approx(float(lines[4]))
    assert rp.get_batched_tile() == tuned
    # a corrupt line for the same key is skipped: the tuner searches and appends again
    cache.write_text(f"{key} 0 1024 2 0.001\n")
    rp.autotune_batched(Xd, plist, cache_path=str(cache))
    rows = cache.read_text().strip().split("\n")
    assert len(rows) == 2 and rows[1].split()[0] == key
    rp.set_batched_tile(8, 1024, 2)


def test_batched_special_instances_and_replay():
    """Zero input, warm start from labels, lambda = 0 and the same call replayed
    from the captured graph (bitwise identical)."""
    rng = np.random.default_rng(3)
    X0 = np.zeros((30, 20), np.float32, order="F")
    X1, _, _, _ = synth.clustered(100, 80, 4, seed=5, sep=4.0, dtype=np.float32)
    X2 = np.asfortranarray(rng.normal(size=(17, 23)).astype(np.float32))
    init = torch.from_numpy(rng.integers(0, 4, 80).astype(np.int32)).cuda()
    Xd = [dev(X0), dev(X1), dev(X2)]
    plist, keep = rp.batch_params([2, 4, 3], [1.0, 0.7, 0.0], tol=1e-6,
                                  init_labels=[None, init, None])
    outs, infos, status = rp.solve_batched(Xd, plist)
    assert infos[0]["status"] == 0 and infos[0]["iters"] == 0
    assert not outs[0][0].any() and not outs[0][1].any()
    o = oracle.solve(X1, oracle.make_params(4, lam=0.7, tol=1e-6), init_labels=init.cpu().numpy())
    assert infos[1]["iters"] == o["info"]["iters"] and infos[1]["init_lloyd"] == 0
    nX = np.linalg.norm(X1.astype(np.float64))
    assert rel(host(outs[1][0]), o["L"], nX) <= F32_TOL
    assert infos[2]["iters"] == 2
    np.testing.assert_allclose(host(outs[2][0]), X2.astype(np.float64), atol=0)
    snap = [(a.clone(), b.clone(), c.clone()) for a, b, c in outs]
    outs2, infos2, _ = rp.solve_batched(Xd, plist, outs=outs)
    for (a, b, c), (a2, b2, c2) in zip(snap, outs2):
        assert torch.equal(a, a2) and torch.equal(b, b2) and torch.equal(c, c2)
    assert infos2 == infos


def test_batched_size_mix_converges():
    """The 256-instance size mix (d, n log-uniform in [200, 4000], rank 5-50,
    1-20 % corruptions in [-50, 50], c = rank, lambda = 1/sqrt(max(d, n)),
    tol 1e-6) in one launch: every instance converges and X = L + S to tol."""
    Xs, ranks, lams = [], [], []
    for i in range(256):
        X, r, meta = synth.batch_instance(i)
        Xs.append(dev(X))
        ranks.append(r)
        lams.append(1.0 / np.sqrt(max(meta["d"], meta["n"])))
    say("batched size mix: solving")
    plist, _ = rp.batch_params(ranks, lams, tol=1e-6)
    outs, infos, status = rp.solve_batched(Xs, plist)
    assert status == rp.OK
    for i, (X, (L, S, lab)) in enumerate(zip(Xs, outs)):
        assert infos[i]["status"] == 0
        r = torch.linalg.norm(X.double() - L.double() - S.double()) / torch.linalg.norm(X.double())
        assert float(r) <= 1.5e-6, (i, float(r))
        assert int(lab.min()) >= 0 and int(lab.max()) < ranks[i]


# ------------------------------------------------------- warm-start kernels

def test_sketch_and_features_match_oracle():
    from oracle import mlp as omlp
    rng = np.random.default_rng(31)
    d, n, c = 1037, 311, 7
    X = np.asfortranarray(rng.normal(0, 3, (d, n)).astype(np.float32))
    Y = rp.sketch(dev(X), seed=77)                       # (n, 65)
    Yo = oracle.sketch(X, 77)                            # (65, n)
    Yg = Y.cpu().numpy().astype(np.float64).T
    assert rel(Yg, Yo, 1.0) <= 2e-6
    F = rp.features(Y, d, c).cpu().numpy().astype(np.float64)
    Fo = omlp.features(Yo, d, c)
    assert np.abs(F - Fo).max() <= 1e-4


@pytest.mark.parametrize("hidden,batch", [(32, 300), (256, 1000)])
def test_mlp_forward_backward_adam_match_oracle(hidden, batch):
    """The hand-written network kernels against the FP64 reference: outputs,
    loss and its gradient, parameter gradients, one Adam step."""
    from oracle import mlp as omlp
    dims = [68, hidden, hidden, hidden, 65]
    rng = np.random.default_rng(hidden + batch)
    p = (omlp.init_params(dims, 5) + 0.01 * rng.normal(size=omlp.layer_slices(dims)[1])).astype(np.float32)
    x = rng.normal(size=(batch, 68)).astype(np.float32)
    t = rng.normal(size=(batch, 65)).astype(np.float32)
    P = torch.from_numpy(p).cuda()
    Xg = torch.from_numpy(x).cuda()
    Tg = torch.from_numpy(t).cuda()
    out, acts = rp.mlp_forward(P, hidden, Xg)
    yo, acts_o = omlp.forward(p.astype(np.float64), dims, x.astype(np.float64))
    assert rel(out.cpu().numpy(), yo, 1.0) <= 2e-5
    loss, dy = rp.mlp_loss(out, Tg, 4.0)
    lo, dyo = omlp.loss_grad(out.cpu().numpy().astype(np.float64), t, 4.0)
    assert loss == pytest.approx(lo, rel=1e-6)
    np.testing.assert_allclose(dy.cpu().numpy(), dyo, rtol=1e-5, atol=1e-9)
    g = rp.mlp_backward(P, hidden, Xg, acts, dy)
    go = omlp.backward(p.astype(np.float64), dims, acts_o, dyo)
    assert rel(g.cpu().numpy(), go, 1.0) <= 1e-4
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    P2 = P.clone()
    rp.mlp_adam(P2, g, m, v, 1e-3, 1)
    rp.mlp_adam(P2, g, m, v, 1e-3, 2)
    po, mo, vo = omlp.adam(p.astype(np.float64), g.cpu().numpy().astype(np.float64), 0.0, 0.0,
                           1e-3, 0.9, 0.999, 1e-8, 1)
    po, mo, vo = omlp.adam(po, g.cpu().numpy().astype(np.float64), mo, vo, 1e-3, 0.9, 0.999, 1e-8, 2)
    np.testing.assert_allclose(P2.cpu().numpy(), po, rtol=0, atol=2e-6)


# --------------------------------------------------- embedding initialisation

def _embedding_cases():
    """(X, embedding view, c, lam) with embedding rows 13 (ld 16), 64 (> d) and 8."""
    cases = []
    for (d, n, c, er, ld, seed) in [(300, 200, 5, 13, 16, 41), (10, 150, 4, 64, 64, 42),
                                    (1030, 241, 4, 8, 9, 43)]:
        X, _, _, _ = synth.clustered(d, n, c, seed=seed, sep=4.0, noise=0.5, frac=0.05, amp=8.0,
                                     dtype=np.float32, min_size=2)
        E, _, _, _ = synth.clustered(er, n, c, seed=seed + 100, sep=6.0, noise=0.3, frac=0.0,
                                     amp=1.0, dtype=np.float32, min_size=2)
        buf = np.zeros((ld, n), np.float32, order="F")
        buf[:er] = E
        Ed = dev(buf)[:er]
        cases.append((X, E, Ed, c, 0.5 if seed % 2 else float(np.sqrt(max(d, n)))))
    return cases


def _refine_on_x(X, lab, c, max_lloyd=100):
    """Groups of an embedding refined on X: Lloyd from the means of X over them."""
    C0, _ = oracle.group_means(X, lab, c)
    lab2, _, steps = oracle.lloyd(X, C0, lab, max_lloyd)
    return lab2, steps


def _oracle_from_embedding(X, E, c, lam, seed, refine=1, **kw):
    """The oracle's chain for an embedding start: K-means of the embedding's columns
    (then Lloyd on X when refine == 1), or with refine == 2 k-means++ seeds placed on
    the embedding whose columns of X start the nearest-seed assignment and Lloyd on X."""
    if refine == 2:
        seeds = oracle.kmeanspp(E, c, seed)
        X64 = np.asarray(X, np.float64, order="F")
        C = np.asfortranarray(X64[:, seeds])
        lab = oracle.assign(X64, C)
        C, _ = oracle.group_means(X64, lab, c, mean_init=C)
        lab, _, steps = oracle.lloyd(X64, C, lab, 100)
        o = oracle.solve(X, oracle.make_params(c, lam=lam, seed=seed, **kw), init_labels=lab)
        return o, steps
    lab, _, steps = oracle.kmeans(E, c, seed, 100)
    ref = 0
    if refine:
        lab, ref = _refine_on_x(X, lab, c)
    o = oracle.solve(X, oracle.make_params(c, lam=lam, seed=seed, **kw), init_labels=lab)
    return o, steps + ref


@pytest.mark.parametrize("refine", [1, 0, 2])
def test_init_embedding_single_solve_matches_oracle(refine):
    """Groups from K-means of an embedding's columns, refined by Lloyd on X (or not:
    init_embedding_refine = 0), or K-means of X from seeds placed on the embedding
    (2), then the iterations: identical to the oracle's chain from the same embedding."""
    for i, (X, E, Ed, c, lam) in enumerate(_embedding_cases()):
        o, steps = _oracle_from_embedding(X, E, c, lam, seed=i + 3, refine=refine, tol=1e-6)
        g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=o["info"]["iters"], seed=i + 3,
                     precision=rp.F32, init_embedding=Ed, embedding_refine=refine)
        say(f"embedding case {i} {X.shape} iters {g['info']['iters']} init_lloyd "
            f"{g['info']['init_lloyd']} / {steps}")
        assert g["info"]["init_lloyd"] == steps
        np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
        assert rel(host(g["S"]), o["S"], nX) <= F32_TOL
    with pytest.raises(rp.RespcaError):
        rp.solve(dev(X, np.float64), rank=c, precision=rp.F64, init_embedding=Ed)


@pytest.mark.parametrize("refine", [1, 0, 2])
def test_init_embedding_batched_matches_oracle(refine):
    """Embedding, label and cold instances side by side in one persistent launch
    (embedding groups refined by Lloyd on X, or not, or seeds placed on the
    embedding for the K-means of X)."""
    cases = _embedding_cases()
    shapes, Xs = _batch_mix()
    X_lab, X_cold = Xs[1], Xs[2]
    lab0 = np.random.default_rng(5).integers(0, shapes[1][2], X_lab.shape[1]).astype(np.int32)
    Xall = [cs[0] for cs in cases] + [X_lab, X_cold]
    ranks = [cs[3] for cs in cases] + [shapes[1][2], shapes[2][2]]
    lams = [cs[4] for cs in cases] + [0.7, 0.4]
    seeds = [11, 12, 13, 14, 15]
    T = []
    for i, (X, r, lam, sd) in enumerate(zip(Xall, ranks, lams, seeds)):
        if i < len(cases):
            o, steps = _oracle_from_embedding(X, cases[i][1], r, lam, sd, refine=refine,
                                              tol=1e-6)
            o["emb_steps"] = steps
        elif i == len(cases):
            o = oracle.solve(X, oracle.make_params(r, lam=lam, tol=1e-6, seed=sd), init_labels=lab0)
        else:
            o = oracle.solve(X, oracle.make_params(r, lam=lam, tol=1e-6, seed=sd))
        T.append(o)
    emb = [cs[2] for cs in cases] + [None, None]
    labs = [None] * len(cases) + [torch.from_numpy(lab0).cuda(), None]
    plist, keep = rp.batch_params(ranks, lams, tol=0.0, max_iter=0, seeds=seeds, init_labels=labs,
                                  init_embeddings=emb, embedding_refine=refine)
    for p, o in zip(plist, T):
        p.max_iter = o["info"]["iters"]
    outs, infos, status = rp.solve_batched([dev(X) for X in Xall], plist)
    for i, (X, o) in enumerate(zip(Xall, T)):
        say(f"batched embedding instance {i} {X.shape} iters {infos[i]['iters']} / {o['info']['iters']}")
        assert infos[i]["iters"] == o["info"]["iters"]
        want_init = o["emb_steps"] if "emb_steps" in o else o["info"]["init_lloyd"]
        assert infos[i]["init_lloyd"] == want_init
        np.testing.assert_array_equal(outs[i][2].cpu().numpy(), o["labels"])
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(outs[i][0]), o["L"], nX) <= F32_TOL, i
        assert rel(host(outs[i][1]), o["S"], nX) <= F32_TOL, i


def test_warmstart_batched_matches_oracle_network():
    """Batched warm start: every instance's predicted sketches and rho0 against the
    FP64 sketch -> features -> network chain, and against the one-instance call."""
    from oracle import mlp as omlp
    hidden = 32
    dims = [68, hidden, hidden, hidden, 65]
    p = omlp.init_params(dims, 9).astype(np.float32)
    P = torch.from_numpy(p).cuda()
    rng = np.random.default_rng(8)
    shapes = [(300, 200, 5), (17, 90, 3), (1030, 411, 8)]
    Xs = [np.asfortranarray(rng.normal(0, 2, (d, n)).astype(np.float32)) for d, n, _ in shapes]
    views, rho0s, fbs = rp.warmstart_batched([dev(X) for X in Xs], [s[2] for s in shapes], P, hidden,
                                             sketch_seed=21)
    for X, (d, n, c), v, r0, fb in zip(Xs, shapes, views, rho0s, fbs):
        Yo = oracle.sketch(X, 21)
        yo, _ = omlp.forward(p.astype(np.float64), dims, omlp.features(Yo, d, c))
        assert v.shape == (64, n) and v.stride() == (1, 65)
        assert rel(v.cpu().numpy().astype(np.float64).T, yo[:, :64], 1.0) <= 5e-4
        s = np.linalg.norm(X.astype(np.float64)) / np.sqrt(d * n)
        assert not fb
        assert r0 == pytest.approx(np.exp(yo[:, 64].mean()) / s, rel=1e-3)
        _, r1, _ = rp.warmstart(dev(X), c, P, hidden, sketch_seed=21)
        assert r0 == pytest.approx(r1, rel=1e-4)   # batched sketch sums on the matrix cores


def test_warm_started_batched_solve_matches_oracle_chain():
    """Whole warm-started path (sketch -> network -> K-means of the predicted sketches ->
    iterations from rho0) against the same chain on the oracle side, for a network
    with fixed random weights: labels equal, L and S within the FP32 bar."""
    from oracle import mlp as omlp
    hidden = 64
    dims = [68, hidden, hidden, hidden, 65]
    p = omlp.init_params(dims, 17).astype(np.float32)
    P = torch.from_numpy(p).cuda()
    shapes = [(400, 300, 4), (90, 500, 6)]
    Xs = [synth.clustered(d, n, c, seed=60 + i, sep=4.0, noise=0.3, frac=0.05, amp=8.0,
                          dtype=np.float32, min_size=3)[0] for i, (d, n, c) in enumerate(shapes)]
    views, rho0s, _ = rp.warmstart_batched([dev(X) for X in Xs], [s[2] for s in shapes], P, hidden,
                                           sketch_seed=5)
    T = []
    for X, (d, n, c), r0 in zip(Xs, shapes, rho0s):
        yo, _ = omlp.forward(p.astype(np.float64), dims, omlp.features(oracle.sketch(X, 5), d, c))
        s = np.linalg.norm(X.astype(np.float64)) / np.sqrt(d * n)
        rho0_o = float(np.exp(yo[:, 64].mean()) / s)
        assert r0 == pytest.approx(rho0_o, rel=1e-4)
        lab, _, steps = oracle.kmeans(np.asfortranarray(yo[:, :64].T), c, 0, 100)
        lab2, ref = _refine_on_x(X, lab, c)
        o = oracle.solve(X, oracle.make_params(c, lam=0.5, tol=1e-6, rho0=rho0_o), init_labels=lab2)
        o["emb_steps"] = steps + ref
        T.append(o)
    plist, keep = rp.batch_params([s[2] for s in shapes], [0.5, 0.5], tol=0.0, max_iter=0, rho0=rho0s,
                                  init_embeddings=views)
    for pp, o in zip(plist, T):
        pp.max_iter = o["info"]["iters"]
    outs, infos, _ = rp.solve_batched([dev(X) for X in Xs], plist)
    for i, (X, o) in enumerate(zip(Xs, T)):
        say(f"warm chain instance {i}: iters {infos[i]['iters']} init_lloyd {infos[i]['init_lloyd']}")
        assert infos[i]["init_lloyd"] == o["emb_steps"]
        np.testing.assert_array_equal(outs[i][2].cpu().numpy(), o["labels"])
        nX = np.linalg.norm(X.astype(np.float64))
        assert rel(host(outs[i][0]), o["L"], nX) <= F32_TOL
        assert rel(host(outs[i][1]), o["S"], nX) <= F32_TOL


def test_embedding_and_batched_warm_start_error_paths():
    """Invalid embedding shapes and warm-start batches are rejected with clear codes."""
    X, _, _, _ = synth.clustered(40, 30, 3, seed=1, dtype=np.float32)
    Xd = dev(X)
    bad_ld = torch.zeros((8, 30), dtype=torch.float32, device="cuda")[:8]
    p = rp.make_params(3, 0.5, 1e-6, 50, 1e-4, 1.5, 1e10, 100, 0, rp.F32)
    p.init_embedding = bad_ld.data_ptr()
    p.init_embedding_ld = 4          # below the row count
    p.init_embedding_rows = 8
    L = rp.empty_colmajor(40, 30, torch.float32, Xd.device)
    S = rp.empty_colmajor(40, 30, torch.float32, Xd.device)
    info = rp.Info()
    h = rp.handle(0)
    st = rp.lib().respca_solve(h._h, rp.ct.byref(p), 40, 30, Xd.data_ptr(), 40, L.data_ptr(), 40,
                               S.data_ptr(), 40, None, rp.ct.byref(info), rp._stream(None))
    assert st == rp.ERR_INVALID
    from oracle import mlp as omlp
    P = torch.from_numpy(omlp.init_params([68, 8, 8, 8, 65], 1).astype(np.float32)).cuda()
    with pytest.raises(rp.RespcaError):
        rp.warmstart_batched([Xd], [31], P, 8)            # more groups than columns
    with pytest.raises(rp.RespcaError):
        rp.warmstart_batched([Xd] * 1025, [3] * 1025, P, 8)   # above the batch limit
