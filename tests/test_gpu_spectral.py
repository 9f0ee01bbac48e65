"""Spectral-clustering p-step on the GPU against the FP64 oracle (oracle/spectral.py).

The row embedding is compared through what does not depend on the choice of
eigenbasis: the Gram matrix of its unit rows (E^T E, n x n) and the eigenvalues.
Whole solves are iteration-locked to the oracle's stop; labels, iteration and
Lloyd counts must be equal, L and S within the FP64 / FP32 bars, the support of
S equal on well-separated entries."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import spectral as osp  # noqa: E402
from paper_1904_07497_amd import respca as rp  # noqa: E402
from paper_1904_07497_amd import synth  # noqa: E402
from tests._trajectory import support_check  # noqa: E402

pytestmark = pytest.mark.gpu

F64_TOL, F32_TOL = 1e-10, 1e-5


def dev(a):
    return torch.from_numpy(np.asfortranarray(a)).to("cuda")


def host(t):
    return np.asfortranarray(t.detach().cpu().numpy().astype(np.float64))


def rel(a, b, fallback):
    den = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / (den if den > 0 else fallback)


def say(msg):
    print(msg, flush=True)


def _blocks(d, n, c, seed, spread=0.3, sep=20.0):
    """c tight, well separated groups of uneven size in R^d (columns shuffled)."""
    rng = np.random.default_rng(seed)
    centers = sep * rng.standard_normal((d, c))
    lab = rng.integers(0, c, n)
    lab[:c] = np.arange(c)
    X = centers[:, lab] + spread * rng.standard_normal((d, n))
    return np.asfortranarray(X), lab


@pytest.mark.parametrize("case", ["rings", "blocks", "ragged", "relative"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_embedding_matches_oracle(case, dtype):
    if case == "rings":
        X, _ = synth.rings(seed=1)
        c, sigma = 2, 0.5
    elif case == "blocks":
        X, _ = _blocks(37, 301, 5, seed=2)
        c, sigma = 5, 3.0
    elif case == "ragged":   # several 64-column tiles with a ragged edge, ragged 16-row stages
        X, _ = synth.rings(counts=(400, 500, 333), radii=(1.0, 3.0, 6.0), d=131, seed=3)
        c, sigma = 3, 0.7
    else:   # relative width: 0.15 times the spread of the columns, data scaled by 1e-3
        X, _ = synth.rings(counts=(300, 400), radii=(1.0, 4.0), d=40, seed=6)
        X = 1e-3 * X
        c, sigma = 2, -0.15
    X = X.astype(dtype, order="F")
    Xo = X.astype(np.float64)
    say(f"embedding {case} {X.shape} c={c} {np.dtype(dtype).name}")
    emb, vals, info = rp.spectral_embedding(dev(X), c, sigma, seed=4)
    U, ovals = osp.embedding(Xo, c, sigma)
    R = osp.unit_rows(U)
    E = emb.cpu().numpy()          # c x n, column j = unit row j
    assert info["eig_unconverged"] == 0
    np.testing.assert_allclose(vals, ovals, atol=1e-9)
    G_gpu = E.T @ E
    G_or = R @ R.T
    assert np.abs(G_gpu - G_or).max() <= 1e-7, np.abs(G_gpu - G_or).max()
    # unit rows
    np.testing.assert_allclose(np.linalg.norm(E, axis=0), 1.0, atol=1e-12)


def test_embedding_argument_checks():
    X = dev(np.ones((4, 10)))
    for kw, status in [(dict(sigma=0.0), rp.ERR_INVALID), (dict(sigma=float("nan")), rp.ERR_INVALID),
                       (dict(sigma=float("-inf")), rp.ERR_INVALID),
                       (dict(rank=10), rp.ERR_INVALID), (dict(rank=41), rp.ERR_UNSUPPORTED)]:
        args = dict(rank=2, sigma=1.0)
        args.update(kw)
        if args["rank"] == 41:
            X2 = dev(np.random.default_rng(0).standard_normal((4, 60)))
        else:
            X2 = X
        with pytest.raises(rp.RespcaError) as e:
            rp.spectral_embedding(X2, args["rank"], args["sigma"])
        assert e.value.status == status, kw


@pytest.mark.parametrize("dtype,precision", [(np.float64, rp.F64), (np.float32, rp.F32),
                                             (np.float32, rp.BF16GEMM_F32)])
def test_spectral_solve_matches_oracle(dtype, precision):
    """Lightly corrupted rings, lambda = 0.2: the spectral p-step's whole solve,
    iteration-locked to the oracle's stop at tol 1e-6."""
    X, ring = synth.rings(seed=3, frac=0.02, amp=2.0, dtype=dtype)
    d, n = X.shape
    c, sigma, lam = 2, 0.5, 0.2
    p = oracle.make_params(c, lam=lam, tol=1e-6, seed=0)
    o = osp.solve(X, p, sigma)
    T = o["info"]["iters"]
    say(f"spectral solve {X.shape} T={T} precision={precision}")
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=0, precision=precision,
                 pstep=rp.PSTEP_SPECTRAL, sigma=sigma)
    gi = g["info"]
    assert gi["iters"] == T and gi["eig_unconverged"] == 0
    assert gi["init_lloyd"] == o["info"]["init_lloyd"]
    assert gi["lloyd_steps"] == o["info"]["lloyd_steps"]
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    lab = o["labels"]
    assert np.array_equal(lab == lab[0], ring == ring[0])   # the rings themselves
    Xo = X.astype(np.float64)
    nX = np.linalg.norm(Xo)
    tol = F64_TOL if dtype == np.float64 else F32_TOL
    assert rel(host(g["L"]), o["L"], nX) <= tol
    assert rel(host(g["S"]), o["S"], nX) <= tol
    frac = support_check(Xo, o["L"], o["theta_prev"], o["rho_t"], host(g["S"]), o["S"],
                         np.finfo(dtype).eps)
    assert frac > 0.5


def test_spectral_solve_relative_width_matches_oracle():
    """The relative kernel width (sigma < 0: |sigma| times the columns' spread, which
    follows L as the L-step shrinks it): three rings, iteration-locked FP32 solve
    against the oracle; the groups are the rings."""
    X, ring = synth.rings(counts=(150, 200, 250), radii=(1.0, 4.0, 7.0), d=30, noise=0.01, seed=8,
                          frac=0.01, amp=0.5, dtype=np.float32)
    c, sigma, lam = 3, -0.1, 0.05
    p = oracle.make_params(c, lam=lam, tol=1e-6, seed=0)
    o = osp.solve(X, p, sigma)
    T = o["info"]["iters"]
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=0, precision=rp.F32,
                 pstep=rp.PSTEP_SPECTRAL, sigma=sigma)
    assert g["info"]["iters"] == T and g["info"]["eig_unconverged"] == 0
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    lab = o["labels"]
    assert all(len(set(lab[ring == r])) == 1 for r in range(3)) and len(set(lab.tolist())) == 3
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F32_TOL


def test_spectral_solve_two_moons_matches_oracle():
    """The spectral benchmark's kind of data at a smaller size (two moons, relative
    width 0.1, lambda 0.05): iteration-locked FP32 solve against the oracle, and the
    groups are the moons."""
    X, moon = synth.moons(counts=(300, 300), d=100, noise=0.005, seed=5, frac=0.002, amp=0.3,
                          dtype=np.float32)
    c, sigma, lam = 2, -0.1, 0.05
    p = oracle.make_params(c, lam=lam, tol=1e-6, seed=0)
    o = osp.solve(X, p, sigma)
    T = o["info"]["iters"]
    say(f"spectral moons solve {X.shape} T={T}")
    g = rp.solve(dev(X), rank=c, lam=lam, tol=0.0, max_iter=T, seed=0, precision=rp.F32,
                 pstep=rp.PSTEP_SPECTRAL, sigma=sigma)
    assert g["info"]["iters"] == T and g["info"]["eig_unconverged"] == 0
    assert g["info"]["lloyd_steps"] == o["info"]["lloyd_steps"]
    np.testing.assert_array_equal(g["labels"].cpu().numpy(), o["labels"])
    assert np.array_equal(o["labels"] == o["labels"][0], moon == moon[0])
    nX = np.linalg.norm(X.astype(np.float64))
    assert rel(host(g["L"]), o["L"], nX) <= F32_TOL
    assert rel(host(g["S"]), o["S"], nX) <= F32_TOL


def test_spectral_iterate_matches_oracle_step():
    """One iteration with the spectral p-step from an arbitrary state (three blocks,
    random groups): labels, L, S and Theta / rho against the oracle's step."""
    X, _ = _blocks(50, 400, 3, seed=7, spread=0.5, sep=10.0)
    d, n = X.shape
    rng = np.random.default_rng(1)
    st = {"L": np.asfortranarray(X + 0.1 * rng.standard_normal((d, n))),
          "S": np.zeros((d, n), order="F"),
          "Theta": np.asfortranarray(rng.uniform(-1, 1, (d, n))),
          "labels": rng.integers(0, 3, n).astype(np.int32),
          "C": np.asfortranarray(rng.standard_normal((d, 3))), "rho": 0.3}
    p = oracle.make_params(3, lam=0.5)
    ref = osp.step(p, X, st, 2.0)
    gs = {"L": dev(st["L"]), "S": dev(st["S"]), "Theta": dev(st["Theta"]),
          "labels": torch.from_numpy(st["labels"].copy()).cuda(), "C": dev(st["C"]), "rho": 0.3}
    norms, info = rp.iterate(dev(X), gs, iters=1, lam=0.5, precision=rp.F64,
                             pstep=rp.PSTEP_SPECTRAL, sigma=2.0)
    np.testing.assert_array_equal(gs["labels"].cpu().numpy(), ref["labels"])
    assert info["lloyd_steps"] == ref["lloyd"]
    nX = np.linalg.norm(X)
    for k in ("L", "S"):
        assert rel(host(gs[k]), ref[k], nX) <= F64_TOL, k
    assert np.linalg.norm(host(gs["Theta"]) - ref["Theta"]) / 0.3 / nX <= F64_TOL
    np.testing.assert_allclose(norms[0], ref["norms"], rtol=1e-9)


def test_spectral_option_error_paths():
    X = dev(np.random.default_rng(0).standard_normal((20, 50)).astype(np.float32))
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=2, lam=1.0, pstep=rp.PSTEP_SPECTRAL, sigma=0.0)
    assert e.value.status == rp.ERR_INVALID
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=2, lam=1.0, pstep=7, sigma=1.0)
    assert e.value.status == rp.ERR_INVALID
    with pytest.raises(rp.RespcaError) as e:
        rp.solve(X, rank=41, lam=1.0, pstep=rp.PSTEP_SPECTRAL, sigma=1.0)
    assert e.value.status == rp.ERR_UNSUPPORTED
    plist, _ = rp.batch_params([2], [1.0])
    plist[0].pstep, plist[0].spectral_sigma = rp.PSTEP_SPECTRAL, 1.0
    with pytest.raises(rp.RespcaError) as e:
        rp.solve_batched([X], plist)
    assert e.value.status == rp.ERR_UNSUPPORTED
    st = {"L": X.clone(), "S": torch.zeros_like(X), "Theta": torch.zeros_like(X),
          "labels": torch.zeros(50, dtype=torch.int32, device="cuda"),
          "C": rp.empty_colmajor(20, 2, torch.float32, "cuda").zero_(), "rho": 0.1}
    with pytest.raises(rp.RespcaError) as e:
        rp.iterate(X, st, iters=1, lam=1.0, noalloc=True, pstep=rp.PSTEP_SPECTRAL, sigma=1.0)
    assert e.value.status == rp.ERR_UNSUPPORTED
