"""Pins of the spectral-clustering p-step reference (oracle/spectral.py): the
normalised spectral clustering of Ng, Jordan & Weiss that Sec. 4.2 names as the
nonlinear alternative to K-means.  Each pin is fixed by hand or by a property the
mathematics fixes, not by re-running the same formulas."""
import math

import numpy as np
import pytest

import oracle
from oracle import spectral as sp
from paper_1904_07497_amd import synth

# points on a line; with sigma^2 = 1 / (2 ln 2) two points at distance 1 have
# affinity exp(-ln 2) = 1/2 and at distance 2 exp(-4 ln 2) = 1/16
SIGMA = 1.0 / math.sqrt(2.0 * math.log(2.0))
BLOCKS = np.array([[0.0, 1.0, 100.0, 101.0, 102.0]])


def test_two_points_closed_form():
    """W = [[0, 1/2], [1/2, 0]], D = I/2, A = [[0, 1], [1, 0]]: eigenvalues +-1; the
    top eigenvector is (1, 1)/sqrt 2 and its unit rows are both +-1 of one sign."""
    Y = np.array([[0.0, 1.0]])
    W = sp.affinity(Y, SIGMA)
    np.testing.assert_allclose(W, [[0.0, 0.5], [0.5, 0.0]], rtol=1e-15)
    A, deg = sp.normalized_affinity(W)
    np.testing.assert_allclose(A, [[0.0, 1.0], [1.0, 0.0]], rtol=1e-15)
    U, vals = sp.embedding(Y, 1, SIGMA)
    assert vals[0] == pytest.approx(1.0, rel=1e-15)
    np.testing.assert_allclose(np.abs(U[:, 0]), [2 ** -0.5] * 2, rtol=1e-14)
    R = sp.unit_rows(U)
    assert abs(R[0, 0]) == pytest.approx(1.0) and R[0, 0] == pytest.approx(R[1, 0])


def test_hand_worked_block_spectrum():
    """Blocks {0, 1} and {100, 101, 102} (no affinity across: exp(-99^2 ln 2) is 0 in
    double).  Block 1: A = [[0, 1], [1, 0]], eigenvalues 1, -1.  Block 2: degrees
    9/16, 1, 9/16, so A = [[0, 2/3, 1/9], [2/3, 0, 2/3], [1/9, 2/3, 0]] with
    eigenvalues 1 (vector (3, 4, 3) / sqrt 34), -1/9 (vector (1, 0, -1)) and, from
    the zero trace, -8/9."""
    W = sp.affinity(BLOCKS, SIGMA)
    assert W[2, 4] == pytest.approx(1 / 16, rel=1e-14) and W[0, 2] == 0.0
    assert np.all(np.diag(W) == 0)
    A, deg = sp.normalized_affinity(W)
    np.testing.assert_allclose(deg, [0.5, 0.5, 9 / 16, 1.0, 9 / 16], rtol=1e-14)
    np.testing.assert_allclose(A[2:, 2:], [[0, 2 / 3, 1 / 9], [2 / 3, 0, 2 / 3], [1 / 9, 2 / 3, 0]],
                               rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(A)), [-1, -8 / 9, -1 / 9, 1, 1],
                               atol=1e-14)
    # the top-2 eigenspace is spanned by D^{1/2} times the block indicators
    U, vals = sp.embedding(BLOCKS, 2, SIGMA)
    np.testing.assert_allclose(vals, [1.0, 1.0], atol=1e-14)
    va = np.array([1, 1, 0, 0, 0]) / math.sqrt(2)
    vb = np.array([0, 0, 3, 4, 3]) / math.sqrt(34)
    np.testing.assert_allclose(U @ U.T, np.outer(va, va) + np.outer(vb, vb), atol=1e-13)
    # unit rows: equal within a block, orthogonal across blocks
    R = sp.unit_rows(U)
    np.testing.assert_allclose(R[0], R[1], atol=1e-13)
    np.testing.assert_allclose(R[2], R[4], atol=1e-13)
    np.testing.assert_allclose(R[3], R[2], atol=1e-13)
    assert abs(R[0] @ R[2]) < 1e-13


def test_spectral_init_recovers_the_blocks():
    lab, _ = sp.spectral_init(BLOCKS, 2, SIGMA, seed=0)
    assert lab[0] == lab[1] and lab[2] == lab[3] == lab[4] and lab[0] != lab[2]


def test_isolated_point_gets_a_zero_row():
    """A point with no affinity to any other (degree 0) has a zero row in A and in
    the embedding, and unit_rows keeps it at zero."""
    Y = np.array([[0.0, 1.0, 1000.0]])
    A, deg = sp.normalized_affinity(sp.affinity(Y, SIGMA))
    assert deg[2] == 0 and np.all(A[2] == 0) and np.all(A[:, 2] == 0)
    R = sp.unit_rows(np.array([[0.6, 0.8], [0.0, 0.0]]))
    np.testing.assert_allclose(R, [[0.6, 0.8], [0.0, 0.0]])


def test_rings_split_by_spectral_clustering_not_by_kmeans():
    """Two concentric rings in a random plane of R^20: K-means (c = 2) cuts across
    them; spectral clustering returns the rings."""
    X, ring = synth.rings(seed=1)
    lab, _ = sp.spectral_init(X, 2, 0.5, seed=0)
    assert np.array_equal(lab == lab[0], ring == ring[0])
    lk, _, _ = oracle.kmeans(X, 2, 0)
    agree = max(np.mean(lk == ring), np.mean(lk != ring))
    assert agree < 0.8


def test_row_clustering_does_not_depend_on_the_eigenbasis():
    """K-means of the unit rows is unchanged when the embedding is multiplied by an
    orthogonal c x c matrix (distances between rows are preserved), so two
    implementations whose eigensolvers return different bases of the same
    eigenspace agree."""
    X, _ = synth.rings(counts=(40, 50, 60), radii=(1.0, 3.0, 6.0), seed=4)
    U, _ = sp.embedding(X, 3, 0.6)
    Q, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((3, 3)))
    E1 = np.asfortranarray(sp.unit_rows(U).T)
    E2 = np.asfortranarray(sp.unit_rows(U @ Q).T)
    l1, _, s1 = oracle.kmeans(E1, 3, 5)
    l2, _, s2 = oracle.kmeans(E2, 3, 5)
    assert np.array_equal(l1, l2) and s1 == s2


def test_spectral_step_identities():
    """One iteration with the spectral p-step keeps the L-step and multiplier
    identities (group means of L = group means of D under the incoming groups;
    Theta' = clip(rho B, -1, 1)) and its groups are a Lloyd fixed point of the row
    embedding of L."""
    X, ring = synth.rings(seed=2, frac=0.05, amp=3.0)
    d, n = X.shape
    rng = np.random.default_rng(0)
    p = oracle.make_params(2, lam=0.5)
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.asfortranarray(rng.uniform(-1, 1, (d, n))),
          "labels": rng.integers(0, 2, n).astype(np.int32), "C": np.zeros((d, 2), order="F"),
          "rho": 0.7}
    out = sp.step(p, X, st, 0.5)
    D = X - st["S"] + st["Theta"] / st["rho"]
    for k in range(2):
        m = st["labels"] == k
        np.testing.assert_allclose(out["L"][:, m].mean(axis=1), D[:, m].mean(axis=1), atol=1e-12)
    B = X - out["L"] + st["Theta"] / st["rho"]
    np.testing.assert_allclose(out["Theta"], np.clip(st["rho"] * B, -1, 1), atol=1e-12)
    E = sp.row_embedding(out["L"], 2, 0.5)
    C, _ = oracle.group_means(E, out["labels"], 2)
    assert np.array_equal(oracle.assign(E, C), out["labels"])


def test_spectral_solve_recovers_rings_where_kmeans_pstep_does_not():
    """RES-PCA with the spectral p-step on lightly corrupted rings (2 % of entries
    offset by up to 2) converges and its groups are the rings; with the K-means
    p-step they are not.  (A large lambda would pull every column toward its group
    mean, the common centre of the rings, and erase the structure the clustering
    needs; lambda = 0.2 keeps it.)"""
    X, ring = synth.rings(seed=3, frac=0.02, amp=2.0)
    p = oracle.make_params(2, lam=0.2, tol=1e-6, seed=0)
    o = sp.solve(X, p, 0.5)
    assert o["info"]["status"] == 0
    lab = o["labels"]
    assert np.array_equal(lab == lab[0], ring == ring[0])
    km = oracle.solve(X, p)
    agree = max(np.mean(km["labels"] == ring), np.mean(km["labels"] != ring))
    assert agree < 0.8
    # the stopping criterion holds at the returned iterate
    assert np.linalg.norm(X - o["L"] - o["S"]) <= 1e-6 * np.linalg.norm(X) * (1 + 1e-9)


def test_spectral_solve_recovers_two_moons_where_kmeans_pstep_does_not():
    """Two moons (interleaved half circles with distinct means, the shape of the
    spectral benchmark workload at a smaller size), 0.2 % of entries offset: with
    the relative kernel width the spectral p-step keeps the moons from the first
    clustering to convergence, the K-means p-step cuts across them."""
    X, moon = synth.moons(counts=(300, 300), d=100, noise=0.005, seed=5, frac=0.002, amp=0.3)
    p = oracle.make_params(2, lam=0.05, tol=1e-6, seed=0)
    init, _ = sp.spectral_init(X, 2, -0.1, 0)
    assert np.array_equal(init == init[0], moon == moon[0])
    o = sp.solve(X, p, -0.1)
    assert o["info"]["status"] == 0
    assert np.array_equal(o["labels"] == o["labels"][0], moon == moon[0])
    km = oracle.solve(X, p)["labels"]
    assert max(np.mean(km == moon), np.mean(km != moon)) < 0.9


def test_relative_width_follows_the_scale_of_the_data():
    """sigma < 0 is relative: |sigma| times the RMS distance of the columns to their
    mean, so scaling the data by any factor leaves the affinity unchanged.  The
    spread of three points on a line at 0, 1, 5 is sqrt((4 + 1 + 9) / 3)."""
    Y = np.array([[0.0, 1.0, 5.0]])
    assert sp.spread(Y) == pytest.approx(math.sqrt(14 / 3), rel=1e-15)
    assert sp.kernel_width(Y, 0.7) == 0.7
    assert sp.kernel_width(Y, -0.5) == pytest.approx(0.5 * math.sqrt(14 / 3), rel=1e-15)
    X, _ = synth.rings(seed=1)
    np.testing.assert_allclose(sp.affinity(X, -0.2), sp.affinity(1e-3 * X, -0.2), rtol=1e-12,
                               atol=1e-300)
    np.testing.assert_allclose(sp.affinity(X, -0.2), sp.affinity(X, 0.2 * sp.spread(X)), rtol=1e-14)
