"""Seeded synthetic inputs for RES-PCA runs.

This module only draws random numbers (NumPy PCG64) and lays them out; it holds
none of the method's arithmetic, so both the GPU path and the FP64 CPU checker
can take their inputs from it.

Every matrix is returned as a NumPy array of shape (d, n) in Fortran
(column-major) order: column j is sample j, as in the paper (Sec. 3).  FP32
variants are produced by a single cast of the FP64 draw, so an FP64 consumer
that upcasts them sees exactly the values the FP32 consumer sees.

Workloads (the paper's videos, faces and digits are not available, so these
seeded constructions stand in for them):
  * low_rank_plus_sparse -- X = U V^T + S0 with U, V iid N(0, 1) and S0 zero
    except at a fraction of uniformly drawn positions, where it is uniform in
    [-a, a] (500 x 500 rank 25 at 5 % / [-50, 50]; 10^4 x 10^4 rank 100 at
    10 % / [-100, 100]; and the batched size mix).
  * video -- a 240 x 320 x n "surveillance" clip: a rank-5 slowly varying
    background built from smooth random bases, occluded by moving 20 x 20
    rectangles of uniform intensity (the sparse part), standing in for the
    Highway/Camera-Parameter style clips of the paper's Table 1.
  * clustered -- columns drawn around c well-separated group vectors plus
    sparse corruption: the structure the RES-PCA model assumes (Sec. 3).
  * random_state -- an arbitrary ALM state (S, Theta, labels, centroids) for
    checking one iteration in isolation.
"""
from __future__ import annotations

import math

import numpy as np


def _fortran(a_nd: np.ndarray) -> np.ndarray:
    """(n, d) C-ordered array -> (d, n) Fortran-ordered view (no copy)."""
    return a_nd.T


def low_rank_plus_sparse(d: int, n: int, rank: int, frac: float, amp: float, seed: int,
                         dtype=np.float64):
    """X = U V^T + S0; U (d x r), V (n x r) iid N(0,1); S0 has round(frac*d*n)
    entries at distinct uniform positions, values uniform in [-amp, amp].
    Returns (X, L0, S0) as (d, n) Fortran arrays of ``dtype``."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((d, rank))
    V = rng.standard_normal((n, rank))
    L0 = _fortran(V @ U.T)                         # (d, n), column-major
    k = int(round(frac * d * n))
    pos = rng.choice(d * n, size=k, replace=False) if k > 0 else np.zeros(0, np.int64)
    vals = rng.uniform(-amp, amp, size=k)
    S0 = np.zeros((d, n), order="F")
    S0.reshape(-1, order="F")[pos] = vals
    X = L0 + S0
    X = np.asfortranarray(X)
    if dtype != np.float64:
        X = X.astype(dtype, order="F")
        L0 = L0.astype(dtype, order="F")
        S0 = S0.astype(dtype, order="F")
    return X, L0, S0


def config_small(seed: int = 0, dtype=np.float64):
    """500 x 500, rank 25, 5 % corruptions uniform in [-50, 50]."""
    return low_rank_plus_sparse(500, 500, 25, 0.05, 50.0, seed, dtype)


def config_large(seed: int = 1, dtype=np.float32, d: int = 10000, n: int = 10000):
    """10^4 x 10^4, rank 100, 10 % corruptions uniform in [-100, 100]."""
    return low_rank_plus_sparse(d, n, 100, 0.10, 100.0, seed, dtype)


def _smooth_field(rng, h, w, sigma):
    from scipy.ndimage import gaussian_filter
    f = gaussian_filter(rng.standard_normal((h, w)), sigma=sigma, mode="wrap")
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return f


def _smooth_walk(rng, n, sigma):
    from scipy.ndimage import gaussian_filter1d
    w = gaussian_filter1d(np.cumsum(rng.standard_normal(n)), sigma=sigma, mode="nearest")
    w = w - w.mean()
    return w / max(np.abs(w).max(), 1e-300)


def video(n: int = 2000, h: int = 240, w: int = 320, rank: int = 5, n_rect: int = 4,
          rect: int = 20, seed: int = 2, dtype=np.float32, scale: float = 255.0):
    """Synthetic surveillance clip, d = h*w pixels by n frames (column-major,
    frame j = column j, pixels row-major within the frame).

    Background: L0 = sum_k b_k a_k^T with b_1 a smooth field around 0.5 and
    a_1 = 1, b_2..b_r zero-mean smooth fields (Gaussian-blurred noise, sigma 16 px)
    and a_2..a_r smoothed random walks (sigma 50 frames) of amplitude 0.1-0.3;
    the result is clipped to [0, 1].  Foreground: ``n_rect`` rect x rect squares
    with constant velocity in [-3, 3] px/frame reflecting at the borders and
    uniform intensity in [0, 1]; they occlude the background, so
    S0 = intensity - L0 on covered pixels.  Everything is finally multiplied by
    ``scale`` (default 255: raw 8-bit frames).  The scale matters to the method:
    the S-step threshold 1/rho is absolute, so the iteration at which the
    geometric rho schedule stops depends on the data's magnitude.
    Returns (X, L0, S0)."""
    rng = np.random.default_rng(seed)
    d = h * w
    B = np.empty((d, rank))
    A = np.empty((rank, n))
    B[:, 0] = 0.35 + 0.3 * _smooth_field(rng, h, w, 16.0).reshape(-1)
    A[0, :] = 1.0
    for k in range(1, rank):
        B[:, k] = _smooth_field(rng, h, w, 16.0).reshape(-1) - 0.5
        A[k, :] = rng.uniform(0.1, 0.3) * _smooth_walk(rng, n, 50.0)
    L0nd = np.clip(A.T @ B.T, 0.0, 1.0)            # (n, d): frame j is row j
    Xnd = L0nd.copy()
    pos = np.stack([rng.uniform(0, h - rect, n_rect), rng.uniform(0, w - rect, n_rect)], 1)
    vel = rng.uniform(-3.0, 3.0, (n_rect, 2))
    inten = rng.uniform(0.0, 1.0, n_rect)
    lim = np.array([h - rect, w - rect], dtype=np.float64)
    for j in range(n):
        frame = Xnd[j].reshape(h, w)
        for r in range(n_rect):
            y0, x0 = int(round(pos[r, 0])), int(round(pos[r, 1]))
            frame[y0:y0 + rect, x0:x0 + rect] = inten[r]
        pos += vel
        for ax in range(2):                        # reflect at the borders
            lo = pos[:, ax] < 0
            hi = pos[:, ax] > lim[ax]
            pos[lo, ax] = -pos[lo, ax]
            pos[hi, ax] = 2 * lim[ax] - pos[hi, ax]
            vel[lo | hi, ax] = -vel[lo | hi, ax]
    Xnd *= scale
    L0nd *= scale
    X = _fortran(Xnd)
    L0 = _fortran(L0nd)
    S0 = np.asfortranarray(X - L0)
    if dtype != np.float64:
        X, L0, S0 = (a.astype(dtype, order="F") for a in (X, L0, S0))
    return X, L0, S0


def batch_instance(i: int, base_seed: int = 3_000_000, dtype=np.float32):
    """Instance i of the batched size mix: d, n log-uniform in [200, 4000],
    rank uniform in {5..50}, corruption fraction uniform in [1 %, 20 %],
    values uniform in [-50, 50], U, V iid N(0, 1).  Returns (X, rank, meta)."""
    rng = np.random.default_rng(base_seed + i)
    d = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
    n = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
    r = int(rng.integers(5, 51))
    frac = float(rng.uniform(0.01, 0.20))
    X, L0, S0 = low_rank_plus_sparse(d, n, r, frac, 50.0, int(rng.integers(0, 2**62)), dtype)
    return X, r, {"d": d, "n": n, "rank": r, "frac": frac, "L0": L0, "S0": S0}


def batch_shapes(count: int = 256, base_seed: int = 3_000_000):
    """(d, n, rank) of the first ``count`` batched instances without drawing the data."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        d = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
        n = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
        r = int(rng.integers(5, 51))
        out.append((d, n, r))
    return out


def clustered(d: int, n: int, c: int, seed: int, sep: float = 10.0, noise: float = 0.0,
              frac: float = 0.05, amp: float = 5.0, dtype=np.float64, min_size: int = 2):
    """Columns grouped around c group vectors: X[:, j] = G[:, g_j] + noise + S0[:, j].
    G has iid N(0, sep^2) entries; group sizes are at least ``min_size``; S0 has a
    fraction ``frac`` of entries uniform in [-amp, amp].  Returns (X, L0, S0, g)."""
    rng = np.random.default_rng(seed)
    G = rng.normal(0.0, sep, (d, c))
    g = np.concatenate([np.repeat(np.arange(c), min_size),
                        rng.integers(0, c, n - c * min_size)]) if n >= c * min_size \
        else rng.integers(0, c, n)
    g = rng.permutation(g).astype(np.int32)
    L0 = np.asfortranarray(G[:, g] + noise * rng.standard_normal((d, n)))
    k = int(round(frac * d * n))
    S0 = np.zeros((d, n), order="F")
    if k:
        pos = rng.choice(d * n, size=k, replace=False)
        S0.reshape(-1, order="F")[pos] = rng.uniform(-amp, amp, k)
    X = np.asfortranarray(L0 + S0)
    if dtype != np.float64:
        X, L0, S0 = (a.astype(dtype, order="F") for a in (X, L0, S0))
    return X, L0, S0, g


def random_state(X: np.ndarray, c: int, seed: int, s_frac: float = 0.1, s_amp: float = 1.0):
    """An arbitrary ALM state for one-iteration checks: labels uniform in [0, c),
    S sparse (fraction s_frac, values uniform in [-s_amp, s_amp]), Theta uniform in
    [-1, 1], L_prev = X plus N(0, 0.01) noise, centroids N(0, 1).  Same dtype as X."""
    rng = np.random.default_rng(seed)
    d, n = X.shape
    dt = X.dtype
    labels = rng.integers(0, c, n).astype(np.int32)
    mask = rng.random((n, d)) < s_frac
    S = _fortran(np.where(mask, rng.uniform(-s_amp, s_amp, (n, d)), 0.0)).astype(dt, order="F")
    Theta = _fortran(rng.uniform(-1.0, 1.0, (n, d))).astype(dt, order="F")
    Lp = (np.asarray(X, np.float64) + 0.1 * _fortran(rng.standard_normal((n, d)))).astype(dt, order="F")
    C = _fortran(rng.standard_normal((c, d))).astype(dt, order="F")
    return {"S": S, "Theta": Theta, "L": Lp, "labels": labels, "C": C}


def rings(counts=(60, 90), radii=(1.0, 4.0), d: int = 20, noise: float = 0.02, seed: int = 0,
          frac: float = 0.0, amp: float = 0.0, dtype=np.float64):
    """Points on concentric circles (the nonlinear group structure spectral
    clustering separates and K-means does not), placed in a random 2-D plane of
    R^d: ring k has counts[k] points at uniform random angles and radius radii[k],
    plus N(0, noise^2) in every coordinate; optionally a fraction `frac` of the
    entries replaced by sparse values uniform in [-amp, amp] added on top.
    Columns are shuffled.  Returns (X (d x n), ring index per column)."""
    rng = np.random.default_rng(seed)
    basis, _ = np.linalg.qr(rng.standard_normal((d, 2)))
    cols, member = [], []
    for k, (m, r) in enumerate(zip(counts, radii)):
        ang = rng.uniform(0.0, 2.0 * math.pi, m)
        pts = np.stack([r * np.cos(ang), r * np.sin(ang)])
        cols.append(basis @ pts + noise * rng.standard_normal((d, m)))
        member.append(np.full(m, k, dtype=np.int32))
    X = np.concatenate(cols, axis=1)
    ring = np.concatenate(member)
    perm = rng.permutation(X.shape[1])
    X, ring = X[:, perm], ring[perm]
    if frac > 0:
        k = int(round(frac * X.size))
        pos = rng.choice(X.size, size=k, replace=False)
        flat = X.reshape(-1, order="F")
        flat[pos] += rng.uniform(-amp, amp, k)
        X = flat.reshape(X.shape, order="F")
    return np.asfortranarray(X.astype(dtype)), ring


def moons(counts=(300, 300), d: int = 20, noise: float = 0.05, seed: int = 0,
          frac: float = 0.0, amp: float = 0.0, dtype=np.float64):
    """Two interleaved half circles of radius 1 (the classic two-moons layout, whose
    groups K-means splits across and spectral clustering follows): moon 0 at angles
    t in [0, pi] on (cos t, sin t), moon 1 on (1 - cos t, 1/2 - sin t), placed in
    a random 2-D plane of R^d with N(0, noise^2) in every coordinate; optionally a
    fraction `frac` of the entries offset by values uniform in [-amp, amp].
    Columns are shuffled.  Returns (X (d x n), moon index per column)."""
    rng = np.random.default_rng(seed)
    basis, _ = np.linalg.qr(rng.standard_normal((d, 2)))
    cols, member = [], []
    for k, m in enumerate(counts):
        t = rng.uniform(0.0, math.pi, m)
        pts = np.stack([np.cos(t), np.sin(t)]) if k == 0 else np.stack([1.0 - np.cos(t), 0.5 - np.sin(t)])
        cols.append(basis @ pts + noise * rng.standard_normal((d, m)))
        member.append(np.full(m, k, dtype=np.int32))
    X = np.concatenate(cols, axis=1)
    moon = np.concatenate(member)
    perm = rng.permutation(X.shape[1])
    X, moon = X[:, perm], moon[perm]
    if frac > 0:
        k = int(round(frac * X.size))
        pos = rng.choice(X.size, size=k, replace=False)
        flat = X.reshape(-1, order="F")
        flat[pos] += rng.uniform(-amp, amp, k)
        X = flat.reshape(X.shape, order="F")
    return np.asfortranarray(X.astype(dtype)), moon
