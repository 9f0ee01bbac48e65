"""Second, independent RES-PCA implementation in NumPy -- tests only, tiny inputs.

It differs from the C oracle on purpose where the paper gives two routes to the
same quantity: the L-step here solves the per-group linear system of the
first-order condition (Sec. 4.1, eq_sub_L_de_deriv) with a dense solver instead
of using the Sherman-Morrison-Woodbury closed form, and distances are formed
with broadcasting.  The control flow (k-means++ from splitmix64, Lloyd until no
label changes, L -> p -> S -> Theta order, the Sec. 5 stopping rule) follows the
same written readings of the paper.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1


def splitmix64_stream(seed: int):
    state = seed & MASK
    while True:
        state = (state + 0x9E3779B97F4A7C15) & MASK
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        yield z ^ (z >> 31)


def uniforms(seed: int):
    for x in splitmix64_stream(seed):
        yield (x >> 11) / float(1 << 53)


def sqdist(Y, C):
    """n x c matrix of squared distances between columns of Y and of C."""
    return ((Y[:, :, None] - C[:, None, :]) ** 2).sum(axis=0)


def assign(Y, C):
    return np.argmin(sqdist(Y, C), axis=1).astype(np.int32)   # argmin: first minimum


def means(Y, labels, C_prev):
    C = C_prev.copy()
    for k in range(C.shape[1]):
        m = labels == k
        if m.any():
            C[:, k] = Y[:, m].mean(axis=1)
    return C


def lloyd(Y, C, labels, max_lloyd):
    steps = 0
    while steps < max_lloyd:
        nxt = assign(Y, C)
        steps += 1
        if np.array_equal(nxt, labels):
            break
        labels = nxt
        C = means(Y, labels, C)
    return labels, C, steps


def kmeanspp(Y, c, seed):
    d, n = Y.shape
    u = uniforms(seed)
    s = min(int(np.floor(next(u) * n)), n - 1)
    seeds = [s]
    d2 = ((Y - Y[:, [s]]) ** 2).sum(axis=0)
    for _ in range(1, c):
        total = float(np.sum(d2))
        uu = next(u)
        if total > 0:
            run = np.cumsum(d2)
            idx = np.nonzero(run > uu * total)[0]
            s = int(idx[0]) if idx.size else int(np.nonzero(d2 > 0)[0][-1])
        else:
            s = next(j for j in range(n) if j not in seeds)
        seeds.append(s)
        d2 = np.minimum(d2, ((Y - Y[:, [s]]) ** 2).sum(axis=0))
    return np.array(seeds)


def kmeans(Y, c, seed, max_lloyd):
    seeds = kmeanspp(Y, c, seed)
    C = Y[:, seeds].copy()
    labels = assign(Y, C)
    C = means(Y, labels, C)
    labels, C, steps = lloyd(Y, C, labels, max_lloyd)
    return labels, C, steps


def l_step_dense(X, S, Theta, labels, c, lam, rho, C_prev):
    """Per group k: L_k (2 lam M_k + rho I) = rho D_k, solved densely."""
    D = X - S + Theta / rho
    L = np.empty_like(D)
    C = C_prev.copy()
    for k in range(c):
        idx = np.nonzero(labels == k)[0]
        if idx.size == 0:
            continue
        nk = idx.size
        M = np.eye(nk) - np.ones((nk, nk)) / nk
        A = 2 * lam * M + rho * np.eye(nk)
        # L_k A = rho D_k  <=>  A^T L_k^T = rho D_k^T
        L[:, idx] = np.linalg.solve(A.T, rho * D[:, idx].T).T
        C[:, k] = D[:, idx].mean(axis=1)
    return L, C


def soft(B, t):
    return np.sign(B) * np.maximum(np.abs(B) - t, 0.0)


def block_soft(B, t):
    """Proximal map of t * sum_j ||B_j||_2, by the Moreau identity: B minus its
    column-wise projection onto the ball of radius t."""
    nb = np.linalg.norm(B, axis=0)
    proj = B * np.minimum(1.0, t / np.where(nb > 0, nb, 1.0))
    return B - proj


def solve(X, c, lam, tol=1e-3, max_iter=500, rho0=1e-4, kappa=1.5, rho_max=1e10,
          max_lloyd=100, seed=0, sparse_norm=0):
    X = np.asarray(X, dtype=np.float64)
    nX = np.linalg.norm(X)
    d, n = X.shape
    labels, C, init_steps = kmeans(X, c, seed, max_lloyd)
    S = np.zeros_like(X)
    Th = np.zeros_like(X)
    Lp = np.zeros_like(X)
    rho = rho0
    it = 0
    crit = np.inf
    for it in range(1, max_iter + 1):
        L, C = l_step_dense(X, S, Th, labels, c, lam, rho, C)
        labels, C, _ = lloyd(L, C, labels, max_lloyd)
        prox = block_soft if sparse_norm == 1 else soft
        Sn = prox(X - L + Th / rho, 1.0 / rho)
        Th = Th + rho * (X - L - Sn)
        crit = max(np.linalg.norm(X - L - Sn), np.linalg.norm(L - Lp), np.linalg.norm(Sn - S)) / nX
        S, Lp = Sn, L
        rho = min(kappa * rho, rho_max)
        if crit <= tol:
            break
    return {"L": Lp, "S": S, "labels": labels, "iters": it, "crit": crit}


def ialm(X, lam=None, tol=1e-7, max_iter=1000, rho=1.5):
    """Inexact ALM for convex RPCA, min ||L||_* + lam ||S||_1 s.t. X = L + S
    (Lin, Chen & Ma 2010), with full SVDs -- tiny inputs only."""
    X = np.asarray(X, dtype=np.float64)
    d, n = X.shape
    if lam is None:
        lam = 1.0 / np.sqrt(max(d, n))
    norm2 = np.linalg.norm(X, 2)
    Y = X / max(norm2, np.abs(X).max() / lam)
    mu = 1.25 / norm2
    mu_max = mu * 1e7
    S = np.zeros_like(X)
    L = np.zeros_like(X)
    nX = np.linalg.norm(X)
    for _ in range(max_iter):
        U, s, Vt = np.linalg.svd(X - S + Y / mu, full_matrices=False)
        L = (U * np.maximum(s - 1.0 / mu, 0.0)) @ Vt
        S = soft(X - L + Y / mu, lam / mu)
        R = X - L - S
        Y = Y + mu * R
        mu = min(mu * rho, mu_max)
        if np.linalg.norm(R) / nX < tol:
            break
    return L, S
