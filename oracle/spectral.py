"""FP64 NumPy reference of the spectral-clustering p-step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module; the GPU library never uses it.

Sec. 4.2 ends by noting that the groups may be found by another clustering
method than K-means, and names spectral clustering as the choice for data whose
groups lie on nonlinear structures (the Remark closing Sec. 3 calls this the
direct nonlinear extension).  The paper gives no further detail, so this module
takes the normalised spectral clustering of Ng, Jordan & Weiss (NIPS 2001):

  affinity      W_ij = exp(-||y_i - y_j||^2 / (2 sigma^2)) for i != j, W_ii = 0
                (sigma given, or a multiple of the columns' spread: kernel_width)
  normalisation A = D^{-1/2} W D^{-1/2},  D = diag(sum_j W_ij)
                (a point with zero degree gets a zero row and column)
  embedding     U = eigenvectors of the c largest eigenvalues of A (n x c)
  rows          each row of U scaled to unit length (a zero row stays zero)
  clustering    K-means of the rows.

Within the RES-PCA iteration only the p-step changes (L-step, S-step and the
multiplier update are those of Sec. 4.1, 4.3 and 4.4): the rows of the
embedding of L are clustered by Lloyd passes that start from the current groups
(their centroids are the group means of the rows, an empty group's centroid is
the zero vector), the same warm start the K-means p-step uses.  The initial
groups are the spectral clustering of the columns of X with k-means++ seeding
from splitmix64(seed), then Lloyd.  K-means on the rows depends on the
embedding only through distances between rows, so any orthonormal basis of the
top-c eigenspace gives the same groups.
"""
from __future__ import annotations

import numpy as np

import oracle


def spread(Y):
    """Root mean square distance of the columns of Y to their mean column."""
    Y = np.asarray(Y, np.float64)
    mean = Y.mean(axis=1, keepdims=True)
    return float(np.sqrt(np.mean(np.sum((Y - mean) ** 2, axis=0))))


def kernel_width(Y, sigma):
    """The kernel width: sigma itself when positive; when negative, |sigma| times the
    spread of the columns (a width that follows the scale of L, which the L-step
    shrinks toward the group means by rho / (2 lambda + rho) in early iterations)."""
    return sigma if sigma > 0 else -sigma * spread(Y)


def affinity(Y, sigma):
    """W (n x n) for the columns of Y (d x n): Gaussian kernel of the squared
    Euclidean distance, computed as the sum of squared differences; zero diagonal.
    sigma < 0 selects the relative width of kernel_width."""
    Y = np.asarray(Y, np.float64)
    n = Y.shape[1]
    sigma = kernel_width(Y, sigma)
    # a zero width (all columns equal) makes every distance zero: W = 1 off the diagonal
    inv = 0.0 if sigma == 0.0 else 1.0 / (2.0 * sigma * sigma)
    W = np.zeros((n, n))
    for j in range(n):
        diff = Y - Y[:, j:j + 1]
        W[:, j] = np.exp(-np.sum(diff * diff, axis=0) * inv)
        W[j, j] = 0.0
    return W


def normalized_affinity(W):
    """A = D^{-1/2} W D^{-1/2}; also returns the degrees."""
    deg = W.sum(axis=1)
    s = np.zeros_like(deg)
    pos = deg > 0
    s[pos] = 1.0 / np.sqrt(deg[pos])
    return s[:, None] * W * s[None, :], deg


def embedding(Y, c, sigma):
    """Eigenvectors (n x c, columns in decreasing eigenvalue order) of the c largest
    eigenvalues of the normalised affinity of Y's columns, and those eigenvalues."""
    A, _ = normalized_affinity(affinity(Y, sigma))
    vals, vecs = np.linalg.eigh(A)
    order = np.argsort(vals)[::-1][:c]
    return vecs[:, order], vals[order]


def unit_rows(U):
    """Rows scaled to unit Euclidean length; zero rows stay zero."""
    nr = np.sqrt(np.sum(U * U, axis=1))
    out = np.zeros_like(U)
    pos = nr > 0
    out[pos] = U[pos] / nr[pos, None]
    return out


def row_embedding(Y, c, sigma):
    """The points K-means clusters: unit rows of the embedding, as the columns of a
    c x n matrix."""
    U, _ = embedding(Y, c, sigma)
    return np.asfortranarray(unit_rows(U).T)


def spectral_init(X, c, sigma, seed, max_lloyd=100):
    """Initial groups: k-means++ (splitmix64(seed)) then Lloyd on the row embedding
    of X's columns.  Returns (labels, Lloyd passes)."""
    E = row_embedding(X, c, sigma)
    labels, _, steps = oracle.kmeans(E, c, seed, max_lloyd)
    return labels, steps


def spectral_pstep(L, labels, c, sigma, max_lloyd=100):
    """p-step: Lloyd on the row embedding of L's columns from the current groups.
    Returns (labels, Lloyd passes)."""
    E = row_embedding(L, c, sigma)
    C0, _ = oracle.group_means(E, labels, c, mean_init=np.zeros((c, c), order="F"))
    lab, _, steps = oracle.lloyd(E, C0, labels, max_lloyd)
    return lab, steps


def step(params, X, state, sigma):
    """One outer iteration with the spectral p-step, in the section order of the
    K-means iteration: L-step (Sec. 4.1), p-step, S-step (Sec. 4.3), multiplier
    and penalty (Sec. 4.4).  Returns a new state dict with norms and lloyd."""
    X = np.asarray(X, np.float64, order="F")
    rho = float(state["rho"])
    c = params.c
    L, C = oracle.l_step(X, state["S"], state["Theta"], state["labels"], c, params.lam, rho,
                         C_init=state["C"])
    labels, steps = spectral_pstep(L, state["labels"], c, sigma, params.max_lloyd)
    S = oracle.s_step(X, L, state["Theta"], rho, params.sparse_norm)
    Theta = oracle.theta_step(X, L, S, state["Theta"], rho)
    norms = np.array([np.linalg.norm(X - L - S), np.linalg.norm(L - state["L"]),
                      np.linalg.norm(S - state["S"])])
    return {"L": L, "S": S, "Theta": Theta, "labels": labels, "C": C,
            "rho": min(params.kappa * rho, params.rho_max), "norms": norms, "lloyd": steps}


def solve(X, params, sigma, init_labels=None, max_iter=None):
    """Whole solve with the spectral p-step: S = Theta = 0, L_0 = 0, rho = rho0,
    groups from spectral_init (or init_labels), centroids the group means of X;
    iterations until the Sec. 5 criterion <= tol or max_iter.  Returns a dict
    like oracle.solve (plus theta_prev and rho_t of the last step)."""
    X = np.asarray(X, np.float64, order="F")
    d, n = X.shape
    c = params.c
    T = params.max_iter if max_iter is None else max_iter
    init_lloyd = 0
    if init_labels is None:
        labels, init_lloyd = spectral_init(X, c, sigma, params.seed, params.max_lloyd)
    else:
        labels = np.ascontiguousarray(init_labels, dtype=np.int32)
    C, _ = oracle.group_means(X, labels, c, mean_init=np.zeros((d, c), order="F"))
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.zeros((d, n), order="F"), "labels": labels, "C": C, "rho": params.rho0}
    nX = np.linalg.norm(X)
    info = {"iters": 0, "lloyd_steps": 0, "init_lloyd": init_lloyd, "status": 1}
    theta_prev, rho_t = st["Theta"], st["rho"]
    for t in range(1, T + 1):
        theta_prev, rho_t = st["Theta"], st["rho"]
        st = step(params, X, st, sigma)
        info["iters"] = t
        info["lloyd_steps"] += st["lloyd"]
        crit = max(st["norms"]) / nX
        info.update(primal=st["norms"][0] / nX, dL=st["norms"][1] / nX, dS=st["norms"][2] / nX,
                    rho_final=rho_t)
        if crit <= params.tol:
            info["status"] = 0
            break
    return {"L": st["L"], "S": st["S"], "Theta": st["Theta"], "labels": st["labels"],
            "C": st["C"], "info": info, "theta_prev": theta_prev, "rho_t": rho_t}
