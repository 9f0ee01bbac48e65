"""Test helpers: the oracle's whole solve driven one outer iteration at a time,
so that the quantities of the last S-step (Theta before it and rho_t) are
available, and the support comparisons of S on well-separated entries.

The trajectory is the oracle's own solve loop (initial groups, then the Sec. 4
steps) taken through its step entry point for a fixed number of iterations; a
CPU test checks that it reproduces oracle.solve bit for bit.
"""
from __future__ import annotations

import numpy as np

import oracle


def trajectory(X, params, max_iter=None, init_labels=None):
    """Run the oracle from its initialisation for exactly ``max_iter`` outer
    iterations (default: the count at which oracle.solve stops with these
    params).  Returns (state, theta_prev, rho_t, iters) where state is the final
    step's output dict, theta_prev the multiplier before the last step and rho_t
    the penalty that step used."""
    X = np.asarray(X, np.float64, order="F")
    d, n = X.shape
    c = params.c
    if max_iter is None:
        max_iter = oracle.solve(X, params, init_labels=init_labels)["info"]["iters"]
    if init_labels is not None:
        labels = np.ascontiguousarray(init_labels, dtype=np.int32)
        C, _ = oracle.group_means(X, labels, c, mean_init=np.zeros((d, c), order="F"))
    else:
        labels, C, _ = oracle.kmeans(X, c, params.seed, params.max_lloyd)
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.zeros((d, n), order="F"), "labels": labels, "C": C, "rho": params.rho0}
    theta_prev, rho_t = st["Theta"], st["rho"]
    for _ in range(max_iter):
        theta_prev, rho_t = st["Theta"], st["rho"]
        st = oracle.step(params, X, st)
    return st, theta_prev, rho_t, max_iter


def support_check(X, L_or, Th_prev, rho, S_gpu, S_or, eps):
    """Zero pattern of S identical on entries where |B| = |X - L + Theta_prev/rho|
    is well away from the threshold 1/rho (margin above 64 eps times the
    magnitudes B is formed from).  Returns the fraction of such entries."""
    B = X - L_or + Th_prev / rho
    margin = np.abs(np.abs(B) - 1.0 / rho)
    bound = 64 * eps * (np.abs(X) + np.abs(L_or) + np.abs(Th_prev) / rho + 1.0 / rho)
    sep = margin > bound
    assert np.array_equal((S_gpu != 0)[sep], (S_or != 0)[sep])
    return sep.mean()


def column_support_check(X, L_or, Th_prev, rho, S_gpu, S_or, eps):
    """l2,1 penalty: zero and non-zero columns of S agree wherever rho ||B_j|| is
    well away from 1.  Returns (fraction separated, fraction of zero columns)."""
    B = X - L_or + Th_prev / rho
    nb = np.linalg.norm(B, axis=0)
    scale = np.linalg.norm(np.abs(X) + np.abs(L_or) + np.abs(Th_prev) / rho, axis=0)
    sep = np.abs(rho * nb - 1.0) > 64 * eps * rho * scale * np.sqrt(X.shape[0])
    gz = np.linalg.norm(S_gpu, axis=0) == 0
    oz = np.linalg.norm(S_or, axis=0) == 0
    assert np.array_equal(gz[sep], oz[sep])
    return sep.mean(), oz.mean()
