"""FP64 CPU oracle for RES-PCA (arXiv 1904.07497) -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The GPU library never imports, links or calls it.

The arithmetic lives in ``respca_oracle.c`` (plain C, FP64, index-order sums);
this module only compiles it with gcc and marshals NumPy arrays through ctypes.
Matrices are NumPy arrays of shape (d, n) in Fortran (column-major) order, so
``X[i, j]`` is entry (i, j) of the paper's X and ``X[:, j]`` is sample j.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "respca_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, ERR_INVALID, ERR_NONFINITE = 0, 1, -1, -2


def build() -> str:
    """Compile the oracle with gcc (no fast-math, so every sum keeps its order)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
           "-ffp-contract=off", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class Params(ct.Structure):
    _fields_ = [("lam", ct.c_double), ("c", ct.c_int32), ("tol", ct.c_double),
                ("max_iter", ct.c_int32), ("rho0", ct.c_double), ("kappa", ct.c_double),
                ("rho_max", ct.c_double), ("max_lloyd", ct.c_int32), ("seed", ct.c_uint64),
                ("sparse_norm", ct.c_int32)]


class Info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("lloyd_steps", ct.c_int32), ("init_lloyd", ct.c_int32),
                ("status", ct.c_int32), ("primal", ct.c_double), ("dL", ct.c_double),
                ("dS", ct.c_double), ("rho_final", ct.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ct.CDLL(_LIB)
        P = ct.POINTER
        dp, ip, lp = P(ct.c_double), P(ct.c_int32), P(ct.c_int64)
        i64, i32, f64 = ct.c_int64, ct.c_int32, ct.c_double
        L.oracle_splitmix64_next.restype = ct.c_uint64
        L.oracle_splitmix64_next.argtypes = [P(ct.c_uint64)]
        L.oracle_uniform01.restype = f64
        L.oracle_uniform01.argtypes = [P(ct.c_uint64)]
        L.oracle_splitmix64_at.restype = ct.c_uint64
        L.oracle_splitmix64_at.argtypes = [ct.c_uint64, ct.c_uint64]
        L.oracle_sketch.argtypes = [i64, i64, dp, ct.c_uint64, dp]
        L.oracle_group_means.argtypes = [i64, i64, i32, dp, ip, dp, lp]
        L.oracle_l_step.argtypes = [i64, i64, i32, f64, f64, dp, dp, dp, ip, dp, dp]
        L.oracle_assign.argtypes = [i64, i64, i32, dp, dp, ip]
        L.oracle_lloyd.restype = i32
        L.oracle_lloyd.argtypes = [i64, i64, i32, dp, dp, ip, i32]
        L.oracle_kmeanspp.argtypes = [i64, i64, i32, dp, ct.c_uint64, lp]
        L.oracle_kmeans.restype = i32
        L.oracle_kmeans.argtypes = [i64, i64, i32, dp, ct.c_uint64, i32, ip, dp]
        L.oracle_s_step.argtypes = [i64, i64, f64, dp, dp, dp, dp]
        L.oracle_s_step_l21.argtypes = [i64, i64, f64, dp, dp, dp, dp]
        L.oracle_theta_step.argtypes = [i64, i64, f64, dp, dp, dp, dp]
        L.oracle_column_norms.argtypes = [i64, i64, dp, dp]
        L.oracle_step.restype = i32
        L.oracle_step.argtypes = [P(Params), i64, i64, dp, dp, dp, dp, ip, dp, dp, dp]
        L.oracle_step_columns.argtypes = [P(Params), i64, i64, dp, dp, dp, ip, dp, f64, i64, lp,
                                          dp, dp, dp, ip, dp]
        L.oracle_solve.restype = i32
        L.oracle_solve.argtypes = [P(Params), i64, i64, dp, dp, dp, ip, dp, ip, P(Info), dp]
        _lib = L
    return _lib


# ----------------------------------------------------------------- marshalling

def _f64(a) -> np.ndarray:
    """Column-major float64 copy/view of a (d, n) array (FP32 inputs are upcast exactly)."""
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and (a.flags.f_contiguous or a.ndim == 1)
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _ip(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_int32))


def _lp(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_int64))


def make_params(c, lam=None, d=None, n=None, tol=1e-3, max_iter=500, rho0=1e-4, kappa=1.5,
                rho_max=1e10, max_lloyd=100, seed=0, sparse_norm=0) -> Params:
    """Defaults follow Sec. 5 (tol 1e-3, 500 iterations, rho0 1e-4, kappa 1.5) and
    lambda = sqrt(max(n, d)) (Sec. 5.1) when ``lam`` is None."""
    if lam is None:
        lam = float(np.sqrt(max(d, n)))
    return Params(float(lam), int(c), float(tol), int(max_iter), float(rho0), float(kappa),
                  float(rho_max), int(max_lloyd), int(seed) & 0xFFFFFFFFFFFFFFFF, int(sparse_norm))


def splitmix64(seed: int, count: int) -> list[int]:
    st = ct.c_uint64(seed)
    return [int(lib().oracle_splitmix64_next(ct.byref(st))) for _ in range(count)]


def uniform01(seed: int, count: int) -> list[float]:
    st = ct.c_uint64(seed)
    return [float(lib().oracle_uniform01(ct.byref(st))) for _ in range(count)]


def splitmix64_at(seed: int, t: int) -> int:
    return int(lib().oracle_splitmix64_at(seed & 0xFFFFFFFFFFFFFFFF, t))


def sketch(X, seed):
    """65 x n column sketch (64 Rademacher projections, then the column norm)."""
    X = _f64(X)
    d, n = X.shape
    Y = np.zeros((65, n), order="F")
    lib().oracle_sketch(d, n, _dp(X), int(seed) & 0xFFFFFFFFFFFFFFFF, _dp(Y))
    return Y


def group_means(Y, labels, c, mean_init=None):
    Y = _f64(Y)
    d, n = Y.shape
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    mean = _f64(np.zeros((d, c)) if mean_init is None else mean_init).copy(order="F")
    counts = np.zeros(c, dtype=np.int64)
    lib().oracle_group_means(d, n, c, _dp(Y), _ip(lab), _dp(mean), _lp(counts))
    return mean, counts


def l_step(X, S, Theta, labels, c, lam, rho, C_init=None):
    X, S, Theta = _f64(X), _f64(S), _f64(Theta)
    d, n = X.shape
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    L = np.zeros((d, n), order="F")
    C = _f64(np.zeros((d, c)) if C_init is None else C_init).copy(order="F")
    lib().oracle_l_step(d, n, c, float(lam), float(rho), _dp(X), _dp(S), _dp(Theta), _ip(lab),
                        _dp(L), _dp(C))
    return L, C


def assign(Y, C):
    Y, C = _f64(Y), _f64(C)
    d, n = Y.shape
    c = C.shape[1]
    lab = np.zeros(n, dtype=np.int32)
    lib().oracle_assign(d, n, c, _dp(Y), _dp(C), _ip(lab))
    return lab


def lloyd(Y, C, labels, max_lloyd=100):
    Y = _f64(Y)
    C = _f64(C).copy(order="F")
    d, n = Y.shape
    c = C.shape[1]
    lab = np.ascontiguousarray(labels, dtype=np.int32).copy()
    steps = lib().oracle_lloyd(d, n, c, _dp(Y), _dp(C), _ip(lab), int(max_lloyd))
    return lab, C, int(steps)


def kmeanspp(Y, c, seed):
    Y = _f64(Y)
    d, n = Y.shape
    seeds = np.zeros(c, dtype=np.int64)
    lib().oracle_kmeanspp(d, n, c, _dp(Y), int(seed) & 0xFFFFFFFFFFFFFFFF, _lp(seeds))
    return seeds


def kmeans(Y, c, seed, max_lloyd=100):
    Y = _f64(Y)
    d, n = Y.shape
    lab = np.zeros(n, dtype=np.int32)
    C = np.zeros((d, c), order="F")
    steps = lib().oracle_kmeans(d, n, c, _dp(Y), int(seed) & 0xFFFFFFFFFFFFFFFF, int(max_lloyd),
                                _ip(lab), _dp(C))
    return lab, C, int(steps)


def s_step(X, L, Theta, rho, sparse_norm=0):
    """Sec. 4.3 S-step; sparse_norm 1: its column-wise l2,1 form."""
    X, L, Theta = _f64(X), _f64(L), _f64(Theta)
    d, n = X.shape
    S = np.zeros((d, n), order="F")
    f = lib().oracle_s_step_l21 if sparse_norm == 1 else lib().oracle_s_step
    f(d, n, float(rho), _dp(X), _dp(L), _dp(Theta), _dp(S))
    return S


def column_norms(S):
    """Sec. 5.3 anomaly scores: ||S_j||_2 for every column of S."""
    S = _f64(S)
    d, n = S.shape
    out = np.zeros(n)
    lib().oracle_column_norms(d, n, _dp(S), _dp(out))
    return out


def theta_step(X, L, S, Theta, rho):
    X, L, S = _f64(X), _f64(L), _f64(S)
    T = _f64(Theta).copy(order="F")
    d, n = X.shape
    lib().oracle_theta_step(d, n, float(rho), _dp(X), _dp(L), _dp(S), _dp(T))
    return T


def step(params: Params, X, state: dict) -> dict:
    """One outer iteration.  ``state`` holds L (L_{t-1}), S, Theta, labels, C, rho;
    a new dict is returned (inputs are not modified) with ``norms`` and ``lloyd``."""
    X = _f64(X)
    d, n = X.shape
    L = _f64(state["L"]).copy(order="F")
    S = _f64(state["S"]).copy(order="F")
    T = _f64(state["Theta"]).copy(order="F")
    lab = np.ascontiguousarray(state["labels"], dtype=np.int32).copy()
    C = _f64(state["C"]).copy(order="F")
    rho = ct.c_double(float(state["rho"]))
    norms = np.zeros(3)
    steps = lib().oracle_step(ct.byref(params), d, n, _dp(X), _dp(L), _dp(S), _dp(T), _ip(lab),
                              _dp(C), ct.byref(rho), _dp(norms))
    return {"L": L, "S": S, "Theta": T, "labels": lab, "C": C, "rho": rho.value,
            "norms": norms, "lloyd": int(steps)}


def step_columns(params: Params, X, state: dict, sel):
    """One iteration (single assignment pass) evaluated only at columns ``sel``;
    group means still use every column.  Returns dict(L, S, Theta, labels) of
    shape (d, len(sel)) / (len(sel),)."""
    X = _f64(X)
    d, n = X.shape
    S, T, C = _f64(state["S"]), _f64(state["Theta"]), _f64(state["C"])
    lab = np.ascontiguousarray(state["labels"], dtype=np.int32)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    m = sel.size
    Lo, So, To = (np.zeros((d, m), order="F") for _ in range(3))
    lo = np.zeros(m, dtype=np.int32)
    mu = np.zeros((d, params.c), order="F")
    lib().oracle_step_columns(ct.byref(params), d, n, _dp(X), _dp(S), _dp(T), _ip(lab), _dp(C),
                              float(state["rho"]), m, _lp(sel), _dp(Lo), _dp(So), _dp(To), _ip(lo),
                              _dp(mu))
    return {"L": Lo, "S": So, "Theta": To, "labels": lo, "mu": mu}


def solve(X, params: Params, init_labels=None, history=False):
    """Whole RES-PCA solve.  Returns dict with L, S, labels, C, info (dict), history."""
    X = _f64(X)
    d, n = X.shape
    c = params.c
    L = np.zeros((d, n), order="F")
    S = np.zeros((d, n), order="F")
    lab = np.zeros(n, dtype=np.int32)
    C = np.zeros((d, c), order="F")
    info = Info()
    hist = np.zeros(3 * max(params.max_iter, 1)) if history else None
    il = None
    if init_labels is not None:
        il = np.ascontiguousarray(init_labels, dtype=np.int32)
    status = lib().oracle_solve(ct.byref(params), d, n, _dp(X), _dp(L), _dp(S), _ip(lab), _dp(C),
                                _ip(il) if il is not None else None, ct.byref(info),
                                _dp(hist) if hist is not None else None)
    out = {"L": L, "S": S, "labels": lab, "C": C, "info": info.as_dict(), "status": int(status)}
    if hist is not None:
        out["history"] = hist[: 3 * info.iters].reshape(-1, 3)
    return out
