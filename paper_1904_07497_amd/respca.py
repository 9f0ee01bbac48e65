"""Thin ctypes binding of librespca (include/respca.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  torch supplies device memory and streams.  A (d, n) column-major
matrix is a torch tensor of shape (d, n) whose stride is (1, ld) with ld >= d,
e.g. ``t.T`` for a contiguous (n, d) tensor ``t``.

The library must be built (``paper_1904_07497_amd.build``); there is no
fallback, so a missing or unloadable library raises at once.
"""
from __future__ import annotations

import ctypes as ct
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librespca.so")

OK, NOT_CONVERGED = 0, 1
ERR_INVALID, ERR_NONFINITE, ERR_NOMEM, ERR_HIP, ERR_UNSUPPORTED = -1, -2, -3, -4, -5
F64, F32, BF16GEMM_F32 = 0, 1, 2

# Every symbol include/respca.h declares.
EXPORTS = ("respca_create", "respca_destroy", "respca_params_default", "respca_status_string",
           "respca_last_error", "respca_version", "respca_solve", "respca_iterate",
           "respca_iterate_noalloc", "respca_spectral_embedding",
           "respca_kmeans", "respca_profile_enable", "respca_profile_query",
           "respca_solve_batched", "respca_autotune_batched", "respca_profile_batched_phases",
           "respca_set_batched_tile", "respca_get_batched_tile", "respca_bandwidth_probe",
           "respca_mlp_param_count", "respca_mlp_act_count", "respca_sketch", "respca_features",
           "respca_mlp_forward", "respca_mlp_backward", "respca_mlp_loss", "respca_mlp_adam",
           "respca_warmstart", "respca_warmstart_batched", "respca_column_norms")
WARM_IN, WARM_OUT = 68, 65
BATCH_PHASES = ("pack", "init", "seed_distance", "seed_draw", "seed_gather", "sort", "means",
                "finalize", "sweep", "distance", "argmin", "control")
KERNELS = {"sweep": 0, "means": 1, "distance": 2, "seeding": 3, "batched": 4, "colnorm": 5,
           "affinity": 6, "eigen": 7}
PSTEP_KMEANS, PSTEP_SPECTRAL = 0, 1


class Params(ct.Structure):
    _fields_ = [("lam", ct.c_double), ("rank", ct.c_int32), ("tol", ct.c_double),
                ("max_iter", ct.c_int32), ("rho0", ct.c_double), ("kappa", ct.c_double),
                ("rho_max", ct.c_double), ("max_lloyd", ct.c_int32), ("seed", ct.c_uint64),
                ("precision", ct.c_int32), ("init_labels", ct.c_void_p),
                ("history", ct.POINTER(ct.c_double)), ("init_embedding", ct.c_void_p),
                ("init_embedding_ld", ct.c_int64), ("init_embedding_rows", ct.c_int32),
                ("sparse_norm", ct.c_int32), ("pstep", ct.c_int32), ("spectral_sigma", ct.c_double),
                ("init_embedding_refine", ct.c_int32)]


class Info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("lloyd_steps", ct.c_int32), ("init_lloyd", ct.c_int32),
                ("status", ct.c_int32), ("primal", ct.c_double), ("dL", ct.c_double),
                ("dS", ct.c_double), ("rho_final", ct.c_double), ("refined", ct.c_int64),
                ("eig_iters", ct.c_int32), ("eig_unconverged", ct.c_int32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class RespcaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load librespca.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1904_07497_amd.build")
        L = ct.CDLL(LIB_PATH)
        vp, i64, i32 = ct.c_void_p, ct.c_int64, ct.c_int32
        L.respca_create.restype = i32
        L.respca_create.argtypes = [ct.POINTER(vp), i32]
        L.respca_destroy.restype = None
        L.respca_destroy.argtypes = [vp]
        L.respca_params_default.restype = None
        L.respca_params_default.argtypes = [ct.POINTER(Params)]
        L.respca_status_string.restype = ct.c_char_p
        L.respca_status_string.argtypes = [i32]
        L.respca_last_error.restype = ct.c_char_p
        L.respca_last_error.argtypes = [vp]
        L.respca_version.restype = ct.c_char_p
        L.respca_version.argtypes = []
        L.respca_solve.restype = i32
        L.respca_solve.argtypes = [vp, ct.POINTER(Params), i64, i64, vp, i64, vp, i64, vp, i64,
                                   vp, ct.POINTER(Info), vp]
        L.respca_iterate.restype = i32
        L.respca_iterate.argtypes = [vp, ct.POINTER(Params), i64, i64, vp, i64, vp, i64, vp, i64,
                                     vp, i64, vp, vp, ct.POINTER(ct.c_double), i32,
                                     ct.POINTER(ct.c_double), ct.POINTER(Info), vp]
        L.respca_spectral_embedding.restype = i32
        L.respca_spectral_embedding.argtypes = [vp, i32, i64, i64, vp, i64, i32, ct.c_double,
                                                ct.c_uint64, vp, ct.POINTER(ct.c_double),
                                                ct.POINTER(Info), vp]
        L.respca_column_norms.restype = i32
        L.respca_column_norms.argtypes = [vp, i32, i64, i64, vp, i64, vp, vp]
        L.respca_iterate_noalloc.restype = i32
        L.respca_iterate_noalloc.argtypes = L.respca_iterate.argtypes
        L.respca_profile_enable.restype = i32
        L.respca_profile_enable.argtypes = [vp, i32]
        L.respca_profile_query.restype = i32
        L.respca_profile_query.argtypes = [vp, i32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double),
                                           ct.POINTER(ct.c_double), ct.POINTER(ct.c_double)]
        arr = ct.POINTER(ct.c_void_p)
        i64p = ct.POINTER(ct.c_int64)
        L.respca_solve_batched.restype = i32
        L.respca_solve_batched.argtypes = [vp, ct.POINTER(Params), i32, i64p, i64p, arr, i64p, arr, i64p,
                                           arr, i64p, arr, ct.POINTER(Info), vp]
        L.respca_autotune_batched.restype = i32
        L.respca_autotune_batched.argtypes = [vp, ct.POINTER(Params), i32, i64p, i64p, arr, i64p, arr,
                                              i64p, arr, i64p, ct.c_char_p, ct.POINTER(ct.c_double), vp]
        L.respca_bandwidth_probe.restype = i32
        L.respca_bandwidth_probe.argtypes = [vp, i32, i32, i32, i64, i32, ct.POINTER(ct.c_double),
                                             ct.POINTER(ct.c_double), vp]
        L.respca_set_batched_tile.restype = i32
        L.respca_set_batched_tile.argtypes = [vp, i32, i32, i32]
        i32p = ct.POINTER(ct.c_int32)
        L.respca_get_batched_tile.restype = i32
        L.respca_get_batched_tile.argtypes = [vp, i32p, i32p, i32p]
        L.respca_profile_batched_phases.restype = i32
        L.respca_profile_batched_phases.argtypes = [vp, ct.POINTER(ct.c_double), i32,
                                                    ct.POINTER(ct.c_int64)]
        L.respca_mlp_param_count.restype = i64
        L.respca_mlp_param_count.argtypes = [i32]
        L.respca_mlp_act_count.restype = i64
        L.respca_mlp_act_count.argtypes = [i32, i32]
        L.respca_sketch.restype = i32
        L.respca_sketch.argtypes = [vp, i64, i64, vp, i64, ct.c_uint64, vp, vp]
        L.respca_features.restype = i32
        L.respca_features.argtypes = [vp, i64, i64, i32, vp, vp, vp]
        L.respca_mlp_forward.restype = i32
        L.respca_mlp_forward.argtypes = [vp, i32, vp, i32, vp, vp, vp]
        L.respca_mlp_backward.restype = i32
        L.respca_mlp_backward.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, vp]
        L.respca_mlp_loss.restype = i32
        L.respca_mlp_loss.argtypes = [vp, i32, vp, vp, ct.c_float, vp, ct.POINTER(ct.c_double), vp]
        L.respca_mlp_adam.restype = i32
        L.respca_mlp_adam.argtypes = [vp, i64, vp, vp, vp, vp, ct.c_float, ct.c_float, ct.c_float,
                                      ct.c_float, i32, vp]
        L.respca_warmstart.restype = i32
        L.respca_warmstart.argtypes = [vp, i32, vp, i64, i64, i32, vp, i64, ct.c_uint64, ct.c_uint64,
                                       vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int32), vp]
        L.respca_warmstart_batched.restype = i32
        L.respca_warmstart_batched.argtypes = [vp, i32, vp, i32, i64p, i64p, ct.POINTER(ct.c_int32),
                                               arr, i64p, ct.c_uint64, vp, ct.POINTER(ct.c_double),
                                               ct.POINTER(ct.c_int32), vp]
        L.respca_kmeans.restype = i32
        L.respca_kmeans.argtypes = [vp, ct.POINTER(Params), i64, i64, vp, i64, vp, vp,
                                    ct.POINTER(Info), vp]
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().respca_status_string(int(s)).decode()


def version() -> str:
    return lib().respca_version().decode()


def default_params() -> Params:
    p = Params()
    lib().respca_params_default(ct.byref(p))
    return p


def make_params(rank=0, lam=None, tol=1e-3, max_iter=500, rho0=1e-4, kappa=1.5, rho_max=1e10,
                max_lloyd=100, seed=0, precision=F32, sparse_norm=0, pstep=0, sigma=0.0) -> Params:
    p = default_params()
    p.lam = math.nan if lam is None else float(lam)
    p.rank, p.tol, p.max_iter = int(rank), float(tol), int(max_iter)
    p.rho0, p.kappa, p.rho_max = float(rho0), float(kappa), float(rho_max)
    p.max_lloyd, p.seed, p.precision = int(max_lloyd), int(seed) & (2**64 - 1), int(precision)
    p.sparse_norm = int(sparse_norm)
    p.pstep, p.spectral_sigma = int(pstep), float(sigma)
    return p


# ------------------------------------------------------------------ handles

class Handle:
    """Owns a respca_handle (device workspace) for one HIP device."""

    def __init__(self, device: int = 0):
        h = ct.c_void_p()
        s = lib().respca_create(ct.byref(h), int(device))
        if s != OK:
            raise RespcaError(s, "respca_create failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            lib().respca_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().respca_last_error(self._h).decode()

    def check(self, s: int, allow=(OK, NOT_CONVERGED)):
        if s not in allow:
            raise RespcaError(s, self.last_error())
        return s


_handles: dict = {}


def handle(device: int = 0) -> Handle:
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


# -------------------------------------------------------------- marshalling

def _colmajor(t, name):
    import torch
    if t.dim() != 2 or t.stride(0) != 1 or t.stride(1) < t.shape[0]:
        raise ValueError(f"{name} must be a (d, n) column-major tensor (stride (1, ld), ld >= d)")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    return t.data_ptr(), int(t.stride(1)) if t.shape[1] > 1 else max(int(t.stride(1)), t.shape[0])


def _dtype_precision(t, precision):
    import torch
    if precision is None:
        precision = F64 if t.dtype == torch.float64 else F32
    want = torch.float64 if precision == F64 else torch.float32
    if t.dtype != want:
        raise ValueError(f"precision {precision} needs {want}, got {t.dtype}")
    return precision


def empty_colmajor(d, n, dtype, device):
    import torch
    return torch.empty((n, d), dtype=dtype, device=device).T


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ct.c_void_p(stream.cuda_stream)


def solve(X, rank=0, lam=None, tol=1e-3, max_iter=500, rho0=1e-4, kappa=1.5, rho_max=1e10,
          max_lloyd=100, seed=0, precision=None, init_labels=None, history=False,
          out=None, stream=None, init_embedding=None, sparse_norm=0, pstep=0, sigma=0.0,
          embedding_refine=1):
    """RES-PCA of X (d x n column-major tensor).  Returns dict(L, S, labels, info[, history]).
    sparse_norm: 0 the l1 penalty on S, 1 the column-wise l2,1 penalty.  pstep:
    PSTEP_KMEANS, or PSTEP_SPECTRAL with kernel width sigma."""
    import torch
    precision = _dtype_precision(X, precision)
    d, n = X.shape
    xp, ldx = _colmajor(X, "X")
    if out is None:
        L = empty_colmajor(d, n, X.dtype, X.device)
        S = empty_colmajor(d, n, X.dtype, X.device)
        labels = torch.empty(n, dtype=torch.int32, device=X.device)
    else:
        L, S, labels = out
    lp, ldl = _colmajor(L, "L")
    sp, lds = _colmajor(S, "S")
    p = make_params(rank, lam, tol, max_iter, rho0, kappa, rho_max, max_lloyd, seed, precision,
                    sparse_norm, pstep, sigma)
    hist = None
    if history:
        hist = (ct.c_double * (3 * max_iter))()
        p.history = ct.cast(hist, ct.POINTER(ct.c_double))
    il = None
    if init_labels is not None:
        il = init_labels.to(device=X.device, dtype=torch.int32).contiguous()
        p.init_labels = il.data_ptr()
    if init_embedding is not None:
        if init_embedding.dtype != torch.float32:
            raise ValueError("init_embedding must be float32")
        ep, eld = _colmajor(init_embedding, "init_embedding")
        p.init_embedding, p.init_embedding_ld = ep, eld
        p.init_embedding_rows = init_embedding.shape[0]
        p.init_embedding_refine = int(embedding_refine)
    info = Info()
    h = handle(X.device.index or 0)
    s = lib().respca_solve(h._h, ct.byref(p), d, n, xp, ldx, lp, ldl, sp, lds, labels.data_ptr(),
                           ct.byref(info), _stream(stream))
    h.check(s)
    res = {"L": L, "S": S, "labels": labels, "info": info.as_dict(), "status": s}
    if hist is not None:
        import numpy as np
        res["history"] = np.ctypeslib.as_array(hist)[: 3 * info.iters].reshape(-1, 3).copy()
    return res


def iterate(X, state: dict, iters=1, rank=None, lam=None, max_lloyd=100, kappa=1.5, rho_max=1e10,
            precision=None, stream=None, sparse_norm=0, noalloc=False, pstep=0, sigma=0.0,
            seed=0):
    """Run ``iters`` outer iterations in place on ``state`` (device tensors L, S,
    Theta (d x n column-major), labels (int32[n]), C (d x c column-major, ld = d)
    and float rho).  Returns (norms [iters x 3], info).  noalloc: call
    respca_iterate_noalloc (workspace from the library's fixed scratch area)."""
    import numpy as np
    precision = _dtype_precision(X, precision)
    d, n = X.shape
    C = state["C"]
    c = C.shape[1] if rank is None else rank
    if C.shape != (d, c) or C.stride(0) != 1 or (c > 1 and C.stride(1) != d):
        raise ValueError("C must be a (d, c) column-major tensor with ld = d")
    xp, ldx = _colmajor(X, "X")
    lp, ldl = _colmajor(state["L"], "L")
    sp, lds = _colmajor(state["S"], "S")
    tp, ldt = _colmajor(state["Theta"], "Theta")
    p = make_params(c, lam, 0.0, max(iters, 1), 1e-4, kappa, rho_max, max_lloyd, seed, precision,
                    sparse_norm, pstep, sigma)
    rho = ct.c_double(float(state["rho"]))
    norms = (ct.c_double * (3 * max(iters, 1)))()
    info = Info()
    h = handle(X.device.index or 0)
    fn = lib().respca_iterate_noalloc if noalloc else lib().respca_iterate
    s = fn(h._h, ct.byref(p), d, n, xp, ldx, lp, ldl, sp, lds, tp, ldt,
           state["labels"].data_ptr(), C.data_ptr(), ct.byref(rho), int(iters),
           ct.cast(norms, ct.POINTER(ct.c_double)), ct.byref(info), _stream(stream))
    h.check(s)
    state["rho"] = rho.value
    return np.ctypeslib.as_array(norms)[: 3 * iters].reshape(-1, 3).copy(), info.as_dict()


def spectral_embedding(Y, rank, sigma, seed=0, precision=None, stream=None):
    """Row embedding of the spectral p-step for the columns of Y: returns (emb
    (rank x n float64, column j = unit row j of the top-rank eigenvectors),
    eigenvalues (numpy, decreasing), info)."""
    import numpy as np
    import torch
    precision = _dtype_precision(Y, precision)
    d, n = Y.shape
    yp, ldy = _colmajor(Y, "Y")
    emb = torch.empty((n, rank), dtype=torch.float64, device=Y.device).T
    vals = (ct.c_double * rank)()
    info = Info()
    h = handle(Y.device.index or 0)
    s = lib().respca_spectral_embedding(h._h, int(precision), d, n, yp, ldy, int(rank), float(sigma),
                                        int(seed) & (2**64 - 1), emb.data_ptr(),
                                        ct.cast(vals, ct.POINTER(ct.c_double)), ct.byref(info),
                                        _stream(stream))
    h.check(s, allow=(OK,))
    return emb, np.ctypeslib.as_array(vals).copy(), info.as_dict()


def column_norms(S, precision=None, stream=None):
    """Anomaly scores of Sec. 5.3: the l2 norm of every column of S (d x n,
    column-major), float64 on S's device."""
    import torch
    precision = _dtype_precision(S, precision)
    d, n = S.shape
    sp, lds = _colmajor(S, "S")
    out = torch.empty(n, dtype=torch.float64, device=S.device)
    h = handle(S.device.index or 0)
    h.check(lib().respca_column_norms(h._h, int(precision), d, n, sp, max(lds, 1), out.data_ptr(),
                                      _stream(stream)), allow=(OK,))
    return out


def kmeans(Y, rank, seed=0, max_lloyd=100, precision=None, stream=None):
    """k-means++ + Lloyd on the columns of Y.  Returns (labels, C, info)."""
    import torch
    precision = _dtype_precision(Y, precision)
    d, n = Y.shape
    yp, ldy = _colmajor(Y, "Y")
    labels = torch.empty(n, dtype=torch.int32, device=Y.device)
    C = empty_colmajor(d, rank, Y.dtype, Y.device)
    p = make_params(rank, 1.0, 1e-3, 1, 1e-4, 1.5, 1e10, max_lloyd, seed, precision)
    info = Info()
    h = handle(Y.device.index or 0)
    s = lib().respca_kmeans(h._h, ct.byref(p), d, n, yp, ldy, labels.data_ptr(), C.data_ptr(),
                            ct.byref(info), _stream(stream))
    h.check(s)
    return labels, C, info.as_dict()


def profile_enable(on: bool = True, units=None, device: int = 0):
    """Turn the library's per-kernel event timing on/off (resets the counters).
    units: names from KERNELS to time (default: all of them)."""
    h = handle(device)
    mask = 0 if not on else (-1 if units is None else sum(1 << KERNELS[u] for u in set(units)))
    h.check(lib().respca_profile_enable(h._h, mask), allow=(OK,))


def profile_query(device: int = 0) -> dict:
    """{kernel: {"launches", "ms", "bytes", "flops"}} accumulated since profile_enable."""
    h = handle(device)
    out = {}
    for name, kid in KERNELS.items():
        n, ms, by, fl = ct.c_int64(), ct.c_double(), ct.c_double(), ct.c_double()
        h.check(lib().respca_profile_query(h._h, kid, ct.byref(n), ct.byref(ms), ct.byref(by),
                                           ct.byref(fl)), allow=(OK,))
        out[name] = {"launches": n.value, "ms": ms.value, "bytes": by.value, "flops": fl.value}
    return out


# ------------------------------------------------------------------ batched

def _batch_args(Xs, params_list, outs):
    import torch
    b = len(Xs)
    P = (Params * b)(*params_list)
    d = (ct.c_int64 * b)(*[x.shape[0] for x in Xs])
    n = (ct.c_int64 * b)(*[x.shape[1] for x in Xs])
    def ptrs(ts, name):
        vals, lds = [], []
        for t in ts:
            p, ld = _colmajor(t, name)
            if t.dtype != torch.float32:
                raise ValueError(f"{name} must be float32")
            vals.append(p)
            lds.append(ld)
        return (ct.c_void_p * b)(*vals), (ct.c_int64 * b)(*lds)
    Xp, ldx = ptrs(Xs, "X")
    Lp, ldl = ptrs([o[0] for o in outs], "L")
    Sp, lds = ptrs([o[1] for o in outs], "S")
    Lab = (ct.c_void_p * b)(*[o[2].data_ptr() for o in outs])
    return b, P, d, n, Xp, ldx, Lp, ldl, Sp, lds, Lab


def batch_params(ranks, lams=None, tol=1e-6, max_iter=500, rho0=1e-4, kappa=1.5, rho_max=1e10,
                 max_lloyd=100, seeds=None, init_labels=None, init_embeddings=None,
                 embedding_refine=1):
    """Per-instance Params (FP32).  ``rho0`` may be a scalar or a per-instance list;
    ``init_labels`` a list of device int32 tensors or None entries; ``init_embeddings``
    a list of (rows, n) column-major float32 device tensors or None entries."""
    import torch
    b = len(ranks)
    out, keep = [], []
    for i in range(b):
        r0 = rho0[i] if isinstance(rho0, (list, tuple)) else rho0
        p = make_params(ranks[i], None if lams is None else lams[i], tol, max_iter, r0, kappa,
                        rho_max, max_lloyd, 0 if seeds is None else seeds[i], F32)
        if init_labels is not None and init_labels[i] is not None:
            p.init_labels = init_labels[i].data_ptr()
            keep.append(init_labels[i])
        if init_embeddings is not None and init_embeddings[i] is not None:
            e = init_embeddings[i]
            if e.dtype != torch.float32:
                raise ValueError("init_embedding must be float32")
            ep, eld = _colmajor(e, "init_embedding")
            p.init_embedding, p.init_embedding_ld, p.init_embedding_rows = ep, eld, e.shape[0]
            p.init_embedding_refine = int(embedding_refine)
            keep.append(e)
        out.append(p)
    return out, keep


def solve_batched(Xs, params_list, outs=None, stream=None, device=0):
    """Solve many instances in one persistent launch.  Xs: list of (d, n) float32
    column-major device tensors; params_list: from batch_params.  Returns
    (outs [(L, S, labels)], infos [dict], status)."""
    import torch
    if outs is None:
        outs = [(empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 torch.empty(x.shape[1], dtype=torch.int32, device=x.device)) for x in Xs]
    b, P, d, n, Xp, ldx, Lp, ldl, Sp, lds, Lab = _batch_args(Xs, params_list, outs)
    info = (Info * b)()
    h = handle(device)
    s = lib().respca_solve_batched(h._h, P, b, d, n, Xp, ldx, Lp, ldl, Sp, lds, Lab, info,
                                   _stream(stream))
    h.check(s)
    return outs, [info[i].as_dict() for i in range(b)], s


def autotune_batched(Xs, params_list, cache_path=None, outs=None, stream=None, device=0):
    """Run the batched tile-shape tuner (result kept in the handle); returns best ms."""
    import torch
    if outs is None:
        outs = [(empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 torch.empty(x.shape[1], dtype=torch.int32, device=x.device)) for x in Xs]
    b, P, d, n, Xp, ldx, Lp, ldl, Sp, lds, _ = _batch_args(Xs, params_list, outs)
    best = ct.c_double(0.0)
    h = handle(device)
    s = lib().respca_autotune_batched(h._h, P, b, d, n, Xp, ldx, Lp, ldl, Sp, lds,
                                      cache_path.encode() if cache_path else None, ct.byref(best),
                                      _stream(stream))
    h.check(s, allow=(OK,))
    return best.value


def set_batched_tile(jc: int, slice_rows: int, blocks_per_cu: int, device: int = 0):
    """Set the batched solver's tile shape (one of the tuner's candidates)."""
    h = handle(device)
    h.check(lib().respca_set_batched_tile(h._h, int(jc), int(slice_rows), int(blocks_per_cu)))


def get_batched_tile(device: int = 0) -> tuple:
    """The batched solver's current tile shape (jc, slice_rows, blocks_per_cu)."""
    h = handle(device)
    a, b, c = ct.c_int32(), ct.c_int32(), ct.c_int32()
    h.check(lib().respca_get_batched_tile(h._h, ct.byref(a), ct.byref(b), ct.byref(c)))
    return a.value, b.value, c.value


def bandwidth_probe(reads: int, writes: int, bytes_per_array: int, reps: int = 10,
                    stream=None, device: int = 0, nontemporal: bool = False) -> tuple:
    """Streaming probe of a read/write mix; returns (GB/s, ms per launch)."""
    h = handle(device)
    g, ms = ct.c_double(0.0), ct.c_double(0.0)
    h.check(lib().respca_bandwidth_probe(h._h, int(reads), int(writes), int(bool(nontemporal)),
                                         int(bytes_per_array), int(reps), ct.byref(g), ct.byref(ms),
                                         _stream(stream)))
    return g.value, ms.value


def batched_phases(device: int = 0) -> dict:
    """Per-phase milliseconds (and step count) of the last batched launch."""
    h = handle(device)
    ms = (ct.c_double * len(BATCH_PHASES))()
    steps = ct.c_int64()
    h.check(lib().respca_profile_batched_phases(h._h, ms, len(BATCH_PHASES), ct.byref(steps)),
            allow=(OK,))
    out = {k: round(ms[i], 3) for i, k in enumerate(BATCH_PHASES)}
    out["steps"] = steps.value
    return out


# ------------------------------------------------------------- warm start

def mlp_param_count(hidden: int) -> int:
    return int(lib().respca_mlp_param_count(hidden))


def mlp_act_count(hidden: int, batch: int) -> int:
    return int(lib().respca_mlp_act_count(hidden, batch))


def sketch(X, seed=0, stream=None):
    """65 x n float32 sketch (returned as an (n, 65) row-major tensor)."""
    import torch
    d, n = X.shape
    xp, ldx = _colmajor(X, "X")
    Y = torch.empty((n, 65), dtype=torch.float32, device=X.device)
    h = handle(X.device.index or 0)
    h.check(lib().respca_sketch(h._h, d, n, xp, ldx, int(seed) & (2**64 - 1), Y.data_ptr(),
                                _stream(stream)), allow=(OK,))
    return Y


def features(Y, d, c, stream=None):
    """(n, 68) network inputs from an (n, 65) sketch of a d x n matrix with c groups."""
    import torch
    n = Y.shape[0]
    F = torch.empty((n, WARM_IN), dtype=torch.float32, device=Y.device)
    h = handle(Y.device.index or 0)
    h.check(lib().respca_features(h._h, d, n, c, Y.data_ptr(), F.data_ptr(), _stream(stream)),
            allow=(OK,))
    return F


def mlp_forward(params, hidden, x, stream=None):
    """Returns (output (B, 65) view, acts buffer)."""
    import torch
    B = x.shape[0]
    acts = torch.empty(mlp_act_count(hidden, B), dtype=torch.float32, device=x.device)
    h = handle(x.device.index or 0)
    h.check(lib().respca_mlp_forward(h._h, hidden, params.data_ptr(), B, x.data_ptr(),
                                     acts.data_ptr(), _stream(stream)), allow=(OK,))
    return acts[3 * B * hidden:].view(B, WARM_OUT), acts


def mlp_backward(params, hidden, x, acts, dy, stream=None):
    import torch
    grad = torch.empty_like(params)
    h = handle(x.device.index or 0)
    h.check(lib().respca_mlp_backward(h._h, hidden, params.data_ptr(), x.shape[0], x.data_ptr(),
                                      acts.data_ptr(), dy.data_ptr(), grad.data_ptr(),
                                      _stream(stream)), allow=(OK,))
    return grad


def mlp_loss(y, t, w_last, stream=None, read=True):
    """(loss, dy); with read=False the loss is not read back (no host synchronisation)
    and None is returned in its place."""
    import torch
    dy = torch.empty_like(y)
    loss = ct.c_double()
    h = handle(y.device.index or 0)
    h.check(lib().respca_mlp_loss(h._h, y.shape[0], y.data_ptr(), t.data_ptr(), float(w_last),
                                  dy.data_ptr(), ct.byref(loss) if read else None, _stream(stream)),
            allow=(OK,))
    return (loss.value if read else None), dy


def mlp_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    h = handle(params.device.index or 0)
    h.check(lib().respca_mlp_adam(h._h, params.numel(), params.data_ptr(), grad.data_ptr(),
                                  m.data_ptr(), v.data_ptr(), float(lr), float(beta1), float(beta2),
                                  float(eps), int(step), _stream(stream)), allow=(OK,))


def warmstart(X, rank, params, hidden, sketch_seed=0, kmeans_seed=0, stream=None):
    """Initial labels (device int32[n]), rho0 and the fallback flag for X."""
    import torch
    d, n = X.shape
    xp, ldx = _colmajor(X, "X")
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    rho0 = ct.c_double()
    fb = ct.c_int32()
    h = handle(X.device.index or 0)
    h.check(lib().respca_warmstart(h._h, hidden, params.data_ptr(), d, n, rank, xp, ldx,
                                   int(sketch_seed) & (2**64 - 1), int(kmeans_seed) & (2**64 - 1),
                                   labels.data_ptr(), ct.byref(rho0), ct.byref(fb), _stream(stream)),
            allow=(OK,))
    return labels, rho0.value, bool(fb.value)


def warmstart_batched(Xs, ranks, params, hidden, sketch_seed=0, stream=None):
    """Warm start of a batch: returns (embeddings, rho0s, fallbacks) where embeddings[i]
    is the (64, n_i) column-major view (leading dimension 65) of the predicted centroid
    sketches of instance i, ready for ``init_embeddings``."""
    import torch
    b = len(Xs)
    dev = Xs[0].device
    ns = [int(X.shape[1]) for X in Xs]
    ptrs, lds = [], []
    for X in Xs:
        if X.dtype != torch.float32:
            raise ValueError("warm start needs float32 instances")
        p, ld = _colmajor(X, "X")
        ptrs.append(p)
        lds.append(ld)
    emb = torch.empty(sum(ns), WARM_OUT, dtype=torch.float32, device=dev)
    rho0 = (ct.c_double * b)()
    fb = (ct.c_int32 * b)()
    h = handle(dev.index or 0)
    h.check(lib().respca_warmstart_batched(
        h._h, hidden, params.data_ptr(), b, (ct.c_int64 * b)(*[int(X.shape[0]) for X in Xs]),
        (ct.c_int64 * b)(*ns), (ct.c_int32 * b)(*[int(r) for r in ranks]),
        (ct.c_void_p * b)(*ptrs), (ct.c_int64 * b)(*lds), int(sketch_seed) & (2**64 - 1),
        emb.data_ptr(), rho0, fb, _stream(stream)), allow=(OK,))
    views, off = [], 0
    for n in ns:
        views.append(emb[off:off + n, :WARM_OUT - 1].t())
        off += n
    return views, list(rho0), [bool(x) for x in fb]
