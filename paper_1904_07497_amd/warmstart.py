"""Learned warm start for RES-PCA: training instances that the method generates and
solves itself, the targets taken from its solutions, the training loop, the
stored model and the cold-versus-warm evaluation.

Every piece of network arithmetic (column sketch, features, forward pass, loss,
backward pass, Adam) runs in the library's kernels; this module schedules those
calls and moves tensors.  For every column the network predicts

* the sketch of the centroid of the group that the solved problem (Sec. 4.2)
  puts the column in, in the units of the input sketch (divided by s sqrt(d)/8,
  s = ||X||_F / sqrt(d n)); K-means of these predictions gives the initial
  groups, so the k-means++ passes over X are not needed;
* log(rho0* s), the scaled initial penalty of Sec. 4.4; its mean over the
  columns gives the instance's rho0 (larger rho0 = fewer of the schedule's
  geometric steps, each a factor kappa).

rho0* of a training instance is the largest value on the grid 1e-4 * 1.5^k
whose run, started from the cold run's groups, still converges to the same
error against the planted L as the cold run (within 1 %).  The solver has the
last word: whatever the network predicts, the iterations run to tolerance.

At inference the predicted sketches are clustered (64 coordinates instead of d),
Lloyd on X refines those groups, and the iterations start from them with the
predicted rho0 (the init_embedding path of the solvers).

Instances follow the batched size mix: d, n log-uniform in [200, 4000], rank
uniform in 5..50, X = U V^T + S0 with U, V iid N(0, 1) and a fraction uniform in
[1 %, 20 %] of entries of S0 uniform in [-50, 50]; they are drawn on the GPU
from per-instance seeds (training 4_000_000 + i, held out 5_000_000 + i).
"""
from __future__ import annotations

import argparse
import math
import time
from pathlib import Path

import numpy as np

from . import respca as rp

MODEL_PATH = Path(__file__).with_name("warmstart_model.npz")
HIDDEN = 256
SKETCH_SEED = 0x5EED5EED
TRAIN_BASE, HELDOUT_BASE = 4_000_000, 5_000_000
COLD_RHO0 = 1e-4
GRID_STEP = 1.5
TOL = 1e-6


# ------------------------------------------------------------------ instances

def instance_meta(seed: int):
    """(d, n, rank, corruption fraction) of one instance of the size mix."""
    rng = np.random.default_rng(seed)
    d = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
    n = int(round(math.exp(rng.uniform(math.log(200), math.log(4000)))))
    r = int(rng.integers(5, 51))
    frac = float(rng.uniform(0.01, 0.20))
    return d, n, r, frac


def make_instance(seed: int, device="cuda"):
    """X = U V^T + S0 drawn on the device.  Returns (X, L0) as (d, n) column-major
    float32 tensors and the meta tuple."""
    import torch
    d, n, r, frac = instance_meta(seed)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    U = torch.randn(d, r, generator=g, device=device)
    V = torch.randn(n, r, generator=g, device=device)
    L0t = V @ U.T                                            # (n, d) row-major = (d, n) column-major
    mask = torch.rand(n, d, generator=g, device=device) < frac
    vals = torch.rand(n, d, generator=g, device=device) * 100.0 - 50.0
    Xt = L0t + vals * mask
    return Xt.T, L0t.T, (d, n, r, frac)


def lam_of(d, n):
    return 1.0 / math.sqrt(max(d, n))


def scale_of(X):
    """s = ||X||_F / sqrt(d n)."""
    import torch
    d, n = X.shape
    return float(torch.linalg.vector_norm(X, dtype=torch.float64)) / math.sqrt(d * n)


def rel_err(L, L0):
    import torch
    return float(torch.linalg.vector_norm(L - L0, dtype=torch.float64) /
                 torch.linalg.vector_norm(L0, dtype=torch.float64))


# --------------------------------------------------------------------- model

def init_params(hidden: int, seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, in the library's parameter layout:
    per layer W (out x in, row-major) then b (out)."""
    dims = [rp.WARM_IN, hidden, hidden, hidden, rp.WARM_OUT]
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(dims[:-1], dims[1:]):
        a = math.sqrt(6.0 / i)
        parts.append(rng.uniform(-a, a, (o, i)).astype(np.float32).ravel())
        parts.append(np.zeros(o, np.float32))
    p = np.concatenate(parts)
    assert p.size == rp.mlp_param_count(hidden)
    return p


def save_model(params, hidden, path=MODEL_PATH, meta=None):
    p = params.detach().cpu().numpy() if hasattr(params, "detach") else np.asarray(params)
    np.savez(path, params=p.astype(np.float32), hidden=np.int32(hidden),
             sketch_seed=np.uint64(SKETCH_SEED),
             meta=np.array("" if meta is None else repr(meta)))


def load_model(path=MODEL_PATH, device="cuda"):
    """(params device tensor, hidden, sketch seed) of a stored model."""
    import torch
    with np.load(path, allow_pickle=False) as z:
        p = torch.from_numpy(np.ascontiguousarray(z["params"], np.float32)).to(device)
        hidden = int(z["hidden"])
        seed = int(z["sketch_seed"])
    if p.numel() != rp.mlp_param_count(hidden):
        raise ValueError("stored model does not match its width")
    return p, hidden, seed


# ------------------------------------------------------------------- solving

def _solve(Xs, ranks, rho0=COLD_RHO0, init_labels=None, init_embeddings=None, outs=None,
           tol=TOL, embedding_refine=1):
    lams = [lam_of(*X.shape) for X in Xs]
    plist, keep = rp.batch_params(ranks, lams, tol=tol, rho0=rho0, init_labels=init_labels,
                                  init_embeddings=init_embeddings, embedding_refine=embedding_refine)
    outs, infos, _ = rp.solve_batched(Xs, plist, outs=outs)
    return outs, infos


def _outs_like(Xs):
    import torch
    return [(rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
             rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
             torch.empty(x.shape[1], dtype=torch.int32, device=x.device)) for x in Xs]


# ------------------------------------------------------------- training data

def chunk_training_data(seeds, grid=15, log=print):
    """Features and targets of the columns of the instances `seeds` (one batched
    cold solve, then one batched solve per grid value of rho0 from the cold groups).
    Returns (F (N, 68), T (N, 65), stats dict)."""
    import torch
    inst = [make_instance(s) for s in seeds]
    Xs = [x for x, _, _ in inst]
    ranks = [m[2] for _, _, m in inst]
    outs, cold = _solve(Xs, ranks)
    cold_err = [rel_err(o[0], L0) for o, (_, L0, _) in zip(outs, inst)]
    labels = [o[2].clone() for o in outs]
    best_k = [0] * len(seeds)
    best_iters = [c["iters"] for c in cold]
    work = _outs_like(Xs)
    for k in range(1, grid + 1):
        _, infos = _solve(Xs, ranks, rho0=COLD_RHO0 * GRID_STEP ** k, init_labels=labels, outs=work)
        for i, (o, inf) in enumerate(zip(work, infos)):
            if (inf["status"] == 0 and cold[i]["status"] == 0 and
                    rel_err(o[0], inst[i][1]) <= cold_err[i] * 1.01 + 1e-9):
                best_k[i] = k
                best_iters[i] = inf["iters"]
    Fs, Ts = [], []
    for i, (X, _, (d, n, r, _)) in enumerate(inst):
        s = scale_of(X)
        Fs.append(rp.features(rp.sketch(X, SKETCH_SEED), d, r))
        YL = rp.sketch(outs[i][0], SKETCH_SEED)[:, :64]
        lab = outs[i][2].long()
        M = torch.zeros(r, 64, device=X.device).index_add_(0, lab, YL)
        cnt = torch.bincount(lab, minlength=r).clamp(min=1).to(M.dtype)
        T = torch.empty(n, rp.WARM_OUT, device=X.device)
        T[:, :64] = (M / cnt[:, None])[lab] / (0.125 * s * math.sqrt(d))
        T[:, 64] = math.log(COLD_RHO0 * GRID_STEP ** best_k[i] * s)
        Ts.append(T)
    stats = {"cold_iters": [c["iters"] for c in cold], "best_iters": best_iters, "best_k": best_k,
             "cold_converged": sum(c["status"] == 0 for c in cold)}
    del inst, Xs, outs, work
    return torch.cat(Fs), torch.cat(Ts), stats


# ------------------------------------------------------------------ training

def train(F, T, hidden=HIDDEN, epochs=8, batch=4096, lr=1e-3, w_last=16.0, seed=0, val_frac=0.05,
          log=print):
    """Adam on the mean squared error (threshold output weighted by w_last) with the
    library's forward/backward/Adam kernels.  Returns (params, history)."""
    import torch
    N = F.shape[0]
    g = torch.Generator(device=F.device)
    g.manual_seed(seed)
    order = torch.randperm(N, generator=g, device=F.device)
    nval = max(1, int(N * val_frac))
    val, tr = order[:nval], order[nval:]
    P = torch.from_numpy(init_params(hidden, seed)).to(F.device)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    step, hist = 0, []

    def val_loss():
        tot = 0.0
        for b0 in range(0, nval, 65536):
            idx = val[b0:b0 + 65536]
            out, _ = rp.mlp_forward(P, hidden, F[idx].contiguous())
            lo, _ = rp.mlp_loss(out, T[idx].contiguous(), w_last)
            tot += lo * idx.numel()
        return tot / nval

    for ep in range(epochs):
        perm = tr[torch.randperm(tr.numel(), generator=g, device=F.device)]
        t0 = time.perf_counter()
        for b0 in range(0, perm.numel() - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            x = F[idx].contiguous()
            out, acts = rp.mlp_forward(P, hidden, x)
            _, dy = rp.mlp_loss(out, T[idx].contiguous(), w_last, read=False)
            grad = rp.mlp_backward(P, hidden, x, acts, dy)
            step += 1
            rp.mlp_adam(P, grad, m, v, lr * (0.5 ** (ep // 3)), step)
        vl = val_loss()
        hist.append(vl)
        log(f"epoch {ep} steps {step} val loss {vl:.5f} ({time.perf_counter() - t0:.1f}s)")
    return P, hist


# ---------------------------------------------------------------- evaluation

def evaluate(params, hidden, seeds, sketch_seed=SKETCH_SEED, chunk=256, log=print,
             groups="embedding"):
    """Cold start against the learned warm start on the instances `seeds` (batched,
    `chunk` per launch).  Solve times are of a second, timed call (graph already
    captured); the warm time includes the network pass.  groups: "embedding" starts
    from the K-means of the predicted centroid sketches, "kmeans" from the cold
    start's K-means of X (the warm start then supplies rho0 only), "seeds" from the
    K-means of X seeded by k-means++ on the predicted sketches.  Returns
    per-instance lists."""
    import torch
    res = {k: [] for k in ("cold_iters", "warm_iters", "cold_err", "warm_err", "cold_status",
                           "warm_status", "fallback", "cold_lloyd", "warm_lloyd", "cold_init_lloyd",
                           "warm_init_lloyd", "cold_steps", "warm_steps")}
    cold_s = warm_s = net_s = 0.0
    for c0 in range(0, len(seeds), chunk):
        inst = [make_instance(s) for s in seeds[c0:c0 + chunk]]
        Xs = [x for x, _, _ in inst]
        ranks = [m[2] for _, _, m in inst]
        outs = _outs_like(Xs)
        _solve(Xs, ranks, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, cold = _solve(Xs, ranks, outs=outs)
        torch.cuda.synchronize()
        cold_s += time.perf_counter() - t0
        res["cold_err"] += [rel_err(o[0], L0) for o, (_, L0, _) in zip(outs, inst)]
        res["cold_iters"] += [c["iters"] for c in cold]
        res["cold_status"] += [c["status"] for c in cold]
        res["cold_lloyd"] += [c["lloyd_steps"] for c in cold]
        res["cold_init_lloyd"] += [c["init_lloyd"] for c in cold]
        res["cold_steps"].append(rp.batched_phases()["steps"])
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            emb, rho0s, fbs = rp.warmstart_batched(Xs, ranks, params, hidden, sketch_seed)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, warm = _solve(Xs, ranks, rho0=rho0s, outs=outs,
                             init_embeddings=None if groups == "kmeans" else emb,
                             embedding_refine=2 if groups == "seeds" else 1)
            torch.cuda.synchronize()
        warm_s += time.perf_counter() - t0
        net_s += t1 - t0
        res["warm_steps"].append(rp.batched_phases()["steps"])
        res["warm_err"] += [rel_err(o[0], L0) for o, (_, L0, _) in zip(outs, inst)]
        res["warm_iters"] += [w["iters"] for w in warm]
        res["warm_status"] += [w["status"] for w in warm]
        res["warm_lloyd"] += [w["lloyd_steps"] for w in warm]
        res["warm_init_lloyd"] += [w["init_lloyd"] for w in warm]
        res["fallback"] += fbs
        log(f"evaluated {min(c0 + chunk, len(seeds))}/{len(seeds)}: cold iters "
            f"{np.mean(res['cold_iters']):.2f} warm iters {np.mean(res['warm_iters']):.2f}")
        del inst, Xs, outs
    res["cold_solves_per_s"] = len(seeds) / cold_s
    res["warm_solves_per_s"] = len(seeds) / warm_s
    res["warm_network_s"] = net_s
    return res


def summary(res):
    ce, we = np.array(res["cold_err"]), np.array(res["warm_err"])
    return {"instances": len(ce),
            "cold_iters_mean": float(np.mean(res["cold_iters"])),
            "warm_iters_mean": float(np.mean(res["warm_iters"])),
            "cold_converged": int(sum(s == 0 for s in res["cold_status"])),
            "warm_converged": int(sum(s == 0 for s in res["warm_status"])),
            "fallbacks": int(sum(res["fallback"])),
            "err_ratio_median": float(np.median(we / ce)),
            "err_ratio_max": float(np.max(we / ce)),
            "cold_lloyd_mean": float(np.mean(res["cold_lloyd"])),
            "warm_lloyd_mean": float(np.mean(res["warm_lloyd"])),
            "cold_init_lloyd_mean": float(np.mean(res["cold_init_lloyd"])),
            "warm_init_lloyd_mean": float(np.mean(res["warm_init_lloyd"])),
            "cold_steps": res["cold_steps"], "warm_steps": res["warm_steps"],
            "warm_network_s": res["warm_network_s"],
            "cold_solves_per_s": res["cold_solves_per_s"],
            "warm_solves_per_s": res["warm_solves_per_s"]}


# ----------------------------------------------------------------------- CLI

def main(argv=None):
    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--instances", type=int, default=8192, help="training instances")
    ap.add_argument("--chunk", type=int, default=256)
    ap.add_argument("--grid", type=int, default=15, help="rho0 grid values above the cold 1e-4")
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--hidden", type=int, default=HIDDEN)
    ap.add_argument("--heldout", type=int, default=1024)
    ap.add_argument("--out", default=str(MODEL_PATH))
    ap.add_argument("--eval-only", action="store_true", help="evaluate the model stored at --out")
    ap.add_argument("--curve", default=None,
                    help="comma-separated training sizes: train one model on each prefix of the "
                         "--instances generated ones and evaluate each on the held-out set "
                         "(prints one JSON line per size; --out is not written)")
    a = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    import torch
    if a.eval_only:
        P, hidden, sseed = load_model(a.out)
        res = evaluate(P, hidden, [HELDOUT_BASE + i for i in range(a.heldout)], sketch_seed=sseed,
                       chunk=a.chunk, log=log)
        log(f"held-out: {summary(res)}")
        return
    t0 = time.perf_counter()
    Fs, Ts, stats = [], [], {"cold_iters": [], "best_iters": [], "best_k": []}
    for c0 in range(0, a.instances, a.chunk):
        seeds = [TRAIN_BASE + i for i in range(c0, min(a.instances, c0 + a.chunk))]
        F, T, st = chunk_training_data(seeds, grid=a.grid, log=log)
        Fs.append(F)
        Ts.append(T)
        for k in stats:
            stats[k] += st[k]
        log(f"training data {c0 + len(seeds)}/{a.instances} instances, {sum(f.shape[0] for f in Fs)} "
            f"columns; cold iters {np.mean(stats['cold_iters']):.2f} -> best {np.mean(stats['best_iters']):.2f} "
            f"({time.perf_counter() - t0:.0f}s)")
    if a.curve:
        import json
        sizes = sorted(int(v) for v in a.curve.split(","))
        cols = np.cumsum([0] + [f.shape[0] for f in Fs])   # columns before instance chunk k
        per_chunk = a.chunk
        for size in sizes:
            k = (min(size, a.instances) + per_chunk - 1) // per_chunk
            Fk = torch.cat(Fs[:k])
            Tk = torch.cat(Ts[:k])
            Pk, hist = train(Fk, Tk, hidden=a.hidden, epochs=a.epochs, log=log)
            res = evaluate(Pk, a.hidden, [HELDOUT_BASE + i for i in range(a.heldout)], log=log)
            line = {"training_instances": min(size, a.instances), "training_columns": int(cols[k]),
                    "val_loss": [round(v, 6) for v in hist]}
            line.update(summary(res))
            print(json.dumps(line), flush=True)
            del Fk, Tk, Pk
        return
    F = torch.cat(Fs)
    T = torch.cat(Ts)
    del Fs, Ts
    P, hist = train(F, T, hidden=a.hidden, epochs=a.epochs, log=log)
    meta = {"instances": a.instances, "columns": int(F.shape[0]), "epochs": a.epochs,
            "val_loss": hist, "cold_iters_mean": float(np.mean(stats["cold_iters"])),
            "best_iters_mean": float(np.mean(stats["best_iters"])),
            "best_k_hist": np.bincount(stats["best_k"], minlength=a.grid + 1).tolist()}
    save_model(P, a.hidden, a.out, meta)
    log(f"saved {a.out}: {meta}")
    del F, T
    if a.heldout:
        res = evaluate(P, a.hidden, [HELDOUT_BASE + i for i in range(a.heldout)], log=log)
        log(f"held-out: {summary(res)}")


if __name__ == "__main__":
    main()
