"""RES-PCA solves/s on one MI355X, with the sweep's HBM roofline and the FP64
CPU checker timed beside it.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload large]
                    [--precision bf16|fp32] [--no-compare] [--no-cpu-baseline]
                    [--tune-cache FILE] [--calibrate-copy] [--calibrate-mix] [--no-accuracy]
    python bench.py --workload small          (500 x 500 FP64, compared with the oracle)
    python bench.py --summarize-counters UNIT WORKLOAD ROOT   (no GPU)

A step is one whole RES-PCA solve (initial K-means of X, then outer ALM
iterations L -> p -> S -> Theta/rho until the Sec. 5 criterion <= tol) of
one synthetic input that is already resident in HBM.  The default workload is
10^4 x 10^4 FP32: X = U V^T (rank 100, U, V iid N(0, 1)) plus 10 % of entries
uniform in [-100, 100], c = 100 groups, lambda = 0.01, tol = 1e-6.

One JSON line is printed.  `roofline` describes the dominant kernel (the
single-kernel unit with the largest summed event time: the sweep), with
achieved = algorithmic bytes per launch / mean launch time, both measured live
by the library's event timing on the launch stream over the timed region;
`assignment_stage_roofline` gives the same figure for the assignment pass, a
chain of kernels.  `traffic` comes from the rocprofv3
counter summary committed under profiles/ when it was taken on the current
kernel source, else null.  `cpu_baseline` times the FP64 CPU checker on a
bounded sample of the same workload and scales it to solves/s (see `sample`).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STREAM_NT_BYTES = 64 * 1024 * 1024   # arrays the library streams nontemporally (per array)
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # dense, per MI355X

WORKLOADS = {
    "large": dict(name="RES-PCA FP32 10000x10000 rank-100 + 10% sparse in [-100,100], c=100 (true "
                       "rank given), lambda=0.01, tol=1e-6", d=10000, n=10000, rank=100, lam=0.01,
                  tol=1e-6, gen="large"),
    "large_c5": dict(name="RES-PCA FP32 10000x10000 rank-100 + 10% sparse in [-100,100], c=5 (rank "
                          "withheld), lambda=0.01, tol=1e-6", d=10000, n=10000, rank=5, lam=0.01,
                     tol=1e-6, gen="large"),
    "batched": dict(name="RES-PCA FP32 batch of 256 instances: d, n log-uniform in [200, 4000], rank "
                         "uniform in 5..50, 1-20% sparse in [-50,50], c=rank, lambda=1/sqrt(max(d,n)), "
                         "tol=1e-6; one persistent launch replayed from a hipGraph", batch=256,
                    tol=1e-6, gen="batched"),
    "warmstart": dict(name="learned warm start vs cold start, RES-PCA FP32: 1024 held-out instances "
                           "of the batched size mix (d, n log-uniform in [200, 4000], rank 5..50, "
                           "1-20% sparse in [-50,50]) drawn on the device, c=rank, "
                           "lambda=1/sqrt(max(d,n)), tol=1e-6; launches of 256 instances, network "
                           "pass included; warm runs start from the predicted rho0 and the K-means "
                           "of X seeded by k-means++ on the predicted centroid sketches",
                      instances=1024, chunk=256, tol=1e-6, gen="warmstart"),
    "video": dict(name="RES-PCA FP32 synthetic 240x320x2000 clip (rank-5 background, 4 moving 20x20 "
                       "squares, 8-bit scale), c=5, lambda=sqrt(76800), tol=1e-6", d=76800, n=2000,
                  rank=5, lam=None, tol=1e-6, gen="video"),
    "large_lloyd1": dict(name="RES-PCA FP32 10000x10000 rank-100 + 10% sparse in [-100,100], c=100, "
                              "lambda=0.01, tol=1e-6, p-step = one Lloyd assignment per outer "
                              "iteration (instead of K-means to convergence)", d=10000, n=10000,
                         rank=100, lam=0.01, tol=1e-6, gen="large", max_lloyd=1),
    "large_l21": dict(name="RES-PCA FP32 10000x10000 rank-100 + 10% sparse in [-100,100], c=100, "
                           "lambda=0.01, tol=1e-6, column-wise l2,1 penalty on S (the alternative "
                           "norm of Sec. 3) in place of l1", d=10000, n=10000, rank=100, lam=0.01,
                      tol=1e-6, gen="large", sparse_norm=1),
    "small": dict(name="RES-PCA FP64 500x500 rank-25 (U, V iid N(0,1)) + 5% sparse in [-50,50], c=25, "
                       "lambda=1/sqrt(500), tol=1e-7; seeds 0-4, each solve compared with the FP64 "
                       "oracle's whole solve", d=500, n=500, rank=25, lam=1.0 / 500 ** 0.5, tol=1e-7,
                  seeds=(0, 1, 2, 3, 4), gen="small"),
    "spectral": dict(name="RES-PCA FP32 with the spectral-clustering p-step (Sec. 4.2 nonlinear "
                          "alternative): two interleaved half circles (two moons, 4000 points each) in "
                          "a random plane of R^2000, N(0, 0.001^2) noise, 0.02% of entries offset by "
                          "U[-0.3, 0.3], c=2, kernel width 0.1 x the columns' spread (relative), "
                          "lambda=0.05, tol=1e-6", d=2000, counts=(4000, 4000), noise=0.001,
                     frac=0.0002, amp=0.3, rank=2, sigma=-0.1, lam=0.05, tol=1e-6, gen="spectral"),
    "scaling": dict(name="scalability (Sec. 5): seeded random subsets of the synthetic 240x320x2000 "
                         "clip at ratios 1/8, 1/4, 1/2, 1 of n (all d) and of d (all n), c=5, "
                         "lambda=sqrt(max(d,n)), 30 outer iterations (no tolerance), 10 runs each",
                    d=76800, n=2000, rank=5, iters=30, runs=10, ratios=(0.125, 0.25, 0.5, 1.0),
                    gen="scaling"),
}


# source files whose kernels make up each profiled unit
KERNEL_SOURCES = {
    "sweep": ("kernels.hip", "kernels.h", "device_common.h"),
    "means": ("kernels.hip", "kernels.h", "device_common.h"),
    "seeding": ("kernels.hip", "kernels.h", "device_common.h"),
    "distance": ("distance.hip", "dist_tile.h", "kernels.hip", "kernels.h", "device_common.h"),
    "batched": ("batched.hip", "batched.h", "dist_tile.h", "device_common.h", "kernels.h"),
    "colnorm": ("kernels.hip", "kernels.h", "device_common.h"),
    "affinity": ("spectral.hip", "spectral.h"),
    "eigen": ("spectral.hip", "spectral.h"),
}


def kernel_source_sha(kernel: str) -> str:
    """Hash of the source files of one profiled unit (a counter summary is used only
    if it was taken on exactly this source)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1904_07497_amd", "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """Per-launch HBM bytes (fetch + write, each scaled by the copy-kernel factor)
    from the committed counter summary, only if taken on the current source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != kernel_source_sha(kernel):
        return None
    return rec.get("bytes_per_launch")


def make_input(wl, dtype):
    import numpy as np
    from paper_1904_07497_amd import synth
    if wl["gen"] == "large":
        X, _, _ = synth.config_large(1, np.float32, d=wl["d"], n=wl["n"])
    else:
        X, _, _ = synth.video(n=wl["n"], seed=2, dtype=np.float32)
    return X


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cores() -> int:
    """CPU cores this process may run on (the oracle itself is single-threaded)."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def timed_oracle_solve(X64, c, lam, tol, seed=0):
    """One whole FP64 oracle solve, timed (one thread)."""
    import oracle
    t = time.perf_counter()
    o = oracle.solve(X64, oracle.make_params(c, lam=lam, tol=tol, seed=seed))
    return {"seconds": round(time.perf_counter() - t, 3), "iters": o["info"]["iters"],
            "shape": list(X64.shape), "c": c}


def accuracy_vs_oracle(rp, Xd, X, wl, prec, T, final_L, sample=64, seed=0):
    """Error of the solve's last iteration against the FP64 oracle: the GPU
    trajectory is replayed to iterate T-1 (respca_kmeans + respca_iterate, the
    same kernels in the same order as respca_solve), the oracle then takes the
    last iteration from that state at `sample` seeded columns (group means over
    every column, then per column L, S, Theta) and the GPU its last iteration;
    relative Frobenius errors over the sampled columns, labels compared where
    the oracle's nearest and second-nearest centroid distances are clear of the
    FP32 rounding of the distance computation."""
    import numpy as np
    import torch
    import oracle
    d, n = X.shape
    c = wl["rank"]
    labels, C, _ = rp.kmeans(Xd, c, seed=seed, max_lloyd=100, precision=prec)
    st = {"L": rp.empty_colmajor(d, n, Xd.dtype, Xd.device).zero_(),
          "S": rp.empty_colmajor(d, n, Xd.dtype, Xd.device).zero_(),
          "Theta": rp.empty_colmajor(d, n, Xd.dtype, Xd.device).zero_(),
          "labels": labels, "C": C, "rho": 1e-4}
    if T > 1:
        rp.iterate(Xd, st, iters=T - 1, lam=wl["lam"], max_lloyd=100, precision=prec,
                   sparse_norm=wl.get("sparse_norm", 0))
    host = {k: (np.asfortranarray(v.cpu().numpy().astype(np.float64)) if torch.is_tensor(v)
                and v.dtype != torch.int32 else (v.cpu().numpy() if torch.is_tensor(v) else v))
            for k, v in st.items()}
    rho_t = st["rho"]
    rp.iterate(Xd, st, iters=1, lam=wl["lam"], max_lloyd=1, precision=prec,
               sparse_norm=wl.get("sparse_norm", 0))
    replay_diff = float(torch.linalg.norm(st["L"].double() - final_L.double()) /
                        torch.linalg.norm(final_L.double()))
    rng = np.random.default_rng(seed)
    sel = np.unique(np.concatenate([[0, n - 1], rng.choice(n, sample - 2, replace=False)]))
    t = time.perf_counter()
    o = oracle.step_columns(oracle.make_params(c, lam=wl["lam"], d=X.shape[0], n=X.shape[1],
                                               max_lloyd=1, sparse_norm=wl.get("sparse_norm", 0)),
                            np.asfortranarray(X.astype(np.float64)), host, sel)
    t_or = time.perf_counter() - t
    idx = torch.from_numpy(sel).to(Xd.device)

    def rel(g, ref):
        g = np.asarray(g.index_select(1, idx).double().cpu().numpy())
        den = np.linalg.norm(ref)
        return float(np.linalg.norm(g - ref) / (den if den > 0 else 1.0))

    mu = o["mu"]
    dist = ((o["L"][:, :, None] - mu[:, None, :]) ** 2).sum(axis=0)
    srt = np.sort(dist, axis=1)
    cn = np.sqrt((mu ** 2).sum(axis=0)).max()
    ln = np.sqrt((o["L"] ** 2).sum(axis=0))
    sep = (srt[:, 1] - srt[:, 0]) > 2 * d * np.finfo(np.float32).eps * (cn ** 2 + 2 * cn * ln + ln ** 2)
    lab = st["labels"].cpu().numpy()[sel]
    Xsel = X[:, sel].astype(np.float64)
    dth = st["Theta"].index_select(1, idx).double().cpu().numpy() / rho_t - o["Theta"] / rho_t
    return {"rel_err_L": rel(st["L"], o["L"]), "rel_err_S": rel(st["S"], o["S"]),
            "err_Theta_over_rho_vs_X": float(np.linalg.norm(dth) / np.linalg.norm(Xsel)),
            "labels_equal_on_separated": int((lab == o["labels"])[sep].sum()),
            "separated_columns": int(sep.sum()), "columns": int(sel.size),
            "replayed_L_vs_timed_solve": replay_diff, "oracle_seconds": round(t_or, 2),
            "how": (f"last iteration ({T}) of the timed solve's trajectory, replayed on the GPU to "
                    f"iterate {T - 1}; the FP64 oracle takes iteration {T} from that state at "
                    f"{sel.size} seeded columns (group means over all columns)")}


def cpu_baseline(X, wl, gpu_info):
    """Time the FP64 CPU checker on one outer iteration of the same workload and
    scale to one whole solve with the iteration / pass counts of the GPU solve."""
    import numpy as np
    import oracle
    d, n = X.shape
    c = wl["rank"]
    lam = wl["lam"] if wl["lam"] is not None else float(np.sqrt(max(d, n)))
    X64 = np.asfortranarray(X.astype(np.float64))
    rng = np.random.default_rng(0)
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.zeros((d, n), order="F"), "labels": rng.integers(0, c, n).astype(np.int32),
          "C": np.zeros((d, c), order="F"), "rho": 1e-4}
    p = oracle.make_params(c, lam=lam, max_lloyd=1, sparse_norm=wl.get("sparse_norm", 0))
    t = time.perf_counter()
    o = oracle.step(p, X64, st)                      # L-step + one assignment + S + Theta
    t_step = time.perf_counter() - t
    t = time.perf_counter()
    lab = oracle.assign(o["L"], o["C"])              # one extra Lloyd assignment pass
    t_assign = time.perf_counter() - t
    t = time.perf_counter()
    oracle.group_means(o["L"], lab, c)               # one Lloyd centroid pass
    t_mean = time.perf_counter() - t
    t = time.perf_counter()
    oracle.kmeanspp(X64, 2, 0)                       # two k-means++ distance passes
    t_d2 = (time.perf_counter() - t) / 2
    it, ll, il = gpu_info["iters"], gpu_info["lloyd_steps"], gpu_info["init_lloyd"]
    t_solve = (c * t_d2 + (il + 1) * (t_assign + t_mean) + it * t_step
               + (ll - it) * (t_assign + t_mean))
    sample = (f"one FP64 outer iteration (L-step, one assignment pass, S-step, Theta update) of the "
              f"same {d}x{n} c={c} input ({t_step:.2f} s), one assignment pass ({t_assign:.2f} s), "
              f"one centroid pass ({t_mean:.2f} s), one k-means++ distance pass ({t_d2:.3f} s); "
              f"solve time = {c}*seed pass + {il + 1} init assignment+centroid passes + {it} "
              f"iterations + {ll - it} extra Lloyd passes (counts of the GPU solve) = {t_solve:.1f} s")
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": sample, "host_cores_available": host_cores()}


def batched_cpu_baseline(Xh_median, c_median, lam_median, shapes, ranks, infos, count):
    """FP64 oracle on the median instance, scaled per instance by its size and the
    GPU run's pass counts; returns the cpu_baseline object for `count` solves."""
    import numpy as np
    import oracle
    X64 = np.asfortranarray(Xh_median.astype(np.float64))
    d, n = X64.shape
    c = c_median
    rng = np.random.default_rng(0)
    st = {"L": np.zeros((d, n), order="F"), "S": np.zeros((d, n), order="F"),
          "Theta": np.zeros((d, n), order="F"), "labels": rng.integers(0, c, n).astype(np.int32),
          "C": np.zeros((d, c), order="F"), "rho": 1e-4}
    t = time.perf_counter(); o = oracle.step(oracle.make_params(c, lam=lam_median, max_lloyd=1), X64, st)
    t_step = time.perf_counter() - t
    t = time.perf_counter(); lab = oracle.assign(o["L"], o["C"]); t_assign = time.perf_counter() - t
    t = time.perf_counter(); oracle.group_means(o["L"], lab, c); t_mean = time.perf_counter() - t
    t = time.perf_counter(); oracle.kmeanspp(X64, 2, 0); t_d2 = (time.perf_counter() - t) / 2
    base = t_step - t_assign
    total = 0.0
    for (di, ni), ci, f in zip(shapes, ranks, infos):
        sz = di * ni / (d * n)
        ta = t_assign * sz * ci / c
        tm, tb, td = t_mean * sz, base * sz, t_d2 * sz
        total += (ci * td + (f["init_lloyd"] + 1) * (ta + tm) + f["iters"] * (tb + ta)
                  + (f["lloyd_steps"] - f["iters"]) * (ta + tm))
    return {"value": count / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "host_cores_available": host_cores(),
            "median_instance_whole_solve": timed_oracle_solve(X64, c, lam_median, 1e-6),
            "sample": (f"FP64 oracle on the median instance ({d}x{n}, c={c}): one outer iteration "
                       f"{t_step:.3f} s, one assignment pass {t_assign:.3f} s, one centroid pass "
                       f"{t_mean:.4f} s, one k-means++ distance pass {t_d2:.4f} s; every instance's "
                       f"solve time = these costs scaled by its d*n (and c for assignments) times the "
                       f"pass counts of its cold GPU solve (seeding, initial Lloyd, iterations, Lloyd); "
                       f"total {total:.1f} s for {count} solves")}


def batched_roofline(prof, workload):
    nl = max(prof["launches"], 1)
    secs = prof["ms"] / 1e3 / nl
    bpl = prof["bytes"] / nl
    ach = bpl / secs / 1e9 if secs > 0 else 0.0
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic("batched", workload),
            "kernel": "batched (persistent launch)", "bytes_per_launch": bpl,
            "mean_launch_ms": round(secs * 1e3, 3)}


def tune(rp, Xs, plist, outs, cache):
    t = time.perf_counter()
    ms = rp.autotune_batched(Xs, plist, cache_path=cache, outs=outs)
    return ms, time.perf_counter() - t


def bench_batched(args, wl):
    """256 uneven instances per step, one persistent launch (graph replay)."""
    import numpy as np
    import torch

    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import synth

    Xh, Xs, ranks, lams = [], [], [], []
    for i in range(wl["batch"]):
        X, r, meta = synth.batch_instance(i)
        Xh.append(X)
        Xs.append(torch.from_numpy(X).to("cuda:0"))
        ranks.append(r)
        lams.append(1.0 / np.sqrt(max(meta["d"], meta["n"])))
    plist, _ = rp.batch_params(ranks, lams, tol=wl["tol"])
    outs = [(rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
             rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
             torch.empty(x.shape[1], dtype=torch.int32, device=x.device)) for x in Xs]
    tuned_ms, tune_s = tune(rp, Xs, plist, outs, args.tune_cache)
    for _ in range(max(args.warmup, 1)):
        _, infos, _ = rp.solve_batched(Xs, plist, outs=outs)
    torch.cuda.synchronize()
    rp.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, infos, status = rp.solve_batched(Xs, plist, outs=outs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = rp.profile_query()["batched"]
    rp.profile_enable(False)
    phases = rp.batched_phases()
    elapsed = t1 - t0
    iters = [f["iters"] for f in infos]
    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(wl["batch"] * args.steps / elapsed, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "batch": wl["batch"],
                   "sum_dn": int(sum(x.shape[0] * x.shape[1] for x in Xs)),
                   "iters_min_median_max": [min(iters), int(np.median(iters)), max(iters)],
                   "all_converged": all(f["status"] == 0 for f in infos),
                   "tuner_seconds": round(tune_s, 2), "tuned_launch_ms": round(tuned_ms, 3)},
        "roofline": batched_roofline(prof, "batched"),
        "phases_ms": phases,
    }
    if not args.no_compare:
        # the plain FP32 method one instance at a time (same parameters) on the first
        # 64 instances of the mix, for the batching gain
        m = min(64, len(Xs))
        for i in range(2):
            rp.solve(Xs[i], rank=ranks[i], lam=lams[i], tol=wl["tol"], precision=rp.F32)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(m):
            rp.solve(Xs[i], rank=ranks[i], lam=lams[i], tol=wl["tol"], precision=rp.F32)
        torch.cuda.synchronize()
        line["sequential_fp32_solves_per_s"] = round(m / (time.perf_counter() - t0), 2)
        line["sequential_sample"] = f"first {m} instances of the batch, one respca_solve each"
    if not args.no_cpu_baseline:
        dn = [x.shape[0] * x.shape[1] for x in Xh]
        im = int(np.argsort(dn)[len(dn) // 2])
        line["cpu_baseline"] = batched_cpu_baseline(Xh[im], ranks[im], lams[im],
                                                    [x.shape for x in Xh], ranks, infos, wl["batch"])
    print(json.dumps(line), flush=True)


def bench_warmstart(args, wl):
    """Held-out instances solved from the learned warm start (network pass, then
    the batched solver from the predicted rho0, with the groups of the K-means of X
    seeded on the predicted centroid sketches; --warm-groups kmeans: the cold
    start's K-means of X; embedding: the K-means of the sketches themselves) against
    the cold start on the same instances; a step is one pass over all of them."""
    import numpy as np
    import torch

    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import warmstart as ws

    P, hidden, sseed = ws.load_model()
    inst = [ws.make_instance(ws.HELDOUT_BASE + i) for i in range(wl["instances"])]
    chunk = wl["chunk"]
    chunks = []
    for c0 in range(0, len(inst), chunk):
        part = inst[c0:c0 + chunk]
        Xs = [x for x, _, _ in part]
        ranks = [m[2] for _, _, m in part]
        lams = [ws.lam_of(*x.shape) for x in Xs]
        outs = [(rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 rp.empty_colmajor(x.shape[0], x.shape[1], x.dtype, x.device),
                 torch.empty(x.shape[1], dtype=torch.int32, device=x.device)) for x in Xs]
        chunks.append((Xs, ranks, lams, outs))
    cold_p = [rp.batch_params(r, l, tol=wl["tol"])[0] for _, r, l, _ in chunks]
    tuned_ms, tune_s = tune(rp, chunks[0][0], cold_p[0], chunks[0][3], args.tune_cache)

    def warm_pass():
        infos, keep = [], []
        for Xs, ranks, lams, outs in chunks:
            emb, rho0s, fbs = rp.warmstart_batched(Xs, ranks, P, hidden, sseed)
            if args.warm_groups == "embedding":
                plist, k = rp.batch_params(ranks, lams, tol=wl["tol"], rho0=rho0s, init_embeddings=emb,
                                           embedding_refine=args.embedding_refine)
            elif args.warm_groups == "seeds":   # seeds placed on the embedding, K-means of X
                plist, k = rp.batch_params(ranks, lams, tol=wl["tol"], rho0=rho0s, init_embeddings=emb,
                                           embedding_refine=2)
            else:   # the predicted rho0 only; groups by the cold start's K-means of X
                plist, k = rp.batch_params(ranks, lams, tol=wl["tol"], rho0=rho0s)
            infos += rp.solve_batched(Xs, plist, outs=outs)[1]
            keep.append((emb, k, fbs))
        return infos, keep

    def cold_pass():
        infos = []
        for (Xs, _, _, outs), plist in zip(chunks, cold_p):
            infos += rp.solve_batched(Xs, plist, outs=outs)[1]
        return infos

    def errors():
        out = []
        for ci, (_, _, _, outs) in enumerate(chunks):
            for k, o in enumerate(outs):
                out.append(ws.rel_err(o[0], inst[ci * chunk + k][1]))
        return out

    for _ in range(max(args.warmup, 1)):
        cold_pass()
        warm_pass()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cold = cold_pass()
    torch.cuda.synchronize()
    cold_s = time.perf_counter() - t0
    cold_phases = rp.batched_phases()   # the last cold launch
    cold_err = errors()
    rp.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        warm, keep = warm_pass()
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - t0
    prof = rp.profile_query()["batched"]
    rp.profile_enable(False)
    warm_phases = rp.batched_phases()   # the last warm launch (same instances as cold_phases)
    # the network pass alone (sketch, features, MLP, pooling) for all chunks
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for Xs, ranks, _, _ in chunks:
        rp.warmstart_batched(Xs, ranks, P, hidden, sseed)
    torch.cuda.synchronize()
    net_ms = 1e3 * (time.perf_counter() - t0) / len(chunks)
    warm_err = errors()
    fallbacks = sum(sum(k[2]) for k in keep)
    ratio = np.array(warm_err) / np.array(cold_err)
    count = len(inst)
    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(count * args.steps / warm_s, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(1e3 * warm_s / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "instances": count, "per_launch": chunk,
                   "model": f"MLP 68-{hidden}-{hidden}-{hidden}-65 (stored weights)",
                   "warm_iters_mean": round(float(np.mean([f["iters"] for f in warm])), 3),
                   "cold_iters_mean": round(float(np.mean([f["iters"] for f in cold])), 3),
                   "warm_converged": sum(f["status"] == 0 for f in warm),
                   "cold_converged": sum(f["status"] == 0 for f in cold),
                   "fallbacks": int(fallbacks),
                   "embedding_refine": args.embedding_refine,
                   "warm_groups": args.warm_groups,
                   "err_vs_planted_ratio_warm_over_cold": {
                       "median": round(float(np.median(ratio)), 5), "max": round(float(ratio.max()), 5)},
                   "tuner_seconds": round(tune_s, 2)},
        "cold_solves_per_s": round(count * args.steps / cold_s, 2),
        "speedup_vs_cold": round(cold_s / warm_s, 4),
        "network_pass_ms_per_launch": round(net_ms, 3),
        "phases_ms_last_launch": {"warm": warm_phases, "cold": cold_phases},
        "roofline": batched_roofline(prof, "warmstart"),
    }
    if not args.no_cpu_baseline:
        shapes = [tuple(x.shape) for x, _, _ in inst]
        ranks = [m[2] for _, _, m in inst]
        dn = [a * b for a, b in shapes]
        im = int(np.argsort(dn)[len(dn) // 2])
        line["cpu_baseline"] = batched_cpu_baseline(inst[im][0].cpu().numpy(), ranks[im],
                                                    ws.lam_of(*shapes[im]), shapes, ranks, cold, count)
    print(json.dumps(line), flush=True)


def calibrate_copy(args):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE
    counters: prints the bytes each launch reads and writes."""
    import torch
    nbytes = 1 << 30
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(max(args.steps, 1)):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                      "launches": max(args.steps, 1)}), flush=True)


def calibrate_mix(args):
    """Practical bandwidth ceilings: the library's streaming probe over 1 GiB
    arrays for the read/write mixes of the method's passes."""
    from paper_1904_07497_amd import respca as rp
    mixes = [(1, 0, "streaming read"), (1, 1, "copy"), (2, 0, "means pass on the compact state (X, B)"),
             (3, 0, "means pass (X, S, Theta)"), (3, 1, "3 reads + 1 write"),
             (3, 2, "l1 sweep on the compact state (X, B, L in; L, B out)"),
             (4, 3, "sweep (X, S, Theta, L in; L, S, Theta out)")]
    out = []
    for r, w, what in mixes:
        for nt in (False, True):
            gbps, ms = rp.bandwidth_probe(r, w, 1 << 30, reps=max(args.steps, 5), nontemporal=nt)
            out.append({"reads": r, "writes": w, "nontemporal": nt, "what": what,
                        "GBps": round(gbps, 1), "frac_of_8TBps": round(gbps / HBM_PEAK_GBS, 4),
                        "ms_per_launch": round(ms, 4)})
    print(json.dumps({"bandwidth_probe": out, "bytes_per_array": 1 << 30,
                      "reps": max(args.steps, 5)}), flush=True)


# profiled units that are one kernel per launch (candidates for the `roofline` object)
SINGLE_KERNEL_UNITS = ("sweep", "colnorm")

# kernels (name prefixes) that make up each profiled unit, for the counter summaries
UNIT_KERNELS = {
    "sweep": ("k_sweep_seg",),
    "means": ("k_group_partial",),
    "distance": ("k_split_centroids", "k_dist_", "k_refine", "k_assign_finish", "k_argmin",
                 "k_col_sqnorm"),
    "colnorm": ("k_l21_factor",),
    "batched": ("k_batched",),
    "affinity": ("k_sp_affinity",),
    "eigen": ("k_sp_mv_mfma", "k_sp_mv_reduce"),
}


def kernel_base(name):
    """The kernel's own identifier from a (demangled or mangled) dispatch name."""
    import re
    m = re.search(r"(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name


def read_counter_csvs(root):
    """Mean counter value per (kernel, counter) over the dispatches in every
    *counter_collection.csv under `root` (rocprofv3 --pmc -f csv output)."""
    import csv
    sums, counts = {}, {}
    for dirpath, _, files in os.walk(root):
        for fn in files:
            if not fn.endswith("counter_collection.csv"):
                continue
            with open(os.path.join(dirpath, fn)) as f:
                for row in csv.DictReader(f):
                    key = (row["Kernel_Name"], row["Counter_Name"])
                    sums[key] = sums.get(key, 0.0) + float(row["Counter_Value"])
                    counts[key] = counts.get(key, 0) + 1
    return {k: (sums[k] / counts[k], counts[k]) for k in sums}


def summarize_counters(unit, workload, root):
    """Per-launch HBM bytes of one unit from FETCH_SIZE / WRITE_SIZE counter runs
    (root/{copy,<workload>}_{FETCH_SIZE,WRITE_SIZE}), each scaled by what the same
    counter reads for the 1 GiB device copy of --calibrate-copy; writes
    profiles/traffic_<unit>_<workload>.json with the hash of the unit's sources."""
    def one(sub, counter):
        vals = read_counter_csvs(os.path.join(root, f"{sub}_{counter}"))
        return {k[0]: v for k, v in vals.items() if k[1] == counter}

    factors = {}
    for counter in ("FETCH_SIZE", "WRITE_SIZE"):
        copy = [v for k, v in one("copy", counter).items() if "copyBuffer" in k]
        if not copy:
            raise SystemExit(f"no copy kernel in {root}/copy_{counter}")
        factors[counter] = (1 << 30) / (copy[0][0] * 1024.0)
    fetch, write = one(workload, "FETCH_SIZE"), one(workload, "WRITE_SIZE")
    parts, total = [], 0.0
    for name in sorted(fetch):
        if not any(kernel_base(name).startswith(p) for p in UNIT_KERNELS[unit]):
            continue
        fb = fetch[name][0] * 1024.0 * factors["FETCH_SIZE"]
        wb = write.get(name, (0.0, 0))[0] * 1024.0 * factors["WRITE_SIZE"]
        parts.append({"kernel": display_name(name), "dispatches": fetch[name][1],
                      "fetch_kib_per_dispatch": round(fetch[name][0], 1),
                      "write_kib_per_dispatch": round(write.get(name, (0.0, 0))[0], 1),
                      "fetch_bytes_per_dispatch": int(fb), "write_bytes_per_dispatch": int(wb)})
        total += fb + wb
    rec = {"kernel": unit, "workload": workload, "bytes_per_launch": int(total),
           "fetch_factor": round(factors["FETCH_SIZE"], 5),
           "write_factor": round(factors["WRITE_SIZE"], 5),
           "kernel_source_sha": kernel_source_sha(unit), "parts": parts}
    path = os.path.join(ROOT, "profiles", f"traffic_{unit}_{workload}.json")
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec), flush=True)


def display_name(name):
    """A dispatch name without its argument list and namespaces."""
    if name.startswith("_Z"):
        return kernel_base(name)
    for pre in ("void ", "respca::", "(anonymous namespace)::"):
        name = name.replace(pre, "")
    return name.split("(")[0]


def summarize_stats(root, title, command, out_name):
    """profiles/<out_name>.md from a rocprofv3 --kernel-trace --stats run (the
    *kernel_stats.csv under root): calls, total, average, min and max per kernel."""
    import csv
    path = None
    for dirpath, _, files in os.walk(root):
        for fn in files:
            if fn.endswith("kernel_stats.csv"):
                path = os.path.join(dirpath, fn)
    if path is None:
        raise SystemExit(f"no kernel_stats.csv under {root}")
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# Kernel statistics: {title}", "",
             "Command (on one MI355X; rocprofv3 runs from /tmp, R is the repository root):", "",
             "```", "cd /tmp && export TMPDIR=/tmp; R=<repository root>", command, "```", "",
             "| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = display_name(r["Name"])
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    out = os.path.join(ROOT, "profiles", f"{out_name}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def summarize_pmc(root, title, command, out_name, top=8):
    """profiles/<out_name>.md from one rocprofv3 --pmc run with SQ_VALU_MFMA_BUSY_CYCLES,
    SQ_INSTS_VALU_MFMA_MOPS_*, SQ_WAIT_INST_ANY, SQ_WAVE_CYCLES, SQ_LDS_BANK_CONFLICT,
    SQ_LDS_IDX_ACTIVE and GRBM_GUI_ACTIVE: per kernel (mean per dispatch) the MFMA
    busy fraction of the SIMD cycles, the fraction of wave cycles spent waiting,
    the LDS bank-conflict cycles per active LDS cycle and the MFMA flops.
    GRBM_GUI_ACTIVE is summed over the 8 XCDs, so a dispatch lasts GRBM / 8 cycles
    on each of the 1024 SIMDs (256 CUs x 4)."""
    import collections
    vals = read_counter_csvs(root)
    per = collections.defaultdict(dict)
    calls = {}
    for (k, cn), (v, c) in vals.items():
        per[k][cn] = v
        calls[k] = max(calls.get(k, 0), c)
    rows = []
    for k, cs in per.items():
        cyc = cs.get("GRBM_GUI_ACTIVE", 0.0) / 8.0
        if cyc <= 0:
            continue
        mops = sum(v for cn, v in cs.items() if cn.startswith("SQ_INSTS_VALU_MFMA_MOPS"))
        busy = cs.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (cyc * 1024)
        wait = cs.get("SQ_WAIT_INST_ANY", 0.0) / max(cs.get("SQ_WAVE_CYCLES", 0.0), 1.0)
        lds = cs.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(cs.get("SQ_LDS_IDX_ACTIVE", 0.0), 1.0)
        rows.append((cyc * calls[k], display_name(k), calls[k], cyc, busy, wait, lds, mops * 512))
    rows.sort(key=lambda r: -r[0])
    lines = [f"# MFMA and wait counters: {title}", "",
             "Command (on one MI355X; rocprofv3 runs from /tmp, R is the repository root):", "",
             "```", "cd /tmp && export TMPDIR=/tmp; R=<repository root>", command, "```", "",
             "Per dispatch (means): cycles = GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs); "
             "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (cycles x 1024 SIMDs); waiting = "
             "SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES; LDS conflicts = SQ_LDS_BANK_CONFLICT / "
             "SQ_LDS_IDX_ACTIVE; MFMA flops = SQ_INSTS_VALU_MFMA_MOPS_* x 512.", "",
             "| kernel | dispatches | cycles | MFMA busy | waiting | LDS conflicts | MFMA flops |",
             "|---|---|---|---|---|---|---|"]
    for _, name, n, cyc, busy, wait, lds, fl in rows[:top]:
        lines.append(f"| `{name}` | {n} | {cyc:.0f} | {100 * busy:.1f} % | {100 * wait:.1f} % | "
                     f"{lds:.2f} | {fl:.3e} |")
    out = os.path.join(ROOT, "profiles", f"{out_name}.md")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="bf16", choices=["bf16", "fp32"],
                    help="distance contraction: split-bf16 MFMA with exact refinement, or FP32 MFMA")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip timing the other precision in the same run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--embedding-refine", type=int, default=1, choices=[0, 1],
                    help="warmstart workload: Lloyd passes on X after the embedding's K-means (1) "
                         "or the iterations straight from the embedding's groups (0)")
    ap.add_argument("--warm-groups", default="seeds", choices=["embedding", "kmeans", "seeds"],
                    help="warmstart workload, with the predicted rho0 in every case: initial groups "
                         "from the K-means of the predicted centroid sketches (embedding), from the "
                         "cold start's K-means of X (kmeans), or from the K-means of X seeded by "
                         "k-means++ on the predicted sketches (seeds)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the last-iteration comparison with the FP64 oracle")
    ap.add_argument("--tune-cache", default=None,
                    help="batched tile-shape cache file (read if it holds the shape bucket, else written)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--calibrate-mix", action="store_true",
                    help="run only the streaming bandwidth probe for the passes' read/write mixes")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("UNIT", "WORKLOAD", "ROOT"),
                    help="write profiles/traffic_UNIT_WORKLOAD.json from FETCH_SIZE/WRITE_SIZE "
                         "counter runs under ROOT (no GPU needed)")
    ap.add_argument("--summarize-stats", nargs=4, metavar=("ROOT", "TITLE", "COMMAND", "NAME"),
                    help="write profiles/NAME.md from a rocprofv3 --stats run under ROOT (no GPU needed)")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("ROOT", "TITLE", "COMMAND", "NAME"),
                    help="write profiles/NAME.md from a rocprofv3 --pmc MFMA/wait counter run under "
                         "ROOT (no GPU needed)")
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(*args.summarize_pmc)
        return
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on a "
              f"single MI355X; see the sharding notes in the design document)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1904_07497_amd import respca as rp

    if args.calibrate_copy:
        calibrate_copy(args)
        return
    if args.calibrate_mix:
        calibrate_mix(args)
        return
    wl = WORKLOADS[args.workload]
    if wl["gen"] == "batched":
        bench_batched(args, wl)
        return
    if wl["gen"] == "warmstart":
        bench_warmstart(args, wl)
        return
    if wl["gen"] == "scaling":
        bench_scaling(args, wl)
        return
    if wl["gen"] == "small":
        bench_small(args, wl)
        return
    if wl["gen"] == "spectral":
        bench_spectral(args, wl)
        return
    X = make_input(wl, np.float32)
    Xd = torch.from_numpy(X).to("cuda:0")
    d, n = X.shape

    def timed(precision, steps, warmup, units, max_lloyd=None):
        """Solves timed end to end; the library's event timing covers `units` only
        (each event pair can idle the device for microseconds)."""
        prec = rp.BF16GEMM_F32 if precision == "bf16" else rp.F32
        kw = dict(rank=wl["rank"], lam=wl["lam"], tol=wl["tol"], seed=0, precision=prec,
                  max_lloyd=max_lloyd if max_lloyd is not None else wl.get("max_lloyd", 100),
                  sparse_norm=wl.get("sparse_norm", 0))
        out = (rp.empty_colmajor(d, n, Xd.dtype, Xd.device),
               rp.empty_colmajor(d, n, Xd.dtype, Xd.device),
               torch.empty(n, dtype=torch.int32, device=Xd.device))
        for _ in range(warmup):
            rp.solve(Xd, out=out, **kw)
        torch.cuda.synchronize()
        rp.profile_enable(True, units=units)
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos.append(rp.solve(Xd, out=out, **kw)["info"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = rp.profile_query()
        rp.profile_enable(False)
        return t1 - t0, infos, prof, out

    # one solve with every unit timed gives the per-unit table and the dominant
    # kernel: the single-kernel unit with the largest summed time (the assignment
    # stage chains five kernels and the means and seeding units two or three, so
    # none has one launch duration to set beside a profiler's per-kernel average;
    # the assignment stage is reported beside it); the timed solves then carry
    # events around that kernel, the sweep and the assignment stage only
    _, _, prof_all, _ = timed(args.precision, 1, args.warmup, None)
    prof_all = {k: v for k, v in prof_all.items() if v["launches"] > 0}
    dom = max((k for k in prof_all if k in SINGLE_KERNEL_UNITS), key=lambda k: prof_all[k]["ms"])
    units = sorted({dom, "sweep", "distance"} | ({"colnorm"} if "colnorm" in prof_all else set()))
    elapsed, infos, prof, out = timed(args.precision, args.steps, 0, units)
    ms_per_step = 1e3 * elapsed / args.steps

    def roofline_of(name):
        k = prof[name]
        nl = max(k["launches"], 1)
        secs = k["ms"] / 1e3 / nl
        bpl, fpl = k["bytes"] / nl, k["flops"] / nl
        mfma = "bf16" if args.precision == "bf16" else "fp32"
        ridge = MFMA_PEAK_TFLOPS[mfma] * 1e12 / (HBM_PEAK_GBS * 1e9)
        if fpl > 0 and fpl / bpl > ridge:
            ach = fpl / secs / 1e12 if secs > 0 else 0.0
            return {"bound": "mfma", "achieved": round(ach, 2), "peak": MFMA_PEAK_TFLOPS[mfma],
                    "unit": "TFLOP/s", "frac": round(ach / MFMA_PEAK_TFLOPS[mfma], 4),
                    "traffic": load_traffic(name, args.workload), "kernel": name,
                    "flops_per_launch": fpl, "bytes_per_launch": bpl,
                    "mean_launch_ms": round(secs * 1e3, 4)}
        ach = bpl / secs / 1e9 if secs > 0 else 0.0
        return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": load_traffic(name, args.workload),
                "kernel": name, "bytes_per_launch": bpl, "mean_launch_ms": round(secs * 1e3, 4)}

    def sweep_with_ceiling(r, rp, array_bytes):
        """The sweep's figure beside the measured ceiling of its read/write mix (the
        library's streaming probe over arrays of the sweep's size, in the sweep's
        own load/store form: nontemporal from 64 MiB per array): 3 reads + 2
        writes for the l1 sweep on the compact state, 4 + 3 for the l2,1 sweep."""
        reads, writes = (4, 3) if wl.get("sparse_norm", 0) == 1 else (3, 2)
        nt = array_bytes >= STREAM_NT_BYTES
        gbps, _ = rp.bandwidth_probe(reads, writes, (array_bytes // 16) * 16, reps=10, nontemporal=nt)
        r = dict(r)
        r[f"ceiling_{reads}r{writes}w_GBps"] = round(gbps, 1)
        r["ceiling_nontemporal"] = nt
        r["frac_of_ceiling"] = round(r["achieved"] / gbps, 4) if gbps > 0 else None
        return r

    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "GBps": round(v["bytes"] / (v["ms"] / 1e3) / 1e9, 1) if v["ms"] > 0 else None,
                   "TFLOPs": round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["ms"] > 0 and v["flops"] else None}
               for k, v in prof_all.items()}
    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "d": d, "n": n, "c": wl["rank"],
                   "precision": ("split-bf16 MFMA distances + exact refinement; FP32 data, double "
                                 "accumulators") if args.precision == "bf16" else
                                "FP32 MFMA distances; FP32 data, double accumulators",
                   "iters": infos[-1]["iters"], "lloyd_steps": infos[-1]["lloyd_steps"],
                   "init_lloyd": infos[-1]["init_lloyd"], "refined_columns": infos[-1]["refined"]},
        "sweep_GBps": roofline_of("sweep")["achieved"],
        "sweep_roofline": sweep_with_ceiling(roofline_of("sweep"), rp, d * n * 4),
        "kernels": kernels,
        "kernels_note": "per-unit event times of one extra solve with every unit timed",
        "roofline": roofline_of(dom),
        "assignment_stage_roofline": dict(
            roofline_of("distance"),
            note="one assignment pass: centroid split, distance tile, bounded argmin, exact "
                 "refinement of near ties (five kernels) against d*n*w algorithmic bytes"),
    }
    if not args.no_compare:
        other = "fp32" if args.precision == "bf16" else "bf16"
        e2, i2, _, out2 = timed(other, args.steps, args.warmup, units)
        Lr, Sr = out2[0].double(), out2[1].double()
        line[f"{other}_solves_per_s"] = round(args.steps / e2, 4)
        line[f"{other}_iters"] = i2[-1]["iters"]
        line[f"rel_err_L_vs_{other}"] = float(torch.linalg.norm(out[0].double() - Lr) / torch.linalg.norm(Lr))
        line[f"rel_err_S_vs_{other}"] = float(torch.linalg.norm(out[1].double() - Sr) /
                                              max(float(torch.linalg.norm(Sr)), 1e-300))
        line["labels_equal_fraction"] = float((out[2] == out2[2]).double().mean())
    if wl.get("max_lloyd", 100) != 100:
        # the same workload with the method's p-step (K-means to convergence)
        e3, i3, _, out3 = timed(args.precision, 1, 0, units, max_lloyd=100)
        Lr = out3[0].double()
        line["full_kmeans_solves_per_s"] = round(1.0 / e3, 4)
        line["full_kmeans_iters"] = i3[-1]["iters"]
        line["full_kmeans_lloyd_steps"] = i3[-1]["lloyd_steps"]
        line["rel_diff_L_vs_full_kmeans"] = float(torch.linalg.norm(out[0].double() - Lr) /
                                                  torch.linalg.norm(Lr))
        line["config"]["max_lloyd"] = wl["max_lloyd"]
    if wl.get("sparse_norm", 0):
        line["config"]["sparse_norm"] = "l2,1"
        line["colnorm_roofline"] = roofline_of("colnorm")
    if not args.no_accuracy:
        prec = rp.BF16GEMM_F32 if args.precision == "bf16" else rp.F32
        line["accuracy_vs_oracle"] = accuracy_vs_oracle(rp, Xd, X, wl, prec, infos[-1]["iters"],
                                                        out[0])
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(X, wl, infos[-1])
    print(json.dumps(line), flush=True)


def bench_spectral(args, wl):
    """Whole solves with the spectral p-step; the dominant kernels are the affinity
    (Gram matrix on FP64 MFMA, 2 n^2 d flops) and the eigen block products."""
    import numpy as np
    import torch
    import oracle
    from oracle import spectral as osp
    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import synth

    X, moon = synth.moons(counts=wl["counts"], d=wl["d"], noise=wl["noise"], seed=5, frac=wl["frac"],
                          amp=wl["amp"], dtype=np.float32)
    d, n = X.shape
    Xd = torch.from_numpy(X).to("cuda:0")
    kw = dict(rank=wl["rank"], lam=wl["lam"], tol=wl["tol"], seed=0, precision=rp.F32,
              pstep=rp.PSTEP_SPECTRAL, sigma=wl["sigma"])
    out = (rp.empty_colmajor(d, n, Xd.dtype, Xd.device), rp.empty_colmajor(d, n, Xd.dtype, Xd.device),
           torch.empty(n, dtype=torch.int32, device=Xd.device))
    for _ in range(max(args.warmup, 1)):
        info = rp.solve(Xd, out=out, **kw)["info"]
        progress(f"spectral warm-up solve: {info['iters']} iterations, {info['eig_iters']} "
                 f"eigen iterations")
    torch.cuda.synchronize()
    rp.profile_enable(True, units=["affinity", "eigen", "sweep"])
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = rp.solve(Xd, out=out, **kw)["info"]
        progress(f"spectral timed solve {i + 1}/{args.steps}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rp.profile_query()
    rp.profile_enable(False)
    lab = out[2].cpu().numpy()
    groups = len(wl["counts"])

    def per_moon(labels):
        return [np.bincount(labels[moon == r], minlength=wl["rank"]).tolist() for r in range(groups)]

    def recovered(labels):
        return bool(all(len(set(labels[moon == r])) == 1 for r in range(groups))
                    and len(set(labels.tolist())) == groups)

    moon_groups = per_moon(lab)
    # the same solve with the K-means p-step, for contrast (untimed)
    km = rp.solve(Xd, rank=wl["rank"], lam=wl["lam"], tol=wl["tol"], seed=0, precision=rp.F32)
    km_lab = km["labels"].cpu().numpy()

    def unit(name, peak, unit_name, use_flops):
        k = prof[name]
        nl = max(k["launches"], 1)
        secs = k["ms"] / 1e3 / nl
        per = (k["flops"] if use_flops else k["bytes"]) / nl
        ach = per / secs / (1e12 if use_flops else 1e9) if secs > 0 else 0.0
        return {"bound": "mfma" if use_flops else "hbm", "achieved": round(ach, 2), "peak": peak,
                "unit": unit_name, "frac": round(ach / peak, 4),
                "traffic": load_traffic(name, args.workload), "kernel": name,
                ("flops_per_launch" if use_flops else "bytes_per_launch"): per,
                "launches": k["launches"], "mean_launch_ms": round(secs * 1e3, 4)}

    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(args.steps / elapsed, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "d": d, "n": n, "c": wl["rank"], "iters": info["iters"],
                   "lloyd_steps": info["lloyd_steps"], "eig_iters": info["eig_iters"],
                   "eig_unconverged": info["eig_unconverged"], "moons_recovered": recovered(lab),
                   "groups_per_moon": moon_groups, "kmeans_pstep_recovered": recovered(km_lab),
                   "kmeans_pstep_groups_per_moon": per_moon(km_lab)},
        "roofline": unit("affinity", 78.6, "TFLOP/s", True),
        "eigen_roofline": unit("eigen", HBM_PEAK_GBS, "GB/s", False),
        "sweep_roofline": unit("sweep", HBM_PEAK_GBS, "GB/s", False),
    }
    progress("spectral GPU part done; CPU baseline")
    if not args.no_cpu_baseline:
        # the FP64 oracle's spectral p-step (affinity, normalisation, dense eigensolver,
        # Lloyd on the rows) on a 1200-column subset, scaled to n columns by n^2 d for
        # the affinity and n^3 for the eigensolver
        rng = np.random.default_rng(0)
        m = 1200
        sub = np.asfortranarray(X[:, np.sort(rng.choice(n, m, replace=False))].astype(np.float64))
        t = time.perf_counter()
        W = osp.affinity(sub, wl["sigma"])
        t_aff = time.perf_counter() - t
        t = time.perf_counter()
        A, _ = osp.normalized_affinity(W)
        np.linalg.eigh(A)
        t_eig = time.perf_counter() - t
        scale2, scale3 = (n / m) ** 2, (n / m) ** 3
        per_pstep = t_aff * scale2 + t_eig * scale3
        sweep_s = 0.0
        st = {"L": np.zeros((d, m), order="F"), "S": np.zeros((d, m), order="F"),
              "Theta": np.zeros((d, m), order="F"), "labels": (np.arange(m) % wl["rank"]).astype(np.int32),
              "C": np.zeros((d, wl["rank"]), order="F"), "rho": 1e-4}
        t = time.perf_counter()
        oracle.step(oracle.make_params(wl["rank"], lam=wl["lam"], max_lloyd=1), sub, st)
        sweep_s = (time.perf_counter() - t) * (n / m)
        total = (info["iters"] + 1) * per_pstep + info["iters"] * sweep_s
        line["cpu_baseline"] = {"value": 1.0 / total, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "host_cores_available": host_cores(),
                                "sample": (f"FP64 oracle on a {m}-column subset: affinity {t_aff:.2f} s, "
                                           f"normalisation + dense eigensolver {t_eig:.2f} s, one K-means "
                                           f"outer iteration {sweep_s * m / n:.2f} s; scaled to n={n} by "
                                           f"n^2 (affinity), n^3 (eigensolver) and n (iteration), times "
                                           f"{info['iters'] + 1} spectral clusterings and {info['iters']} "
                                           f"iterations = {total:.0f} s")}
    print(json.dumps(line), flush=True)


def bench_small(args, wl):
    """The 500 x 500 FP64 configuration: whole solves of five seeded inputs per
    step (latency-bound: 47 iterations of a 2 MB problem), each compared with the
    FP64 oracle's whole solve of the same input."""
    import numpy as np
    import torch
    import oracle
    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import synth

    Xh = [synth.config_small(s)[0] for s in wl["seeds"]]
    Xs = [torch.from_numpy(X).to("cuda:0") for X in Xh]
    kw = dict(rank=wl["rank"], lam=wl["lam"], tol=wl["tol"], seed=0, precision=rp.F64)
    outs = [(rp.empty_colmajor(500, 500, torch.float64, "cuda:0"),
             rp.empty_colmajor(500, 500, torch.float64, "cuda:0"),
             torch.empty(500, dtype=torch.int32, device="cuda:0")) for _ in Xs]
    for _ in range(max(args.warmup, 1)):
        for X, o in zip(Xs, outs):
            rp.solve(X, out=o, **kw)
    torch.cuda.synchronize()
    rp.profile_enable(True, units=["sweep"])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = [rp.solve(X, out=o, **kw)["info"] for X, o in zip(Xs, outs)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = rp.profile_query()["sweep"]
    rp.profile_enable(False)
    acc = []
    t_or = 0.0
    for X, o, inf in zip(Xh, outs, infos):
        t = time.perf_counter()
        ref = oracle.solve(X, oracle.make_params(wl["rank"], lam=wl["lam"], tol=wl["tol"], seed=0))
        t_or += time.perf_counter() - t
        nL = np.linalg.norm(ref["L"])
        nS = np.linalg.norm(ref["S"])
        acc.append({"rel_err_L": float(np.linalg.norm(o[0].cpu().numpy() - ref["L"]) / nL),
                    "rel_err_S": float(np.linalg.norm(o[1].cpu().numpy() - ref["S"]) / nS),
                    "labels_equal": bool(np.array_equal(o[2].cpu().numpy(), ref["labels"])),
                    "iters": inf["iters"], "oracle_iters": ref["info"]["iters"]})
    count = len(Xs) * args.steps
    nl = max(prof["launches"], 1)
    secs = prof["ms"] / 1e3 / nl
    ach = prof["bytes"] / nl / secs / 1e9 if secs > 0 else 0.0
    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(count / elapsed, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl["name"], "d": 500, "n": 500, "c": wl["rank"],
                   "solves_per_step": len(Xs), "iters": [a["iters"] for a in acc]},
        "accuracy_vs_oracle": {"max_rel_err_L": max(a["rel_err_L"] for a in acc),
                               "max_rel_err_S": max(a["rel_err_S"] for a in acc),
                               "labels_equal": all(a["labels_equal"] for a in acc),
                               "iters_equal": all(a["iters"] == a["oracle_iters"] for a in acc),
                               "how": "whole GPU solve vs whole FP64 oracle solve, each seed"},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "sweep",
                     "bytes_per_launch": prof["bytes"] / nl, "mean_launch_ms": round(secs * 1e3, 4),
                     "note": "a 500 x 500 FP64 sweep moves 14 MB: launch latency, not HBM, bounds it"},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = {"value": round(len(Xh) / t_or, 4), "unit": "solves/s", "cores": 1,
                                "kind": "oracle", "host_cores_available": host_cores(),
                                "sample": (f"whole FP64 oracle solves of the same {len(Xh)} inputs, "
                                           f"timed ({t_or:.2f} s in total)")}
    print(json.dumps(line), flush=True)


def bench_scaling(args, wl):
    """Sec. 5 scalability: time of a fixed number of outer iterations on subsets of
    the clip, sampled in n (all rows) and in d (all columns); mean of `runs` solves
    per subset, and least-squares lines of time against n and against d."""
    import numpy as np
    import torch
    from paper_1904_07497_amd import respca as rp
    from paper_1904_07497_amd import synth

    X, _, _ = synth.video(n=wl["n"], seed=2, dtype=np.float32)
    d, n = X.shape
    rng = np.random.default_rng(0)
    prec = rp.BF16GEMM_F32 if args.precision == "bf16" else rp.F32

    def subset(nr, dr):
        cols = np.sort(rng.choice(n, int(round(n * nr)), replace=False)) if nr < 1 else np.arange(n)
        rows = np.sort(rng.choice(d, int(round(d * dr)), replace=False)) if dr < 1 else np.arange(d)
        return torch.from_numpy(np.asfortranarray(X[np.ix_(rows, cols)])).to("cuda:0")

    def run(Xd, profile=False):
        dd, nn = Xd.shape
        kw = dict(rank=wl["rank"], lam=float(np.sqrt(max(dd, nn))), tol=0.0, max_iter=wl["iters"],
                  seed=0, precision=prec)
        out = (rp.empty_colmajor(dd, nn, Xd.dtype, Xd.device),
               rp.empty_colmajor(dd, nn, Xd.dtype, Xd.device),
               torch.empty(nn, dtype=torch.int32, device=Xd.device))
        for _ in range(max(args.warmup, 1)):
            rp.solve(Xd, out=out, **kw)
        torch.cuda.synchronize()
        rp.profile_enable(profile, units=["sweep"] if profile else None)
        ts = []
        for _ in range(wl["runs"]):
            t0 = time.perf_counter()
            info = rp.solve(Xd, out=out, **kw)["info"]
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            assert info["iters"] == wl["iters"]
        prof = rp.profile_query()["sweep"] if profile else None
        rp.profile_enable(False)
        return float(np.mean(ts)), prof

    def fit(xs, ys):
        a, b = np.polyfit(xs, ys, 1)
        pred = a * np.asarray(xs) + b
        ss = float(np.sum((np.asarray(ys) - pred) ** 2))
        st = float(np.sum((np.asarray(ys) - np.mean(ys)) ** 2))
        return {"ms_per_unit": a * 1e3, "intercept_ms": b * 1e3, "r2": 1.0 - ss / st if st > 0 else 1.0}

    full_s, prof = run(subset(1.0, 1.0), profile=True)
    by_n, by_d = [], []
    for r in wl["ratios"]:
        t = full_s if r == 1.0 else run(subset(r, 1.0))[0]
        by_n.append({"n": int(round(n * r)), "d": d, "ms": round(t * 1e3, 3)})
    for r in wl["ratios"]:
        t = full_s if r == 1.0 else run(subset(1.0, r))[0]
        by_d.append({"n": n, "d": int(round(d * r)), "ms": round(t * 1e3, 3)})
    fn = fit([e["n"] for e in by_n], [e["ms"] / 1e3 for e in by_n])
    fd = fit([e["d"] for e in by_d], [e["ms"] / 1e3 for e in by_d])
    nl = max(prof["launches"], 1)
    secs = prof["ms"] / 1e3 / nl
    ach = prof["bytes"] / nl / secs / 1e9 if secs > 0 else 0.0
    line = {
        "metric": "RPCA solves/s + sweep HBM GB/s at rel-err<=1e-5 (BF16/learned vs plain FP32)",
        "value": round(1.0 / full_s, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": wl["runs"],
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(full_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["name"], "d": d, "n": n, "c": wl["rank"], "iters": wl["iters"],
                   "precision": args.precision},
        "time_vs_n": by_n,
        "time_vs_d": by_d,
        "linear_fit_n": {k: round(v, 6) for k, v in fn.items()},
        "linear_fit_d": {k: round(v, 9) for k, v in fd.items()},
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "sweep",
                     "bytes_per_launch": prof["bytes"] / nl, "mean_launch_ms": round(secs * 1e3, 4)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
