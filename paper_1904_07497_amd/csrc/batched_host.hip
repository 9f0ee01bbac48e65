// Host side of the batched solver: per-instance layout and workspace, work
// tables, hipGraph capture/replay of the persistent launch, and the tile-shape
// tuner with its on-disk cache.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/respca.h"
#include "batched.h"
#include "handle.h"
#include "kernels.h"

using namespace respca;

namespace {

constexpr int kTableCount = 6;
constexpr double kBarrierTimeoutS = 4.0;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Every per-call input that the captured graph depends on lives in this header
// block (descriptors, work tables, k-means++ uniforms); it is staged in pinned
// memory and copied to the device by the graph's first node.
struct Staged {
    size_t inst_off, sync_off, table_off, u_off, header_bytes;  // device header layout
    size_t readback_off;                                        // pinned readback area
    size_t stage_bytes;
};

struct Call {
    std::vector<BatchInst> inst;
    std::vector<int32_t> tables[kTableCount];
    std::vector<double> u;
    std::vector<size_t> u_start;
    size_t array_bytes = 0;  // per-instance arrays after the header
    int cmax = 0;
    int64_t max_steps = 0;
};

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 1469598103934665603ULL) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ULL;
    }
    return h;
}

respca_status validate(respca_handle h, const respca_params* params, int32_t batch, const int64_t* d,
                       const int64_t* n, const void* const* X, const int64_t* ldx, void* const* L,
                       const int64_t* ldl, void* const* S, const int64_t* lds,
                       std::vector<Resolved>& res) {
    if (!params || batch < 1 || !d || !n || !X || !ldx || !L || !ldl || !S || !lds)
        return fail(h, RESPCA_ERR_INVALID, "NULL argument or empty batch");
    if (batch > kMaxBatch) return fail(h, RESPCA_ERR_UNSUPPORTED, "batch above 1024 instances");
    res.resize(batch);
    for (int i = 0; i < batch; ++i) {
        respca_status s = resolve(h, &params[i], d[i], n[i], res[i]);
        if (s != RESPCA_OK) {
            h->err = "instance " + std::to_string(i) + ": " + h->err;
            return s;
        }
        if (res[i].precision != RESPCA_F32)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "batched solver runs FP32 instances only");
        if (res[i].sparse_norm != RESPCA_SPARSE_L1)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "batched solver runs the l1 penalty only");
        if (res[i].pstep != RESPCA_PSTEP_KMEANS)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "batched solver runs the K-means p-step only");
        if (!X[i] || !L[i] || !S[i]) return fail(h, RESPCA_ERR_INVALID, "NULL matrix pointer");
        if (ldx[i] < d[i] || ldl[i] < d[i] || lds[i] < d[i])
            return fail(h, RESPCA_ERR_INVALID, "leading dimension < d");
        if ((int64_t)(d[i] + 3) / 4 * 4 * n[i] >= (int64_t)INT32_MAX)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "batched instance too large");
        if (res[i].init_embedding && (int64_t)(res[i].emb_rows + 3) / 4 * 4 * n[i] >= (int64_t)INT32_MAX)
            return fail(h, RESPCA_ERR_UNSUPPORTED, "batched embedding too large");
        if (res[i].init_labels) {
            std::vector<int32_t> hl(n[i]);
            CK(hipMemcpy(hl.data(), res[i].init_labels, n[i] * sizeof(int32_t), hipMemcpyDeviceToHost));
            for (int64_t j = 0; j < n[i]; ++j)
                if (hl[j] < 0 || hl[j] >= res[i].c)
                    return fail(h, RESPCA_ERR_INVALID, "init_labels out of range");
        }
    }
    return RESPCA_OK;
}

// Per-instance tiling and array layout; tables of work items.
void plan(const BatchTune& tune, int32_t batch, const int64_t* d, const int64_t* n,
          const void* const* X, const int64_t* ldx, void* const* L, const int64_t* ldl,
          void* const* S, const int64_t* lds, int32_t* const* labels,
          const std::vector<Resolved>& res, Call& call) {
    call.inst.assign(batch, BatchInst{});
    for (auto& t : call.tables) t.assign(batch + 1, 0);
    call.u.clear();
    call.u_start.assign(batch, 0);
    call.cmax = 0;
    call.max_steps = 0;
    size_t off = 0;
    for (int i = 0; i < batch; ++i) {
        BatchInst& B = call.inst[i];
        const Resolved& r = res[i];
        B.Xc = (const float*)X[i];
        B.Lc = (float*)L[i];
        B.Sc = (float*)S[i];
        B.labels_out = labels ? labels[i] : nullptr;
        B.init_labels = r.init_labels;
        B.Ec = r.init_embedding;
        B.lde = r.emb_ld;
        B.refine_x = r.emb_refine == 1 ? 1 : 0;
        B.seed_only = r.emb_refine == 2 ? 1 : 0;
        B.ldx = ldx[i];
        B.ldl = ldl[i];
        B.lds = lds[i];
        B.d = (int)d[i];
        B.dp = (int)((d[i] + 3) / 4 * 4);
        B.n = (int)n[i];
        B.c = r.c;
        B.kpad = (r.c + 15) / 16 * 16;
        B.nkc = (B.kpad + 127) / 128;
        B.nrb = (B.dp + kBatchRows - 1) / kBatchRows;
        B.er = B.Ec ? r.emb_rows : 0;
        B.kdp = B.Ec ? (B.er + 3) / 4 * 4 : B.dp;
        B.mrows = std::max(B.dp, B.kdp);
        B.mrb = (B.mrows + kBatchRows - 1) / kBatchRows;
        B.jc = tune.jc;
        int rows = std::max(32, tune.slice_rows / 32 * 32);
        if (rows > B.mrows) rows = (B.mrows + 31) / 32 * 32;
        B.slice_rows = rows;
        B.slices = (B.mrows + rows - 1) / rows;
        const int ntiles = (B.n + 127) / 128;
        B.n_tile = ((B.n + B.jc - 1) / B.jc) * B.nrb;
        B.n_argmin = (B.n + kArgminCols - 1) / kArgminCols;
        const int nseg_max = (B.n + kBatchSegCols - 1) / kBatchSegCols + B.c;
        B.n_sweep = nseg_max * B.mrb;
        B.lambda = r.lambda;
        B.tol = r.tol;
        B.rho0 = r.rho0;
        B.kappa = r.kappa;
        B.rho_max = r.rho_max;
        B.max_iter = r.max_iter;
        B.max_lloyd = r.max_lloyd;
        // work tables (prefix sums)
        const int64_t counts[kTableCount] = {B.n_tile, (B.n + 15) / 16, B.c, (int64_t)nseg_max * B.mrb,
                                             (int64_t)ntiles * B.slices * B.nkc, B.n_argmin};
        for (int t = 0; t < kTableCount; ++t)
            call.tables[t][i + 1] = call.tables[t][i] + (int32_t)counts[t];
        // arrays: offsets relative to the array area (pointers patched later)
        const size_t dpn = (size_t)B.dp * B.n * sizeof(float);
        auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
        B.X = (float*)take(dpn);
        B.L = (float*)take(dpn);
        B.S = (float*)take(dpn);   // the compact l1 state B = X - L + Theta/rho until the end
        B.Z = B.Ec ? (float*)take((size_t)B.kdp * B.n * sizeof(float)) : nullptr;
        B.C = (float*)take((size_t)B.mrows * B.c * sizeof(float));
        B.lab[0] = (int32_t*)take(B.n * sizeof(int32_t));
        B.lab[1] = (int32_t*)take(B.n * sizeof(int32_t));
        B.perm = (int32_t*)take(B.n * sizeof(int32_t));
        B.counts = (int32_t*)take(B.c * sizeof(int32_t));
        B.segb = (int32_t*)take(nseg_max * sizeof(int32_t));
        B.segl = (int32_t*)take(nseg_max * sizeof(int32_t));
        B.segf = (int32_t*)take((2 * (size_t)B.c + 1) * sizeof(int32_t));   // 2c keys when incremental
        B.pmeans = (double*)take((size_t)nseg_max * B.mrows * sizeof(double));
        B.part = (float*)take((size_t)B.slices * B.n * B.kpad * sizeof(float));
        B.d2 = (double*)take(B.n * sizeof(double));
        B.chosen = (int32_t*)take(B.n * sizeof(int32_t));
        B.seeds = (int32_t*)take(B.c * sizeof(int32_t));
        B.cnorm = (double*)take(B.c * sizeof(double));
        B.gsum = (double*)take((size_t)B.mrows * B.c * sizeof(double));
        B.sweep_part = (double*)take(3 * (size_t)std::max(B.n_sweep, B.n_tile) * sizeof(double));
        B.chg = (int32_t*)take(4 * (size_t)B.n_argmin * sizeof(int32_t));   // one per argmin wave
        // k-means++ uniforms from the instance's seed
        call.u_start[i] = call.u.size();
        uint64_t state = r.init_labels ? 0 : r.seed;
        for (int m = 0; m < B.c; ++m) call.u.push_back(uniform01(state));
        call.cmax = std::max(call.cmax, r.init_labels ? 0 : B.c);
        call.max_steps += 2 + (int64_t)r.max_lloyd * (1 + (int64_t)r.max_iter);
    }
    call.array_bytes = off;
    if (call.max_steps > 100000000) call.max_steps = 100000000;
}

Staged layout_of(const Call& call, int32_t batch) {
    Staged s;
    size_t o = 0;
    s.inst_off = o;
    o = align_up(o + batch * sizeof(BatchInst), 256);
    s.sync_off = o;
    o = align_up(o + sizeof(BatchSync), 256);
    s.table_off = o;
    o = align_up(o + (size_t)kTableCount * (batch + 1) * sizeof(int32_t), 256);
    s.u_off = o;
    o = align_up(o + std::max<size_t>(call.u.size(), 1) * sizeof(double), 256);
    s.header_bytes = o;
    s.readback_off = o;
    s.stage_bytes = o + align_up(batch * sizeof(BatchInst) + 256 + sizeof(BatchSync), 256);
    return s;
}

respca_status run_batched(respca_handle h, const Call& call_in, int32_t batch, hipStream_t caller,
                          respca_info* info, double* elapsed_ms) {
    Call call = call_in;
    const Staged L = layout_of(call, batch);
    const size_t total = L.header_bytes + call.array_bytes;
    CKS(ensure(h, h->bws, total));
    if (h->bstage_bytes < L.stage_bytes) {
        if (h->bstage) CK(hipHostFree(h->bstage));
        h->bstage = nullptr;
        h->bstage_bytes = 0;
        CK(hipHostMalloc((void**)&h->bstage, L.stage_bytes, hipHostMallocDefault));
        h->bstage_bytes = L.stage_bytes;
    }
    if (!h->bstream) CK(hipStreamCreateWithFlags(&h->bstream, hipStreamNonBlocking));
    if (!h->bev) CK(hipEventCreateWithFlags(&h->bev, hipEventDisableTiming));

    // patch array offsets into device pointers
    char* base = (char*)h->bws.p;
    char* arr = base + L.header_bytes;
    auto fix = [&](auto*& p) { p = reinterpret_cast<std::remove_reference_t<decltype(p)>>(arr + (size_t)p); };
    const double* u_dev = (const double*)(base + L.u_off);
    for (int i = 0; i < batch; ++i) {
        BatchInst& B = call.inst[i];
        fix(B.X); fix(B.L); fix(B.S); fix(B.C); fix(B.lab[0]); fix(B.lab[1]); fix(B.perm);
        fix(B.counts); fix(B.segb); fix(B.segl); fix(B.segf); fix(B.pmeans); fix(B.part); fix(B.d2);
        fix(B.chosen); fix(B.seeds); fix(B.cnorm); fix(B.gsum); fix(B.sweep_part); fix(B.chg);
        if (B.Ec) fix(B.Z);
        B.u = u_dev + call.u_start[i];
    }
    // stage the header
    char* st = h->bstage;
    std::memcpy(st + L.inst_off, call.inst.data(), batch * sizeof(BatchInst));
    std::memset(st + L.sync_off, 0, sizeof(BatchSync));
    for (int t = 0; t < kTableCount; ++t)
        std::memcpy(st + L.table_off + (size_t)t * (batch + 1) * sizeof(int32_t), call.tables[t].data(),
                    (batch + 1) * sizeof(int32_t));
    if (!call.u.empty()) std::memcpy(st + L.u_off, call.u.data(), call.u.size() * sizeof(double));

    int dev = h->device, cus = 0, rate_khz = 0;
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    const int occ = batched_blocks_per_cu();
    if (occ < 1) return fail(h, RESPCA_ERR_HIP, "batched kernel cannot be resident");
    const int nblocks = cus * std::max(1, std::min(occ, h->tune.blocks_per_cu));

    BatchArgs args;
    args.inst = (BatchInst*)(base + L.inst_off);
    args.batch = batch;
    args.sync = (BatchSync*)(base + L.sync_off);
    args.timeout_ticks = (uint64_t)(kBarrierTimeoutS * (double)rate_khz * 1000.0);
    args.cmax = call.cmax;
    args.max_steps = (int)call.max_steps;
    const int32_t* tb = (const int32_t*)(base + L.table_off);
    args.off_tile = tb;
    args.off_d2 = tb + 1 * (batch + 1);
    args.off_kc = tb + 2 * (batch + 1);
    args.off_seg = tb + 3 * (batch + 1);
    args.off_dist = tb + 4 * (batch + 1);
    args.off_col = tb + 5 * (batch + 1);

    uint64_t sig = fnv1a(st, L.header_bytes);
    sig = fnv1a(&nblocks, sizeof(nblocks), sig);
    sig = fnv1a(&args, sizeof(args), sig);
    if (!(h->bexec && h->bsig == sig)) {
        if (h->bexec) CK(hipGraphExecDestroy(h->bexec));
        if (h->bgraph) CK(hipGraphDestroy(h->bgraph));
        h->bexec = nullptr;
        h->bgraph = nullptr;
        CK(hipStreamBeginCapture(h->bstream, hipStreamCaptureModeThreadLocal));
        hipError_t e1 = hipMemcpyAsync(base, st, L.header_bytes, hipMemcpyHostToDevice, h->bstream);
        launch_batched_reset(args.sync, batch, h->bstream);
        launch_batched(args, nblocks, h->bstream);
        hipError_t e2 = hipMemcpyAsync(st + L.readback_off, base + L.inst_off,
                                       batch * sizeof(BatchInst), hipMemcpyDeviceToHost, h->bstream);
        hipError_t e3 = hipMemcpyAsync(st + L.readback_off + align_up(batch * sizeof(BatchInst), 256),
                                       base + L.sync_off, sizeof(BatchSync), hipMemcpyDeviceToHost,
                                       h->bstream);
        hipGraph_t g = nullptr;
        hipError_t e4 = hipStreamEndCapture(h->bstream, &g);
        CK(e1);
        CK(e2);
        CK(e3);
        CK(e4);
        h->bgraph = g;
        CK(hipGraphInstantiate(&h->bexec, h->bgraph, nullptr, nullptr, 0));
        h->bsig = sig;
    }
    // order after the caller's earlier work, replay, wait
    CK(hipEventRecord(h->bev, caller));
    CK(hipStreamWaitEvent(h->bstream, h->bev, 0));
    hipEvent_t t0 = nullptr, t1 = nullptr;
    double prof_ms = 0.0;
    const bool timed = (h->prof_mask >> RESPCA_KERNEL_BATCHED) & 1u;
    if (!elapsed_ms && timed) elapsed_ms = &prof_ms;
    if (elapsed_ms) {
        CK(hipEventCreate(&t0));
        CK(hipEventCreate(&t1));
        CK(hipEventRecord(t0, h->bstream));
    }
    CK(hipGraphLaunch(h->bexec, h->bstream));
    if (elapsed_ms) CK(hipEventRecord(t1, h->bstream));
    CK(hipStreamSynchronize(h->bstream));
    if (elapsed_ms) {
        float ms = 0.f;
        CK(hipEventElapsedTime(&ms, t0, t1));
        *elapsed_ms = ms;
        CK(hipEventDestroy(t0));
        CK(hipEventDestroy(t1));
    }
    const BatchInst* out = (const BatchInst*)(st + L.readback_off);
    const BatchSync* sy = (const BatchSync*)(st + L.readback_off + align_up(batch * sizeof(BatchInst), 256));
    for (int p = 0; p < BP_COUNT; ++p) h->bphase_ms[p] = (double)sy->phase_ticks[p] / (double)rate_khz;
    h->bsteps = (int64_t)sy->steps;
    if (sy->abort) return fail(h, RESPCA_ERR_HIP, "batched kernel: grid barrier timed out (aborted)");
    respca_status worst = RESPCA_OK;
    double alg_bytes = 0.0;
    for (int i = 0; i < batch; ++i) {
        const BatchInst& B = out[i];
        if (B.status >= 0 && B.nx > 0.0) {
            // passes over X: ||X||; 5 + 1 per outer iteration (the sweep on the compact
            // state: X, B, L in and L, B out; the assignment) and 2 more for each that
            // ran the means pass over X and B (the others had the group sums from the
            // previous sweep); 2 per extra Lloyd pass on L; and the start: the means
            // of X for given labels, seeding (c passes) + nearest-seed assignment + 2 per
            // Lloyd pass for a cold start, or for an embedding 2 per Lloyd pass on X plus
            // two means of X, with its seeding and Lloyd passes counted on the embedding
            double px = 1.0 + 6.0 * B.iters + 2.0 * B.meansd + 2.0 * (B.lloyd_total - B.iters);
            double pz = 0.0;
            if (call.inst[i].init_labels) px += 1.0;
            else if (B.Z && B.seed_only) {   // seeding passes on the embedding, the rest on X
                px += 1.0 + 2.0 * B.init_lloyd;
                pz = (double)B.c;
            } else if (B.Z) {
                px += 2.0 + 2.0 * B.ref_lloyd;
                pz = (double)B.c + 1.0 + 2.0 * (B.init_lloyd - B.ref_lloyd);
            } else px += (double)B.c + 1.0 + 2.0 * B.init_lloyd;
            // a means step done incrementally read only the moved columns (twice each)
            px -= (double)B.inc_steps[0] - (double)B.inc_cols[0] / (double)B.n;
            pz -= (double)B.inc_steps[1] - (double)B.inc_cols[1] / (double)B.n;
            alg_bytes += (double)B.n * sizeof(float) * ((double)B.d * px + (double)B.er * pz);
        }
        if (info) {
            respca_info& f = info[i];
            std::memset(&f, 0, sizeof(f));
            f.iters = B.iters;
            f.lloyd_steps = B.lloyd_total;
            f.init_lloyd = B.init_lloyd;
            f.status = B.status;
            f.primal = B.primal;
            f.dL = B.dL;
            f.dS = B.dS;
            f.rho_final = B.rho_final;
        }
        if (B.status < 0 && (worst >= 0 || B.status < worst)) worst = (respca_status)B.status;
        if (B.status == RESPCA_NOT_CONVERGED && worst == RESPCA_OK) worst = RESPCA_NOT_CONVERGED;
    }
    if (timed) {
        h->prof_launches[RESPCA_KERNEL_BATCHED] += 1;
        h->prof_ms[RESPCA_KERNEL_BATCHED] += *elapsed_ms;
        h->prof_bytes[RESPCA_KERNEL_BATCHED] += alg_bytes;
    }
    if (worst < 0) h->err = "an instance failed (see its info status)";
    return worst;
}

// Candidate tile shapes of the tuner (the only shapes the batched kernel takes).
constexpr int kTuneJc[] = {4, 8, 16, 32};
constexpr int kTuneRows[] = {512, 1024, 2048};
constexpr int kTuneBpc[] = {1, 2};
// Bumped whenever the batched kernel changes, so stale cache lines are not used.
constexpr const char* kTuneVersion = "k3";

template <size_t N>
bool one_of(int v, const int (&set)[N]) {
    for (int x : set)
        if (x == v) return true;
    return false;
}

bool tile_valid(int jc, int rows, int bpc) {
    return one_of(jc, kTuneJc) && one_of(rows, kTuneRows) && one_of(bpc, kTuneBpc);
}

std::string bucket_key(int32_t batch, const int64_t* d, const int64_t* n, const std::vector<Resolved>& r,
                       int device) {
    std::vector<double> dn(batch);
    int cmax = 0;
    for (int i = 0; i < batch; ++i) {
        dn[i] = (double)d[i] * (double)n[i];
        cmax = std::max(cmax, r[i].c);
    }
    std::nth_element(dn.begin(), dn.begin() + batch / 2, dn.end());
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
    for (auto& ch : arch) if (ch == ' ' || ch == ':') ch = '_';
    char key[256];
    std::snprintf(key, sizeof(key), "%s_%s_b%d_dn2^%d_c%d", arch.c_str(), kTuneVersion, batch,
                  (int)std::lround(std::log2(std::max(dn[batch / 2], 1.0))), cmax);
    return key;
}

}  // namespace

extern "C" {

respca_status respca_solve_batched(respca_handle h, const respca_params* params, int32_t batch,
                                   const int64_t* d, const int64_t* n, const void* const* X,
                                   const int64_t* ldx, void* const* L, const int64_t* ldl,
                                   void* const* S, const int64_t* lds, int32_t* const* labels,
                                   respca_info* info, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    std::vector<Resolved> res;
    CKS(validate(h, params, batch, d, n, X, ldx, L, ldl, S, lds, res));
    CK(hipSetDevice(h->device));
    Call call;
    plan(h->tune, batch, d, n, X, ldx, L, ldl, S, lds, labels, res, call);
    return run_batched(h, call, batch, (hipStream_t)stream, info, nullptr);
}

respca_status respca_autotune_batched(respca_handle h, const respca_params* params, int32_t batch,
                                      const int64_t* d, const int64_t* n, const void* const* X,
                                      const int64_t* ldx, void* const* L, const int64_t* ldl,
                                      void* const* S, const int64_t* lds, const char* cache_path,
                                      double* best_ms, void* stream) {
    if (!h) return RESPCA_ERR_INVALID;
    std::vector<Resolved> res;
    CKS(validate(h, params, batch, d, n, X, ldx, L, ldl, S, lds, res));
    CK(hipSetDevice(h->device));
    const std::string key = bucket_key(batch, d, n, res, h->device);
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "r")) {
            char k[256];
            int jc, rows, bpc;
            double ms;
            bool found = false;
            while (std::fscanf(f, "%255s %d %d %d %lf", k, &jc, &rows, &bpc, &ms) == 5)
                if (key == k && tile_valid(jc, rows, bpc)) {
                    h->tune = BatchTune{jc, rows, bpc};
                    if (best_ms) *best_ms = ms;
                    found = true;
                }
            std::fclose(f);
            if (found) return RESPCA_OK;
        }
    }
    BatchTune best = h->tune;
    double best_t = 1e300;
    std::vector<respca_info> info(batch);
    for (int bpc : kTuneBpc)
        for (int rows : kTuneRows)
            for (int jc : kTuneJc) {
                h->tune = BatchTune{jc, rows, bpc};
                Call call;
                plan(h->tune, batch, d, n, X, ldx, L, ldl, S, lds, nullptr, res, call);
                double ms = 0.0;
                respca_status s = run_batched(h, call, batch, (hipStream_t)stream, info.data(), nullptr);
                if (s < 0) return s;
                CKS(run_batched(h, call, batch, (hipStream_t)stream, info.data(), &ms));  // graph replay
                if (ms < best_t) { best_t = ms; best = h->tune; }
            }
    h->tune = best;
    if (best_ms) *best_ms = best_t;
    if (cache_path) {
        if (FILE* f = std::fopen(cache_path, "a")) {
            std::fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), best.jc, best.slice_rows,
                         best.blocks_per_cu, best_t);
            std::fclose(f);
        }
    }
    return RESPCA_OK;
}

respca_status respca_set_batched_tile(respca_handle h, int32_t jc, int32_t slice_rows,
                                      int32_t blocks_per_cu) {
    if (!h) return RESPCA_ERR_INVALID;
    if (!tile_valid(jc, slice_rows, blocks_per_cu))
        return fail(h, RESPCA_ERR_INVALID, "tile shape is not one of the tuner's candidates");
    h->tune = BatchTune{jc, slice_rows, blocks_per_cu};
    return RESPCA_OK;
}

respca_status respca_get_batched_tile(respca_handle h, int32_t* jc, int32_t* slice_rows,
                                      int32_t* blocks_per_cu) {
    if (!h) return RESPCA_ERR_INVALID;
    if (jc) *jc = h->tune.jc;
    if (slice_rows) *slice_rows = h->tune.slice_rows;
    if (blocks_per_cu) *blocks_per_cu = h->tune.blocks_per_cu;
    return RESPCA_OK;
}

respca_status respca_profile_batched_phases(respca_handle h, double* ms, int32_t count,
                                            int64_t* steps) {
    if (!h || count < 0) return RESPCA_ERR_INVALID;
    for (int p = 0; p < count && p < BP_COUNT; ++p)
        if (ms) ms[p] = h->bphase_ms[p];
    if (steps) *steps = h->bsteps;
    return RESPCA_OK;
}

}  // extern "C"
