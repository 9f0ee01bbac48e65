// Device-side descriptors of the batched persistent solver (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace respca {

constexpr int kMaxBatch = 1024;   // instances per batched call (LDS-cached work tables)
constexpr int kBatchRows = 256;   // rows per tile (one wave covers them, 4 per lane)
constexpr int kBatchSegCols = 64; // max columns of one group segment (means and sweep items)
constexpr int kArgminCols = 64;   // columns per argmin item (16 lanes each, 4 per lane group)

// One instance.  The static part is written by the host; the state part is
// owned by the kernel (initialised in its first phases, read back by the host).
struct BatchInst {
    // caller buffers
    const float* Xc;
    float* Lc;
    float* Sc;
    int32_t* labels_out;       // nullable
    const int32_t* init_labels;  // nullable
    const float* Ec;           // nullable: er x n embedding whose columns are clustered first
    int64_t ldx, ldl, lds, lde;
    // internal copies, zero-padded to dp rows (leading dimension dp)
    float* X;
    float* L;
    float* S;                  // B = X - L + Theta/rho of the last sweep (S and Theta follow)
    float* Z;                  // embedding copy zero-padded to kdp rows (null without one)
    float* C;                  // centroids, leading dimension = rows of the current K-means matrix
    int32_t* lab[2];
    int32_t* perm;
    int32_t* counts;
    int32_t* segb;
    int32_t* segl;
    int32_t* segf;
    double* pmeans;            // [segment][rows of the current K-means matrix]
    float* part;               // [slice][n][kpad]
    double* d2;
    int32_t* chosen;
    int32_t* seeds;
    const double* u;           // k-means++ uniforms (host-drawn from splitmix64(seed))
    double* cnorm;
    double* gsum;              // [group][rows]: group sums (double) of the last Lloyd-family means
    double* sweep_part;        // 3 per sweep item (segment x row block), 1 per pack tile
    int32_t* chg;              // 1 per wave of each argmin item
    // shape and tiling.  The initial K-means runs on the columns of X (kdp = dp) or of
    // the embedding (kdp = 4 * ceil(er / 4)); mrows = max(dp, kdp) and mrb row blocks
    // of kBatchRows cover both.
    int d, dp, n, c, kpad, nrb, jc, slices, slice_rows, nkc, n_sweep, n_tile, n_argmin;
    int er, kdp, mrows, mrb;
    // parameters
    double lambda, tol, rho0, kappa, rho_max;
    int max_iter, max_lloyd;
    int refine_x;              // embedding starts: Lloyd on X after the embedding's K-means
    int seed_only;             // embedding starts: the embedding only places the k-means++
                               // seeds; their columns of X start the K-means of X
    // state
    int mode, cur, iters, lloyd_iter, lloyd_total, init_lloyd, ref_lloyd, status, nseg;
    int next_ready;            // pmeans and the sort tables hold the next L-step's group sums
    int meansd;                // outer iterations that ran the means pass over X and B
    int pmode;                 // mode of the previous step
    int moved;                 // columns whose label the previous step's assignment changed
    int inc;                   // this step's means are the incremental update (moved columns only)
    int inc_steps[2];          // incremental means steps on the d-row matrices [0] / the embedding [1]
    int64_t inc_cols[2];       // columns those steps read (two per moved column)
    double rho, nx, rho_final, primal, dL, dS;
    double rho_prev;           // penalty of the last sweep: S holds the compact state B of it
};

// Phases of the persistent kernel, for its per-phase timing.
enum BatchPhase : int {
    BP_PACK = 0, BP_INIT, BP_SEED_D2, BP_SEED_PICK, BP_GATHER, BP_SORT, BP_MEANS, BP_FINALIZE,
    BP_SWEEP, BP_DIST, BP_ARGMIN, BP_CONTROL, BP_COUNT
};

struct BatchSync {
    unsigned count;                  // top-level barrier arrivals (one per group)
    unsigned gen;                    // barrier generation
    int abort;
    int active;
    uint64_t phase_ticks[BP_COUNT];  // wall-clock ticks per phase, measured by workgroup 0
    uint64_t steps;
    unsigned group_count[8 * 64];    // per-group barrier arrivals, one 256-byte line each
};

struct BatchArgs {
    BatchInst* inst;
    int batch;
    BatchSync* sync;
    uint64_t timeout_ticks;
    int cmax;
    int max_steps;
    // prefix tables (batch + 1 entries) of per-instance work items
    const int32_t* off_tile;   // ceil(n/jc) * nrb   (pack, unpack; nrb = ceil(dp/256))
    const int32_t* off_d2;     // ceil(n/16)         (k-means++ distances, four columns per wave)
    const int32_t* off_kc;     // c                  (seed columns, centroids and their norms)
    const int32_t* off_seg;    // (ceil(n/64) + c) * mrb (group partial sums, sweep)
    const int32_t* off_dist;   // ceil(n/128) * slices * nkc (distance tiles)
    const int32_t* off_col;    // ceil(n/kArgminCols) (argmin)
};

void launch_batched_reset(BatchSync* s, int batch, hipStream_t st);
void launch_batched(const BatchArgs& args, int nblocks, hipStream_t st);
int batched_blocks_per_cu();

}  // namespace respca
