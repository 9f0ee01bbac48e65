// Spectral-clustering p-step (internal; not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/respca.h"

namespace respca {

constexpr int kSpectralMaxGroups = 40;    // c limit: the eigen block is c + 8 <= 48 vectors
constexpr int64_t kSpectralMaxN = 32768;  // the n x n affinity is held in HBM (8 n^2 bytes)
constexpr int kSpectralMaxIters = 100;    // filtered subspace iterations per embedding

struct SpectralStats {
    int64_t iters = 0;        // filtered subspace iterations summed over calls
    int64_t calls = 0;
    int64_t unconverged = 0;  // calls that stopped at kSpectralMaxIters
    double last_residual = 0.0;
};

// Eigen block size for n points and c groups.
int spectral_block(int64_t n, int c);

// Row embedding of the columns of Y (d x n, ldy): emb (device, c x n doubles,
// leading dimension c) receives the unit rows of the eigenvectors of the c
// largest eigenvalues of D^{-1/2} W D^{-1/2}, W_ij = exp(-||y_i - y_j||^2 /
// (2 sigma^2)), W_ii = 0.  seed drives the initial block; with warm, the Ritz
// vectors left by the previous call (same n and c, same handle) start the
// iteration instead (within one solve the embedding changes little from one
// p-step to the next).  Enqueued on st; reads back one residual per filtered
// iteration.
template <typename T>
respca_status spectral_embed(respca_handle h, const T* Y, int64_t ldy, int64_t d, int64_t n, int c,
                             double sigma, uint64_t seed, double* emb, SpectralStats* stats,
                             hipStream_t st, bool warm = false);

// The c largest eigenvalues (host, decreasing) found by the last spectral_embed.
respca_status spectral_eigenvalues(respca_handle h, int64_t n, int c, double* out, hipStream_t st);

}  // namespace respca
