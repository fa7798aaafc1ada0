// Host-side launcher of the persistent batched CG kernel (batch_cg.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace gko {

// Per-batch outcome, the worst over all systems (atomicMax).
constexpr int kBatchNotConverged = 1;
constexpr int kBatchBreakdown = 2;
constexpr int kBatchNotSpd = 3;

// Largest system the kernel takes (rows): its iteration vectors live in LDS.
constexpr int64_t kBatchMaxRows = 2048;

struct batch_args {
    int64_t nsys;
    const int64_t *row_off;   // nsys+1
    const int64_t *nnz_off;   // nsys+1
    const int32_t *rp_local;  // row_off[nsys] + nsys local row offsets
    const int32_t *col;       // local column indices
    const void *val;          // values (FP64 or FP32)
    const int32_t *order;     // system ids, most rows first (ties: most nonzeros)
    unsigned *counter;        // work-queue head (reset by the launcher)
    const double *b;
    double *x;
    double tol;
    int32_t maxit;
    int32_t *iters;
    double *relres;
    int *status;
    int64_t max_m;
    int64_t max_row_len;      // longest row of any system
    int block;                // workgroup size: 64, 128, 256 or 512
    bool lean;                // only p in LDS (batch_lean_fits must hold)
    bool waves;               // systems of <= kWaveRows rows one per wavefront (batch_waves_fit)
};

// Rows of up to this many entries are held in registers for a system's solve.
constexpr int kBatchCacheLen = 5;
// Largest system a wavefront solves alone in the wavefront mode: four rows
// per lane in registers.
constexpr int kWaveRows = 4 * 64;

size_t batch_lds_bytes(vt t, int64_t max_m, bool lean, bool waves, int block);
// Whether the wavefront mode can run: FP64 with the direction-only layout
// (lean), FP32 storage when every row fits the register cache.
bool batch_waves_fit(vt t, bool lean, int64_t max_row_len);
// Whether every system of the batch fits the register cache at this
// workgroup size (FP64 only), so that only p needs LDS.
bool batch_lean_fits(vt t, int block, int64_t max_m, int64_t max_row_len);
// err[0]: set to 1 on a malformed system; err[1]: atomicMax of the longest
// row (both must start at zero).
hipError_t batch_validate(hipStream_t s, int64_t nsys, const int64_t *row_off,
                          const int64_t *nnz_off, const int32_t *rp_local, const int32_t *col,
                          int *err);
hipError_t batch_cg(hipStream_t s, vt t, const batch_args &a);
// Workgroups of the persistent kernel resident at once (its grid for batches
// of at least that many systems).
hipError_t batch_resident(vt t, int block, int64_t max_m, bool lean, bool waves, int *workgroups);

}  // namespace gko
