// Host-side launchers of the selector kernels (selector.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gko {

constexpr int kFeatCounters = 12;
constexpr int kNumFeatures = 32;
// One output per SpMV format scored: CSR, CSR merge, COO, ELL, HYB, SELL-P.
constexpr int kMlpIn = 32, kMlpHidden = 64, kMlpOut = 6;
constexpr int kMlpParams = kMlpHidden * kMlpIn + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden +
                           kMlpOut * kMlpHidden + kMlpOut;  // 6662
constexpr int kMlpMaxBlocks = 128;

// Exact integer counters over the entries (see selector.hip); cnt: 12 zeroed uint64.
hipError_t feature_counts(hipStream_t s, int64_t n, int64_t m, const int32_t *rp,
                          const int32_t *col, unsigned long long *cnt);

// Device scratch of the training kernel.
struct mlp_work {
    double *msum;     // sum of the mask
    float *grads;     // kMlpMaxBlocks * kMlpParams
    double *lossp;    // kMlpMaxBlocks
    unsigned *ticket; // zeroed
    float *adam_m, *adam_v;
    int *step;        // Adam steps taken
};

hipError_t mlp_forward(hipStream_t s, int64_t n, const float *X, const float *params,
                       const float *norm, float *out);
hipError_t mlp_mask_sum(hipStream_t s, int64_t count, const float *M, double *out);
hipError_t mlp_norm_fit(hipStream_t s, int64_t n, const float *X, float *norm);
hipError_t mlp_grad(hipStream_t s, const mlp_work &w, int64_t n, const float *X, const float *Y,
                    const float *M, float *params, const float *norm, float *grad_out,
                    double *loss_out, bool adam, float lr, float *loss_hist);

}  // namespace gko
