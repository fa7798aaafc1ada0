// Learned format selector: structural features of a CSR matrix and a small
// MLP (32 -> 64 -> 64 -> 6, ReLU) trained with Adam, all in FP32 on the
// vector ALUs (the network is far too small for matrix cores to matter).
//
// Features: the row-length statistics come from the row-length histogram;
// everything that needs the entries (distances to the diagonal, column gaps,
// touched 64-byte x segments, pattern symmetry, row spans) is accumulated
// here as exact integer sums, so the result does not depend on scheduling.
//
// Training: one launch per full-batch Adam step.  Each workgroup takes tiles
// of 32 samples, runs the forward and backward passes through LDS, and
// accumulates the gradients of the parameters its threads own in a fixed
// sample order; per-workgroup gradients are summed in workgroup order by the
// last workgroup to finish, which also applies the Adam update.
#include <cmath>

#include "device.hpp"
#include "selector_kernels.hpp"

namespace gko {

// ====================================================================== features
// counters: 0 sum|i-j|  1 max|i-j|  2 diag  3 |i-j|<=1  4 |i-j|<=64  5 sum gaps
// 6 pairs  7 gap==1  8 x segments  9 symmetric  10 sum spans  11 nonempty rows
__device__ inline bool row_has(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                               int64_t row, int32_t c) {
    int32_t lo = rp[row], hi = rp[row + 1];
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo < rp[row + 1] && col[lo] == c;
}

constexpr int kFeatW = 32;  // lanes per row

__global__ __launch_bounds__(256) void feature_counts_kernel(int64_t n, int64_t m,
                                                             const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col,
                                                             unsigned long long *cnt) {
    __shared__ unsigned long long lds[kFeatCounters][256 / kWave];
    unsigned long long c[kFeatCounters];
#pragma unroll
    for (int j = 0; j < kFeatCounters; ++j) c[j] = 0ull;
    const int lane = threadIdx.x % kFeatW;
    const int64_t per_block = 256 / kFeatW;
    for (int64_t i = (int64_t)blockIdx.x * per_block + threadIdx.x / kFeatW; i < n;
         i += (int64_t)gridDim.x * per_block) {
        const int32_t b = rp[i], e = rp[i + 1];
        if (lane == 0 && e > b) {
            c[10] += (unsigned long long)((int64_t)col[e - 1] - col[b] + 1);
            c[11] += 1;
        }
        for (int32_t k = b + lane; k < e; k += kFeatW) {
            const int32_t cj = col[k];
            int64_t d = (int64_t)cj - i;
            if (d < 0) d = -d;
            c[0] += (unsigned long long)d;
            if ((unsigned long long)d > c[1]) c[1] = (unsigned long long)d;
            c[2] += d == 0;
            c[3] += d <= 1;
            c[4] += d <= 64;
            if (k > b) {
                const int32_t cp = col[k - 1];
                c[5] += (unsigned long long)((int64_t)cj - cp);
                c[6] += 1;
                c[7] += (cj - cp) == 1;
                c[8] += (cj / 8) != (cp / 8);
            } else {
                c[8] += 1;
            }
            if (n == m && cj < n) c[9] += row_has(rp, col, cj, (int32_t)i);
        }
    }
    // block reduction: wave butterfly (sum, max for counter 1), then LDS
#pragma unroll
    for (int j = 0; j < kFeatCounters; ++j) {
        unsigned long long v = c[j];
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const unsigned long long u = __shfl_xor(v, o);
            v = (j == 1) ? (u > v ? u : v) : v + u;
        }
        if (threadIdx.x % kWave == 0) lds[j][threadIdx.x / kWave] = v;
    }
    __syncthreads();
    if (threadIdx.x < kFeatCounters) {
        const int j = threadIdx.x;
        unsigned long long v = 0;
        for (int w = 0; w < 256 / kWave; ++w)
            v = (j == 1) ? (lds[j][w] > v ? lds[j][w] : v) : v + lds[j][w];
        if (j == 1) atomicMax(cnt + 1, v);
        else atomicAdd(cnt + j, v);
    }
}

hipError_t feature_counts(hipStream_t s, int64_t n, int64_t m, const int32_t *rp,
                          const int32_t *col, unsigned long long *cnt) {
    if (n == 0) return hipSuccess;
    int64_t g = (n + 7) / 8;
    if (g > 4096) g = 4096;
    feature_counts_kernel<<<(unsigned)g, 256, 0, s>>>(n, m, rp, col, cnt);
    return hipGetLastError();
}

// ====================================================================== MLP
constexpr int NI = kMlpIn, NH = kMlpHidden, NO = kMlpOut, NP = kMlpParams;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NO * NH;
constexpr int kT = 256;      // threads per workgroup
constexpr int kS = 32;       // samples per tile
constexpr int kOwn = (NP + kT - 1) / kT;  // parameters owned per thread

struct mlp_lds {
    float W[NP];
    float X[kS][NI];
    float H1[kS][NH];   // activations, then their gradients
    float H2[kS][NH];
    float O[kS][NO];    // outputs, then dL/do
    float mean[NI], inv_std[NI];
};

// Forward pass of one tile (samples s0 .. s0+kS-1 of n), inputs normalised.
__device__ inline void tile_forward(mlp_lds &L, int64_t s0, int64_t n, const float *__restrict__ X) {
    const int t = threadIdx.x;
    for (int e = t; e < kS * NI; e += kT) {
        const int s = e / NI, k = e % NI;
        const int64_t g = s0 + s;
        L.X[s][k] = g < n ? (X[g * NI + k] - L.mean[k]) * L.inv_std[k] : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < kS * NH; e += kT) {
        const int s = e / NH, j = e % NH;
        float a = L.W[OFF_B1 + j];
        for (int k = 0; k < NI; ++k) a += L.W[OFF_W1 + j * NI + k] * L.X[s][k];
        L.H1[s][j] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < kS * NH; e += kT) {
        const int s = e / NH, j = e % NH;
        float a = L.W[OFF_B2 + j];
        for (int k = 0; k < NH; ++k) a += L.W[OFF_W2 + j * NH + k] * L.H1[s][k];
        L.H2[s][j] = a > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    for (int e = t; e < kS * NO; e += kT) {
        const int s = e / NO, j = e % NO;
        float a = L.W[OFF_B3 + j];
        for (int k = 0; k < NH; ++k) a += L.W[OFF_W3 + j * NH + k] * L.H2[s][k];
        L.O[s][j] = a;
    }
    __syncthreads();
}

__device__ inline void load_model(mlp_lds &L, const float *__restrict__ params,
                                  const float *__restrict__ norm) {
    for (int i = threadIdx.x; i < NP; i += kT) L.W[i] = params[i];
    for (int i = threadIdx.x; i < NI; i += kT) {
        L.mean[i] = norm[i];
        L.inv_std[i] = 1.0f / norm[NI + i];
    }
    __syncthreads();
}

__global__ __launch_bounds__(kT) void mlp_forward_kernel(int64_t n, const float *__restrict__ X,
                                                         const float *__restrict__ params,
                                                         const float *__restrict__ norm,
                                                         float *__restrict__ out) {
    __shared__ mlp_lds L;
    load_model(L, params, norm);
    for (int64_t s0 = (int64_t)blockIdx.x * kS; s0 < n; s0 += (int64_t)gridDim.x * kS) {
        tile_forward(L, s0, n, X);
        for (int e = threadIdx.x; e < kS * NO; e += kT) {
            const int64_t g = s0 + e / NO;
            if (g < n) out[g * NO + e % NO] = L.O[e / NO][e % NO];
        }
        __syncthreads();
    }
}

// Gradient of the masked mean squared loss.  grads: gridDim.x * NP partial
// sums; lossp: gridDim.x partial losses.  The last workgroup reduces them in
// workgroup order into grad_out / loss_out and, if adam, updates the model.
__global__ __launch_bounds__(kT) void mlp_grad_kernel(
    int64_t n, const float *__restrict__ X, const float *__restrict__ Y,
    const float *__restrict__ M, float *__restrict__ params, const float *__restrict__ norm,
    const double *__restrict__ msum, float *__restrict__ grads, double *__restrict__ lossp,
    unsigned *ticket, float *__restrict__ grad_out, double *__restrict__ loss_out, bool adam,
    float *__restrict__ am, float *__restrict__ av, int *__restrict__ step, float lr,
    float *__restrict__ loss_hist) {
    __shared__ mlp_lds L;
    __shared__ double red[kT / kWave];
    __shared__ bool last;
    load_model(L, params, norm);
    const int t = threadIdx.x;
    const float inv_m = (float)(1.0 / *msum);
    float g[kOwn];
#pragma unroll
    for (int q = 0; q < kOwn; ++q) g[q] = 0.0f;
    double loss = 0.0;
    for (int64_t s0 = (int64_t)blockIdx.x * kS; s0 < n; s0 += (int64_t)gridDim.x * kS) {
        tile_forward(L, s0, n, X);
        // dL/do = 2 mask (o - y) / sum(mask)
        for (int e = t; e < kS * NO; e += kT) {
            const int s = e / NO, j = e % NO;
            const int64_t gs = s0 + s;
            float d = 0.0f;
            if (gs < n) {
                const float r = L.O[s][j] - Y[gs * NO + j];
                const float mk = M[gs * NO + j];
                loss += (double)mk * (double)r * (double)r;
                d = 2.0f * mk * r * inv_m;
            }
            L.O[s][j] = d;
        }
        __syncthreads();
        // W3, b3 (use H2 activations)
#pragma unroll
        for (int q = 0; q < kOwn; ++q) {
            const int p = t + q * kT;
            if (p >= OFF_W3 && p < NP) {
                float a = 0.0f;
                if (p < OFF_B3) {
                    const int j = (p - OFF_W3) / NH, k = (p - OFF_W3) % NH;
                    for (int s = 0; s < kS; ++s) a += L.O[s][j] * L.H2[s][k];
                } else {
                    for (int s = 0; s < kS; ++s) a += L.O[s][p - OFF_B3];
                }
                g[q] += a;
            }
        }
        __syncthreads();
        // dH2 = (W3^T dO) * [H2 > 0], in place
        for (int e = t; e < kS * NH; e += kT) {
            const int s = e / NH, k = e % NH;
            float a = 0.0f;
            for (int j = 0; j < NO; ++j) a += L.W[OFF_W3 + j * NH + k] * L.O[s][j];
            L.H2[s][k] = L.H2[s][k] > 0.0f ? a : 0.0f;
        }
        __syncthreads();
        // W2, b2 (use dH2 and H1 activations)
#pragma unroll
        for (int q = 0; q < kOwn; ++q) {
            const int p = t + q * kT;
            if (p >= OFF_W2 && p < OFF_W3) {
                float a = 0.0f;
                if (p < OFF_B2) {
                    const int j = (p - OFF_W2) / NH, k = (p - OFF_W2) % NH;
                    for (int s = 0; s < kS; ++s) a += L.H2[s][j] * L.H1[s][k];
                } else {
                    for (int s = 0; s < kS; ++s) a += L.H2[s][p - OFF_B2];
                }
                g[q] += a;
            }
        }
        __syncthreads();
        // dH1 = (W2^T dH2) * [H1 > 0], in place
        for (int e = t; e < kS * NH; e += kT) {
            const int s = e / NH, k = e % NH;
            float a = 0.0f;
            for (int j = 0; j < NH; ++j) a += L.W[OFF_W2 + j * NH + k] * L.H2[s][j];
            L.H1[s][k] = L.H1[s][k] > 0.0f ? a : 0.0f;
        }
        __syncthreads();
        // W1, b1 (use dH1 and the normalised inputs)
#pragma unroll
        for (int q = 0; q < kOwn; ++q) {
            const int p = t + q * kT;
            if (p < OFF_W2) {
                float a = 0.0f;
                if (p < OFF_B1) {
                    const int j = p / NI, k = p % NI;
                    for (int s = 0; s < kS; ++s) a += L.H1[s][j] * L.X[s][k];
                } else {
                    for (int s = 0; s < kS; ++s) a += L.H1[s][p - OFF_B1];
                }
                g[q] += a;
            }
        }
        __syncthreads();
    }
    // per-workgroup partials
#pragma unroll
    for (int q = 0; q < kOwn; ++q) {
        const int p = t + q * kT;
        if (p < NP) grads[(size_t)blockIdx.x * NP + p] = g[q];
    }
    const double bl = block_sum<kT>(loss, red);
    if (t == 0) {
        lossp[blockIdx.x] = bl;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    // the last workgroup: reduce in workgroup order, then (optionally) Adam
    int tstep = 0;
    if (adam) tstep = *step + 1;
    const float c1 = 1.0f - powf(0.9f, (float)tstep), c2 = 1.0f - powf(0.999f, (float)tstep);
    for (int p = t; p < NP; p += kT) {
        double a = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b) {
            const uint32_t bits = __hip_atomic_load(reinterpret_cast<const uint32_t *>(grads) + (size_t)b * NP + p,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            a += (double)__uint_as_float(bits);
        }
        const float gp = (float)a;
        if (grad_out) grad_out[p] = gp;
        if (adam) {
            const float mm = 0.9f * am[p] + 0.1f * gp;
            const float vv = 0.999f * av[p] + 0.001f * gp * gp;
            am[p] = mm;
            av[p] = vv;
            params[p] = params[p] - lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
        }
    }
    if (t == 0) {
        double tot = 0.0;
        for (unsigned b = 0; b < gridDim.x; ++b) tot += load_coherent(lossp + b);
        const double lv = tot / *msum;
        if (loss_out) *loss_out = lv;
        if (adam) {
            if (loss_hist) loss_hist[*step] = (float)lv;
            *step = tstep;
        }
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void mask_sum_kernel(int64_t count, const float *__restrict__ M, double *out) {
    __shared__ double red[256 / kWave];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) s += (double)M[i];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) *out = s;
}

// Per-feature mean and standard deviation (population), std floored at 1e-6.
__global__ void norm_fit_kernel(int64_t n, const float *__restrict__ X, float *__restrict__ norm) {
    __shared__ double red[256 / kWave];
    __shared__ double s_mean;
    for (int k = 0; k < NI; ++k) {
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)X[i * NI + k];
        s = block_sum<256>(s, red);   // valid in thread 0
        if (threadIdx.x == 0) s_mean = s / (double)(n > 0 ? n : 1);
        __syncthreads();
        const double mean = s_mean;
        double v = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += 256) {
            const double d = (double)X[i * NI + k] - mean;
            v += d * d;
        }
        const double var = block_sum<256>(v, red) / (double)(n > 0 ? n : 1);
        if (threadIdx.x == 0) {
            norm[k] = (float)mean;
            const double sd = sqrt(var);
            norm[NI + k] = (float)(sd > 1e-6 ? sd : 1e-6);
        }
        __syncthreads();   // s_mean is rewritten for the next feature
    }
}

static unsigned grad_blocks(int64_t n) {
    int64_t g = (n + kS - 1) / kS;
    if (g > kMlpMaxBlocks) g = kMlpMaxBlocks;
    if (g < 1) g = 1;
    return (unsigned)g;
}

hipError_t mlp_forward(hipStream_t s, int64_t n, const float *X, const float *params,
                       const float *norm, float *out) {
    if (n == 0) return hipSuccess;
    mlp_forward_kernel<<<grad_blocks(n), kT, 0, s>>>(n, X, params, norm, out);
    return hipGetLastError();
}

hipError_t mlp_mask_sum(hipStream_t s, int64_t count, const float *M, double *out) {
    mask_sum_kernel<<<1, 256, 0, s>>>(count, M, out);
    return hipGetLastError();
}

hipError_t mlp_norm_fit(hipStream_t s, int64_t n, const float *X, float *norm) {
    norm_fit_kernel<<<1, 256, 0, s>>>(n, X, norm);
    return hipGetLastError();
}

hipError_t mlp_grad(hipStream_t s, const mlp_work &w, int64_t n, const float *X, const float *Y,
                    const float *M, float *params, const float *norm, float *grad_out,
                    double *loss_out, bool adam, float lr, float *loss_hist) {
    mlp_grad_kernel<<<grad_blocks(n), kT, 0, s>>>(n, X, Y, M, params, norm, w.msum, w.grads,
                                                  w.lossp, w.ticket, grad_out, loss_out, adam,
                                                  w.adam_m, w.adam_v, w.step, lr, loss_hist);
    return hipGetLastError();
}

}  // namespace gko
