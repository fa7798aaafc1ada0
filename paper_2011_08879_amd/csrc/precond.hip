// Block-Jacobi preconditioner setup: explicit inverses of the diagonal blocks
// of bs consecutive rows.  A subwarp of bs lanes owns one block; lane i keeps
// row i of the augmented matrix [D | I] in registers and Gauss-Jordan
// elimination with partial pivoting (ties to the smaller row) proceeds column
// by column: an argmax over the subwarp picks the pivot, two lanes swap rows
// by shuffles, the pivot row is scaled and broadcast, and every other lane
// eliminates.  Multiplies and subtractions are not fused, so the result
// follows the textbook rounding step by step.
#include <cmath>

#include "device.hpp"
#include "solver_kernels.hpp"

namespace gko {

template <int BS>
__global__ __launch_bounds__(256) void bj_invert_kernel(int64_t n, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col,
                                                        const double *__restrict__ val,
                                                        double *__restrict__ inv, int *err) {
#pragma clang fp contract(off)
    const int64_t blk = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / BS;
    const int i = threadIdx.x % BS;
    const int64_t nb = (n + BS - 1) / BS;
    if (blk >= nb) return;  // uniform across the subwarp
    const int64_t r0 = blk * BS;
    const int m = (int)(r0 + BS <= n ? BS : n - r0);
    double a[BS], e[BS];
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        a[j] = 0.0;
        e[j] = (j == i && i < m) ? 1.0 : 0.0;
    }
    if (i < m)
        for (int32_t k = rp[r0 + i]; k < rp[r0 + i + 1]; ++k) {
            const int64_t c = (int64_t)col[k] - r0;
#pragma unroll
            for (int j = 0; j < BS; ++j)
                if (c == j && j < m) a[j] = val[k];
        }
    bool singular = false;
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        if (c < m && !singular) {
            double mag = (i >= c && i < m) ? fabs(a[c]) : -1.0;
            int who = i;
#pragma unroll
            for (int b = 1; b < BS; b <<= 1) {
                const double om = __shfl_xor(mag, b, BS);
                const int ow = __shfl_xor(who, b, BS);
                if (om > mag || (om == mag && ow < who)) {
                    mag = om;
                    who = ow;
                }
            }
            if (mag == 0.0) {
                singular = true;
            } else {
                const int piv = who;
                if (piv != c) {
#pragma unroll
                    for (int j = 0; j < BS; ++j) {
                        const double ap = __shfl(a[j], piv, BS), ac = __shfl(a[j], c, BS);
                        const double ep = __shfl(e[j], piv, BS), ec = __shfl(e[j], c, BS);
                        if (i == c) { a[j] = ap; e[j] = ep; }
                        else if (i == piv) { a[j] = ac; e[j] = ec; }
                    }
                }
                const double d = __shfl(a[c], c, BS);
                if (i == c) {
#pragma unroll
                    for (int j = 0; j < BS; ++j) {
                        a[j] = a[j] / d;
                        e[j] = e[j] / d;
                    }
                }
                const double f = a[c];
#pragma unroll
                for (int j = 0; j < BS; ++j) {
                    const double ra = __shfl(a[j], c, BS), re = __shfl(e[j], c, BS);
                    if (i != c && f != 0.0) {
                        a[j] = a[j] - f * ra;
                        e[j] = e[j] - f * re;
                    }
                }
            }
        }
    }
    if (singular) {
        if (i == 0) atomicOr(err, 1);
        return;
    }
#pragma unroll
    for (int j = 0; j < BS; ++j) inv[blk * BS * BS + (int64_t)i * BS + j] = e[j];
}

template <int BS>
static hipError_t launch_bj(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                            const double *val, double *inv, int *err) {
    const int64_t nb = (n + BS - 1) / BS;
    const int64_t threads = nb * BS;
    bj_invert_kernel<BS><<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(n, rp, col, val, inv, err);
    return hipGetLastError();
}

// Upper triangle of each inverse block, row by row: entry (i, j), j >= i,
// of block k goes to k P + i bs - i (i - 1) / 2 + (j - i), P = bs (bs + 1) / 2.
__global__ void bj_pack_kernel(int64_t nb, int bs, const double *__restrict__ full,
                               double *__restrict__ packed) {
    const int P = bs * (bs + 1) / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nb * P) return;
    const int64_t k = g / P;
    int t = (int)(g % P), i = 0;
    while (t >= bs - i) {
        t -= bs - i;
        ++i;
    }
    packed[g] = full[k * bs * bs + (int64_t)i * bs + i + t];
}

hipError_t bj_pack_upper(hipStream_t s, int64_t nb, int bs, const double *full, double *packed) {
    const int64_t total = nb * (int64_t)(bs * (bs + 1) / 2);
    if (total == 0) return hipSuccess;
    bj_pack_kernel<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(nb, bs, full, packed);
    return hipGetLastError();
}

hipError_t bj_invert(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                     const double *val, int bs, double *inv, int *err) {
    if (n == 0) return hipSuccess;
    switch (bs) {
        case 1: return launch_bj<1>(s, n, rp, col, val, inv, err);
        case 2: return launch_bj<2>(s, n, rp, col, val, inv, err);
        case 4: return launch_bj<4>(s, n, rp, col, val, inv, err);
        case 8: return launch_bj<8>(s, n, rp, col, val, inv, err);
        case 16: return launch_bj<16>(s, n, rp, col, val, inv, err);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gko
