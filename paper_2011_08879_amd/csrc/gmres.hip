// Restarted GMRES(m), FP64, unpreconditioned (Saad and Schultz 1986; Saad,
// Iterative Methods, Alg. 6.9 with the Givens least-squares update of
// Sec. 6.5.3).
//
// Arnoldi step j with w = A v_j written straight into basis slot j+1:
//   dot         h = V_j^T w and w.w in one pass over the j+1 basis vectors
//   update+dot  w -= V_j h, then h' = V_j^T w and the new w.w, in one pass
//               (each thread re-reads its rows of V_j right after the
//               update, mostly from the caches)
//   update      w -= V_j h' (classical Gram-Schmidt twice) only when the
//               first round shrank w below 1/sqrt(2) of its length (Daniel,
//               Gragg, Kaufman and Stewart's criterion); otherwise the
//               launch returns at once
//   step        (one thread) the column of H, the earlier rotations, the new
//               Givens rotation, |g_{j+1}| as the residual estimate, the end
//               of the cycle
//   normalise   v_{j+1} = w / h_{j+1,j}
// The basis is column-major with a leading dimension rounded up to 64
// doubles.  The multi-vector passes keep each thread's rows of w in
// registers and read the basis vectors coalesced, one after another; the
// per-vector sums are wave DPP reductions accumulated per wave in LDS, then
// per-block partials summed in block order by a one-block-per-value kernel,
// so every result repeats bitwise.  A cycle ends with the back substitution
// (one thread) and x += V_k y in one pass.
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"
#include "solver_state.hpp"

namespace gko {

namespace {

constexpr int kG = 256;          // threads per workgroup
constexpr int kGRows = 4;        // rows per thread per chunk
constexpr int kGWaves = kG / kWave;

inline int gmres_blocks(int64_t n) {
    int64_t g = (n + (int64_t)kG * kGRows - 1) / ((int64_t)kG * kGRows);
    if (g > kGmresMaxBlocks) g = kGmresMaxBlocks;
    return g < 1 ? 1 : (int)g;
}

// Phase gates.  mode 0: the passes of an Arnoldi step run only while the
// cycle is open; mode 1: the second Gram-Schmidt round also needs the step
// to have asked for it; mode 2 (cycle start): while the solve runs.
__device__ inline bool gate(const gmres_state *st, int mode) {
    if (mode == 2) return st->done == kRunning;
    return st->cycle_done == 0 && (mode == 0 || st->reorth != 0);
}

// partials[v * gridDim.x + block] <- block sums of V_i . w (v = i < k) and of
// w . w (v = k)
__global__ __launch_bounds__(kG) void gmres_dot_kernel(int64_t n, int k, const double *__restrict__ V,
                                                       int64_t ldv, const double *__restrict__ w,
                                                       const gmres_state *st, int mode,
                                                       double *__restrict__ partials) {
    __shared__ double part[kGmresMaxKrylov + 1][kGWaves];
    if (!gate(st, mode)) return;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int e = threadIdx.x; e < (k + 1) * kGWaves; e += kG) part[e / kGWaves][e % kGWaves] = 0.0;
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kG * kGRows; base < n;
         base += (int64_t)gridDim.x * kG * kGRows) {
        double wr[kGRows];
        double ww = 0.0;
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int64_t l = base + r * kG + threadIdx.x;
            wr[r] = l < n ? w[l] : 0.0;
            ww += wr[r] * wr[r];
        }
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (int64_t)i * ldv;
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < kGRows; ++r) {
                const int64_t l = base + r * kG + threadIdx.x;
                s += (l < n ? vi[l] : 0.0) * wr[r];
            }
            s = wave_total(s);
            if (lane == 0) part[i][wv] += s;
        }
        ww = wave_total(ww);
        if (lane == 0) part[k][wv] += ww;
    }
    __syncthreads();
    for (int v = threadIdx.x; v <= k; v += kG) {
        double s = 0.0;
        for (int q = 0; q < kGWaves; ++q) s += part[v][q];
        partials[(int64_t)v * gridDim.x + blockIdx.x] = s;
    }
}

// w -= sum_i h_i V_i (i ascending), block sums of the new w . w
__global__ __launch_bounds__(kG) void gmres_update_kernel(int64_t n, int k,
                                                          const double *__restrict__ V,
                                                          int64_t ldv, const double *__restrict__ h,
                                                          double *__restrict__ w,
                                                          const gmres_state *st, int mode,
                                                          double *__restrict__ partials) {
    __shared__ double hs[kGmresMaxKrylov];
    __shared__ double red[kGWaves];
    if (!gate(st, mode)) return;
    for (int i = threadIdx.x; i < k; i += kG) hs[i] = h[i];
    __syncthreads();
    double ww = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kG * kGRows; base < n;
         base += (int64_t)gridDim.x * kG * kGRows) {
        double acc[kGRows];
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int64_t l = base + r * kG + threadIdx.x;
            acc[r] = l < n ? w[l] : 0.0;
        }
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (int64_t)i * ldv;
            const double hi = hs[i];
#pragma unroll
            for (int r = 0; r < kGRows; ++r) {
                const int64_t l = base + r * kG + threadIdx.x;
                if (l < n) acc[r] = acc[r] - hi * vi[l];
            }
        }
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int64_t l = base + r * kG + threadIdx.x;
            if (l < n) {
                w[l] = acc[r];
                ww += acc[r] * acc[r];
            }
        }
    }
    ww = block_sum<kG>(ww, red);
    if (threadIdx.x == 0) partials[blockIdx.x] = ww;
}

// The first round's update fused with the second round's dots:
// w -= sum_i h_i V_i, then partials of V_i . w (i < k) and w . w (at k) for
// the new w.  The second read of each V_i[l] follows the first within the
// same thread's chunk, so it mostly hits the caches instead of HBM.
__global__ __launch_bounds__(kG) void gmres_update_dot_kernel(int64_t n, int k,
                                                              const double *__restrict__ V,
                                                              int64_t ldv,
                                                              const double *__restrict__ h,
                                                              double *__restrict__ w,
                                                              const gmres_state *st,
                                                              double *__restrict__ partials) {
    __shared__ double part[kGmresMaxKrylov + 1][kGWaves];
    __shared__ double hs[kGmresMaxKrylov];
    if (!gate(st, 0)) return;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int e = threadIdx.x; e < (k + 1) * kGWaves; e += kG) part[e / kGWaves][e % kGWaves] = 0.0;
    for (int i = threadIdx.x; i < k; i += kG) hs[i] = h[i];
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kG * kGRows; base < n;
         base += (int64_t)gridDim.x * kG * kGRows) {
        double acc[kGRows];
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int64_t l = base + r * kG + threadIdx.x;
            acc[r] = l < n ? w[l] : 0.0;
        }
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (int64_t)i * ldv;
            const double hi = hs[i];
#pragma unroll
            for (int r = 0; r < kGRows; ++r) {
                const int64_t l = base + r * kG + threadIdx.x;
                if (l < n) acc[r] = acc[r] - hi * vi[l];
            }
        }
        double ww = 0.0;
#pragma unroll
        for (int r = 0; r < kGRows; ++r) {
            const int64_t l = base + r * kG + threadIdx.x;
            if (l < n) w[l] = acc[r];
            ww += acc[r] * acc[r];
        }
        // newest vectors first: they were read last, so the most of them are
        // still in the caches (each V_i . w is formed on its own, so the
        // order changes no result)
        for (int i = k - 1; i >= 0; --i) {
            const double *vi = V + (int64_t)i * ldv;
            double sd = 0.0;
#pragma unroll
            for (int r = 0; r < kGRows; ++r) {
                const int64_t l = base + r * kG + threadIdx.x;
                sd += (l < n ? vi[l] : 0.0) * acc[r];
            }
            sd = wave_total(sd);
            if (lane == 0) part[i][wv] += sd;
        }
        ww = wave_total(ww);
        if (lane == 0) part[k][wv] += ww;
    }
    __syncthreads();
    for (int v = threadIdx.x; v <= k; v += kG) {
        double sum = 0.0;
        for (int q = 0; q < kGWaves; ++q) sum += part[v][q];
        partials[(int64_t)v * gridDim.x + blockIdx.x] = sum;
    }
}

// The same for k <= kGRegVecs with one row per thread per chunk: the
// thread's element of every V_i stays in registers between the update and
// the dots, so V is read once (the loops are unrolled to kGRegVecs so the
// register array is indexed statically).
constexpr int kGRegVecs = 32;

__global__ __launch_bounds__(kG) void gmres_update_dot_regs_kernel(int64_t n, int k,
                                                                   const double *__restrict__ V,
                                                                   int64_t ldv,
                                                                   const double *__restrict__ h,
                                                                   double *__restrict__ w,
                                                                   const gmres_state *st,
                                                                   double *__restrict__ partials) {
    __shared__ double part[kGRegVecs + 1][kGWaves];
    __shared__ double hs[kGRegVecs];
    if (!gate(st, 0)) return;
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    for (int e = threadIdx.x; e < (k + 1) * kGWaves; e += kG) part[e / kGWaves][e % kGWaves] = 0.0;
    for (int i = threadIdx.x; i < k; i += kG) hs[i] = h[i];
    __syncthreads();
    for (int64_t base = (int64_t)blockIdx.x * kG; base < n; base += (int64_t)gridDim.x * kG) {
        const int64_t l = base + threadIdx.x;
        const bool ok = l < n;
        double vr[kGRegVecs];
        double acc = ok ? w[l] : 0.0;
#pragma unroll
        for (int i = 0; i < kGRegVecs; ++i) {
            vr[i] = (i < k && ok) ? V[(int64_t)i * ldv + l] : 0.0;
            acc = acc - (i < k ? hs[i] : 0.0) * vr[i];
        }
        if (ok) w[l] = acc;
#pragma unroll
        for (int i = 0; i < kGRegVecs; ++i) {
            if (i < k) {  // uniform
                const double sd = wave_total(vr[i] * acc);
                if (lane == 0) part[i][wv] += sd;
            }
        }
        const double ww = wave_total(acc * acc);
        if (lane == 0) part[k][wv] += ww;
    }
    __syncthreads();
    for (int v = threadIdx.x; v <= k; v += kG) {
        double sum = 0.0;
        for (int q = 0; q < kGWaves; ++q) sum += part[v][q];
        partials[(int64_t)v * gridDim.x + blockIdx.x] = sum;
    }
}

// out[v] <- sum over blocks of partials[v * g + b], block order, one
// workgroup per value
__global__ __launch_bounds__(kG) void gmres_sum_kernel(int g, const double *__restrict__ partials,
                                                       double *__restrict__ out,
                                                       const gmres_state *st, int mode) {
    __shared__ double red[kGWaves];
    if (!gate(st, mode)) return;
    const double *p = partials + (int64_t)blockIdx.x * g;
    double s = 0.0;
    for (int b = threadIdx.x; b < g; b += kG) s += p[b];
    s = block_sum<kG>(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// After the first round: keep h, decide on a second round.  dot1: V^T w
// and w.w before the round; dot2: V^T w and w.w after it.
__global__ void gmres_check_kernel(int j, const double *__restrict__ dot1,
                                   const double *__restrict__ dot2, gmres_state *st,
                                   double *__restrict__ hcol) {
    if (st->cycle_done) return;
    for (int i = 0; i <= j; ++i) hcol[i] = dot1[i];
    // |w_after| < |w_before| / sqrt(2)
    st->reorth = (2.0 * dot2[j + 1] < dot1[j + 1]) ? 1 : 0;
    st->reorths += st->reorth;
    st->ww = dot2[j + 1];
}

// Close step j: h_{j+1,j}, rotations, residual estimate, end of cycle.
__global__ void gmres_step_kernel(int j, int m, const double *__restrict__ dot2,
                                  const double *__restrict__ upd2, gmres_state *st,
                                  double *__restrict__ hcol, double *__restrict__ H,
                                  double *__restrict__ cs, double *__restrict__ sn,
                                  double *__restrict__ gv) {
    if (st->cycle_done) return;
    double ww = st->ww;
    if (st->reorth) {
        for (int i = 0; i <= j; ++i) hcol[i] = hcol[i] + dot2[i];
        ww = upd2[0];
    }
    const double hn = sqrt(ww);
    for (int i = 0; i < j; ++i) {
        const double a = hcol[i], c = hcol[i + 1];
        hcol[i] = cs[i] * a + sn[i] * c;
        hcol[i + 1] = -sn[i] * a + cs[i] * c;
    }
    const double a = hcol[j];
    const double d = sqrt(a * a + hn * hn);
    st->iter += 1;
    st->k = j + 1;
    if (!(d > 0.0)) {
        st->done = kBreakdown;
        st->cycle_done = 1;
        return;
    }
    cs[j] = a / d;
    sn[j] = hn / d;
    hcol[j] = d;
    for (int i = 0; i <= j; ++i) H[(int64_t)i * m + j] = hcol[i];
    H[(int64_t)(j + 1) * m + j] = 0.0;
    gv[j + 1] = -sn[j] * gv[j];
    gv[j] = cs[j] * gv[j];
    const double est = fabs(gv[j + 1]);
    st->est = est;
    st->hn = hn;
    if (std::isnan(est)) {
        st->done = kBreakdown;
        st->cycle_done = 1;
    } else if (est <= st->stop || hn == 0.0 || st->iter >= st->maxit || j + 1 == m) {
        st->cycle_done = 1;
    }
}

__global__ __launch_bounds__(kG) void gmres_scale_kernel(int64_t n, double *__restrict__ v,
                                                         const gmres_state *st) {
    if (st->cycle_done) return;
    const double hn = st->hn;
    for (int64_t l = (int64_t)blockIdx.x * kG + threadIdx.x; l < n; l += (int64_t)gridDim.x * kG)
        v[l] = v[l] / hn;
}

// Back substitution R y = g over the cycle's k columns.
__global__ void gmres_solve_kernel(int m, const double *__restrict__ H,
                                   const double *__restrict__ gv, double *__restrict__ y,
                                   const gmres_state *st) {
    if (st->done == kBreakdown) return;
    const int k = st->k;
    for (int i = k - 1; i >= 0; --i) {
        double s = gv[i];
        for (int l = i + 1; l < k; ++l) s = s - H[(int64_t)i * m + l] * y[l];
        y[i] = s / H[(int64_t)i * m + i];
    }
}

// x += sum_i y_i V_i (i ascending)
__global__ __launch_bounds__(kG) void gmres_xupdate_kernel(int64_t n, const double *__restrict__ V,
                                                           int64_t ldv,
                                                           const double *__restrict__ y,
                                                           double *__restrict__ x,
                                                           const gmres_state *st) {
    __shared__ double ys[kGmresMaxKrylov];
    if (st->done == kBreakdown) return;
    const int k = st->k;
    for (int i = threadIdx.x; i < k; i += kG) ys[i] = y[i];
    __syncthreads();
    for (int64_t l = (int64_t)blockIdx.x * kG + threadIdx.x; l < n; l += (int64_t)gridDim.x * kG) {
        double xl = x[l];
        for (int i = 0; i < k; ++i) xl = xl + ys[i] * V[(int64_t)i * ldv + l];
        x[l] = xl;
    }
}

// Cycle start from v0 = b - A x (unnormalised) and its squared norm.
__global__ void gmres_cycle_kernel(const double *__restrict__ rr, gmres_state *st,
                                   double *__restrict__ gv) {
    if (st->done != kRunning) return;
    const double beta = sqrt(rr[0]);
    st->beta = beta;
    st->cycle_done = 0;
    st->reorth = 0;
    st->k = 0;
    st->hn = beta;   // v0 = r / beta by the scale kernel
    gv[0] = beta;
    if (std::isnan(beta) || std::isinf(beta)) {
        st->done = kBreakdown;
        st->cycle_done = 1;
    } else if (beta <= st->stop) {
        st->done = kConverged;
        st->cycle_done = 1;
    } else if (st->iter >= st->maxit) {
        st->done = kMaxIter;
        st->cycle_done = 1;
    } else {
        st->cycles += 1;
    }
}

// ------------------------------------------------------------ one workgroup
// The whole restarted GMRES(m) of a small CSR system in one launch of one
// 1024-thread workgroup: the same steps, criteria and state as the kernels
// above, without a launch or host poll per step.  Thread t owns rows t,
// t + 1024, ...; w of those rows stays in registers through a step; the
// basis lives in global memory (L2-resident at these sizes); the rotated
// Hessenberg R, g and the rotations in LDS.  Per-vector sums are wave DPP
// sums, then the waves' totals are added in wave order; the small scalar
// work (the column's rotations, the back substitution) runs on thread 0.
constexpr int kSGT = 1024;
constexpr int kSGRows = 4;
constexpr int kSGWaves = kSGT / kWave;

struct small_gmres_lds {
    double red[kSGWaves][kGmresSmallKrylov + 2];
    double R[kGmresSmallKrylov][kGmresSmallKrylov];  // R[i][j], i <= j
    double g[kGmresSmallKrylov + 1], cs[kGmresSmallKrylov], sn[kGmresSmallKrylov];
    double h[kGmresSmallKrylov + 2], h2[kGmresSmallKrylov + 2], y[kGmresSmallKrylov];
    double hcol[kGmresSmallKrylov + 1];
    double hn, est, ww;
    int cycle_done, breakdown;
};

// Vectors taken together by the passes over the basis, so that their loads
// are in flight at once.
constexpr int kSGVecs = 4;

// out[i] = V_i . w for i < k, out[k] = w . w (w: this thread's rows).
__device__ inline void sg_dots(int k, int64_t n, const double *__restrict__ V, int64_t ldv,
                               const double (&w)[kSGRows], double *out, small_gmres_lds &L) {
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    for (int i0 = 0; i0 <= k; i0 += kSGVecs) {
        double s[kSGVecs];
#pragma unroll
        for (int u = 0; u < kSGVecs; ++u) s[u] = 0.0;
#pragma unroll
        for (int r = 0; r < kSGRows; ++r) {
            const int64_t row = t + (int64_t)r * kSGT;
            if (row < n) {
#pragma unroll
                for (int u = 0; u < kSGVecs; ++u) {
                    const int i = i0 + u;
                    if (i < k) s[u] += V[(int64_t)i * ldv + row] * w[r];
                    else if (i == k) s[u] += w[r] * w[r];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kSGVecs; ++u) {
            if (i0 + u > k) break;
            const double tot = wave_total(s[u]);
            if (lane == 0) L.red[wv][i0 + u] = tot;
        }
    }
    __syncthreads();
    if (t <= k) {
        double s = 0.0;
        for (int q = 0; q < kSGWaves; ++q) s += L.red[q][t];
        out[t] = s;
    }
    __syncthreads();
}

// w -= sum_{i < k} c_i V_i over this thread's rows, in ascending i, two
// vectors' loads at a time (four would spill).
__device__ inline void sg_subtract(int k, int64_t n, const double *__restrict__ V, int64_t ldv,
                                   const double *c, double (&w)[kSGRows]) {
    constexpr int U = 2;
    const int t = threadIdx.x;
    for (int i0 = 0; i0 < k; i0 += U) {
        double v[U][kSGRows];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < kSGRows; ++r) {
                const int64_t row = t + (int64_t)r * kSGT;
                v[u][r] = (i0 + u < k && row < n) ? V[(int64_t)(i0 + u) * ldv + row] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (i0 + u < k)
#pragma unroll
                for (int r = 0; r < kSGRows; ++r) w[r] = w[r] - c[i0 + u] * v[u][r];
    }
}

// y = A v over this thread's rows (CSR rows from memory), four entries of a
// row in flight.
__device__ inline void sg_spmv(int64_t n, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ col, const double *__restrict__ val,
                               const double *__restrict__ v, double (&y)[kSGRows]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int r = 0; r < kSGRows; ++r) {
        const int64_t row = t + (int64_t)r * kSGT;
        double s = 0.0;
        if (row < n) {
            const int32_t b = rp[row], e = rp[row + 1];
            int32_t q = b;
            for (; q + 4 <= e; q += 4) {
                const int32_t c0 = col[q], c1 = col[q + 1], c2 = col[q + 2], c3 = col[q + 3];
                const double x0 = v[c0], x1 = v[c1], x2 = v[c2], x3 = v[c3];
                s += val[q] * x0;
                s += val[q + 1] * x1;
                s += val[q + 2] * x2;
                s += val[q + 3] * x3;
            }
            for (; q < e; ++q) s += val[q] * v[col[q]];
        }
        y[r] = s;
    }
}

__global__ __launch_bounds__(kSGT) void gmres_small_kernel(
    int64_t n, int m, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, double *__restrict__ x,
    double *__restrict__ V, int64_t ldv, double stop, int maxit, gmres_state *out) {
    __shared__ small_gmres_lds L;
    const int t = threadIdx.x;
    if (t == 0) L.est = 0.0;  // visible after the first sum's barrier
    int iter = 0, cycles = 0, reorths = 0, done = kRunning, k = 0;
    double beta = 0.0;
    double w[kSGRows];
    for (;;) {
        // cycle start: v0 = b - A x and its norm
        sg_spmv(n, rp, col, val, x, w);
#pragma unroll
        for (int r = 0; r < kSGRows; ++r) {
            const int64_t row = t + (int64_t)r * kSGT;
            w[r] = row < n ? b[row] - w[r] : 0.0;
        }
        sg_dots(0, n, V, ldv, w, L.h, L);
        beta = sqrt(L.h[0]);
        if (std::isnan(beta) || std::isinf(beta)) { done = kBreakdown; break; }
        if (beta <= stop) { done = kConverged; break; }
        if (iter >= maxit) { done = kMaxIter; break; }
        ++cycles;
#pragma unroll
        for (int r = 0; r < kSGRows; ++r) {
            const int64_t row = t + (int64_t)r * kSGT;
            if (row < n) V[row] = w[r] / beta;
        }
        if (t == 0) L.g[0] = beta;
        __syncthreads();
        for (int j = 0; j < m; ++j) {
            // w = A v_j
            sg_spmv(n, rp, col, val, V + (int64_t)j * ldv, w);
            // classical Gram-Schmidt, a second round when the first lost
            // more than 1/sqrt(2) of w
            sg_dots(j + 1, n, V, ldv, w, L.h, L);
            sg_subtract(j + 1, n, V, ldv, L.h, w);
            sg_dots(j + 1, n, V, ldv, w, L.h2, L);
            double ww = L.h2[j + 1];
            const bool reorth = 2.0 * L.h2[j + 1] < L.h[j + 1];
            if (reorth) {
                ++reorths;
                sg_subtract(j + 1, n, V, ldv, L.h2, w);
                sg_dots(0, n, V, ldv, w, &L.ww, L);
                ww = L.ww;
            }
            ++iter;
            k = j + 1;
            if (t == 0) {
                // the column of H, the earlier rotations, the new one
                double *hcol = L.hcol;
                for (int i = 0; i <= j; ++i) hcol[i] = reorth ? L.h[i] + L.h2[i] : L.h[i];
                const double hn = sqrt(ww);
                for (int i = 0; i < j; ++i) {
                    const double a = hcol[i], c = hcol[i + 1];
                    hcol[i] = L.cs[i] * a + L.sn[i] * c;
                    hcol[i + 1] = -L.sn[i] * a + L.cs[i] * c;
                }
                const double a = hcol[j];
                const double d = sqrt(a * a + hn * hn);
                L.hn = hn;
                L.breakdown = 0;
                L.cycle_done = 0;
                if (!(d > 0.0)) {
                    L.breakdown = 1;
                } else {
                    L.cs[j] = a / d;
                    L.sn[j] = hn / d;
                    hcol[j] = d;
                    for (int i = 0; i <= j; ++i) L.R[i][j] = hcol[i];
                    L.g[j + 1] = -L.sn[j] * L.g[j];
                    L.g[j] = L.cs[j] * L.g[j];
                    const double est = fabs(L.g[j + 1]);
                    L.est = est;
                    if (std::isnan(est)) L.breakdown = 1;
                    else if (est <= stop || hn == 0.0 || iter >= maxit || j + 1 == m)
                        L.cycle_done = 1;
                }
            }
            __syncthreads();
            if (L.breakdown) { done = kBreakdown; break; }
            if (L.cycle_done) break;
            const double hn = L.hn;
            double *vn = V + (int64_t)(j + 1) * ldv;
#pragma unroll
            for (int r = 0; r < kSGRows; ++r) {
                const int64_t row = t + (int64_t)r * kSGT;
                if (row < n) vn[row] = w[r] / hn;
            }
            __syncthreads();
        }
        if (done == kBreakdown) break;
        // cycle end: R y = g over the k columns, x += V_k y
        if (t == 0)
            for (int i = k - 1; i >= 0; --i) {
                double s = L.g[i];
                for (int l = i + 1; l < k; ++l) s = s - L.R[i][l] * L.y[l];
                L.y[i] = s / L.R[i][i];
            }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kSGRows; ++r) {
            const int64_t row = t + (int64_t)r * kSGT;
            if (row < n) {
                double xl = x[row];
                for (int i = 0; i < k; ++i) xl = xl + L.y[i] * V[(int64_t)i * ldv + row];
                x[row] = xl;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        out->iter = iter;
        out->cycles = cycles;
        out->reorths = reorths;
        out->done = done;
        out->est = L.est;
        out->beta = beta;
        out->k = k;
    }
}

}  // namespace

int64_t gmres_ld(int64_t n) { return (n + 63) / 64 * 64; }

int64_t gmres_partial_elems(int64_t n, int m) { return (int64_t)(m + 2) * gmres_blocks(n); }

hipError_t gmres_arnoldi_step(hipStream_t s, int64_t n, int m, int j, double *V, int64_t ldv,
                              gmres_state *st, const gmres_work &wk) {
    const int g = gmres_blocks(n);
    double *w = V + (int64_t)(j + 1) * ldv;
    const int k = j + 1;
    // first Gram-Schmidt round; its update also forms the second round's dots
    gmres_dot_kernel<<<g, kG, 0, s>>>(n, k, V, ldv, w, st, 0, wk.partials);
    gmres_sum_kernel<<<k + 1, kG, 0, s>>>(g, wk.partials, wk.dot1, st, 0);
    if (k <= kGRegVecs)
        gmres_update_dot_regs_kernel<<<g, kG, 0, s>>>(n, k, V, ldv, wk.dot1, w, st, wk.partials);
    else
        gmres_update_dot_kernel<<<g, kG, 0, s>>>(n, k, V, ldv, wk.dot1, w, st, wk.partials);
    gmres_sum_kernel<<<k + 1, kG, 0, s>>>(g, wk.partials, wk.dot2, st, 0);
    gmres_check_kernel<<<1, 1, 0, s>>>(j, wk.dot1, wk.dot2, st, wk.hcol);
    // the second round's update, only when the first lost too much of w
    gmres_update_kernel<<<g, kG, 0, s>>>(n, k, V, ldv, wk.dot2, w, st, 1, wk.partials);
    gmres_sum_kernel<<<1, kG, 0, s>>>(g, wk.partials, wk.upd2, st, 1);
    gmres_step_kernel<<<1, 1, 0, s>>>(j, m, wk.dot2, wk.upd2, st, wk.hcol, wk.H, wk.cs, wk.sn,
                                      wk.g);
    gmres_scale_kernel<<<reduction_blocks(n), kG, 0, s>>>(n, w, st);
    return hipGetLastError();
}

hipError_t gmres_cycle_start(hipStream_t s, int64_t n, double *V, gmres_state *st,
                             const gmres_work &wk) {
    // v0 . v0 through the dot pass with no basis vectors
    const int g = gmres_blocks(n);
    gmres_dot_kernel<<<g, kG, 0, s>>>(n, 0, V, 0, V, st, 2, wk.partials);
    gmres_sum_kernel<<<1, kG, 0, s>>>(g, wk.partials, wk.upd1, st, 2);
    gmres_cycle_kernel<<<1, 1, 0, s>>>(wk.upd1, st, wk.g);
    gmres_scale_kernel<<<reduction_blocks(n), kG, 0, s>>>(n, V, st);
    return hipGetLastError();
}

int64_t gmres_small_max_rows() { return (int64_t)kSGT * kSGRows; }

hipError_t gmres_small(hipStream_t s, int64_t n, int m, const int32_t *rp, const int32_t *col,
                       const double *val, const double *b, double *x, double *V, int64_t ldv,
                       double stop, int maxit, gmres_state *out) {
    if (n < 1 || n > gmres_small_max_rows() || m < 1 || m > kGmresSmallKrylov)
        return hipErrorInvalidValue;
    gmres_small_kernel<<<1, kSGT, 0, s>>>(n, m, rp, col, val, b, x, V, ldv, stop, maxit, out);
    return hipGetLastError();
}

hipError_t gmres_cycle_end(hipStream_t s, int64_t n, int m, const double *V, int64_t ldv, double *x,
                           gmres_state *st, const gmres_work &wk) {
    gmres_solve_kernel<<<1, 1, 0, s>>>(m, wk.H, wk.g, wk.y, st);
    gmres_xupdate_kernel<<<reduction_blocks(n), kG, 0, s>>>(n, V, ldv, wk.y, x, st);
    return hipGetLastError();
}

}  // namespace gko
