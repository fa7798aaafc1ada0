// CG on a single workgroup for systems whose direction vector fits in LDS.
//
// For small systems the multi-kernel CG is bound by launch and grid-wide
// reduction latency, not by memory: a 4096-row 2D Laplacian moves about
// 0.7 MB per iteration.  Here the whole solve is one launch on one compute
// unit.  Thread t owns rows t, t+T, t+2T, ...; the solution, residual and
// A p of its rows stay in registers, and only the direction p (gathered by
// the product) lives in LDS.  When every row has at most L entries, a
// thread also keeps its rows' column indices and values in registers
// (padded with zero values), so an iteration reads no global memory at all.
// An iteration costs three workgroup barriers.
//
// The steps are those of the multi-kernel path (Hestenes-Stiefel CG,
// unpreconditioned): stop when r.r <= tol^2 b.b, recompute the true residual
// b - A x, and restart from x when it misses tol (at most twice).  Sums use a
// fixed tree, so results repeat bitwise.
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"
#include "solver_state.hpp"

namespace gko {

namespace {

constexpr int kSmallT = 1024;

// Workgroup sum with one barrier: partials go to one of two slot arrays in
// turn, so a slot array is rewritten only after a later barrier has shown
// that every thread finished reading it.
template <int T>
struct wg_reducer {
    double (*slots)[T / kWave];
    int parity = 0;
    __device__ double operator()(double v) {
        constexpr int NW = T / kWave;
        v = wave_total(v);
        double *red = slots[parity];
        parity ^= 1;
        if ((threadIdx.x % kWave) == 0) red[threadIdx.x / kWave] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NW; ++j) s += red[j];
        return s;
    }
};

// The thread's rows held in registers: L slots per row, unused slots with
// value 0 and the row's own index as column (a harmless in-range read).
// Columns are below 2^16 here (n <= 8192), so two share a register.
template <int R, int L>
struct row_cache {
    static constexpr int LP = L > 0 ? (L + 1) / 2 : 1;
    uint32_t c[R][LP];
    double v[R][L > 0 ? L : 1];
    __device__ int32_t col(int j, int q) const { return (c[j][q / 2] >> (16 * (q & 1))) & 0xffffu; }
};

template <int T, int R, int L>
__device__ inline void load_rows(int32_t n, const int32_t *__restrict__ rp,
                                 const int32_t *__restrict__ col, const double *__restrict__ val,
                                 row_cache<R, L> &rc) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        const int32_t b = i < n ? rp[i] : 0, e = i < n ? rp[i + 1] : 0;
#pragma unroll
        for (int q = 0; q < row_cache<R, L>::LP; ++q) rc.c[j][q] = 0u;
#pragma unroll
        for (int q = 0; q < L; ++q) {
            const bool ok = b + q < e;
            const uint32_t cq = (uint32_t)(ok ? col[b + q] : (i < n ? i : 0));
            rc.c[j][q / 2] |= cq << (16 * (q & 1));
            rc.v[j][q] = ok ? val[b + q] : 0.0;
        }
    }
}

// s_j = (A v)_i for the thread's rows i = tid + j T, v in LDS; entries in
// ascending order, from registers (L > 0) or from global memory.
template <int T, int R, int L>
__device__ inline void rows_product(int32_t n, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col,
                                    const double *__restrict__ val, const row_cache<R, L> &rc,
                                    const double *v, double (&s)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        double a = 0.0;
        if constexpr (L > 0) {
#pragma unroll
            for (int q = 0; q < L; ++q) a += rc.v[j][q] * v[rc.col(j, q)];
            // one row's gathers in flight at a time: keeps the register
            // budget for the cached rows
            __builtin_amdgcn_sched_barrier(0);
        } else if (i < n) {
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) a += val[k] * v[col[k]];
        }
        s[j] = a;
    }
}

template <int T, int R, int L>
__global__ __launch_bounds__(T) void small_cg_kernel(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ x, double tol,
                                                     int32_t maxit, small_cg_result *out) {
    extern __shared__ double p[];  // n: the direction (x while a residual is formed)
    __shared__ double slots[2][T / kWave];
    wg_reducer<T> sum{slots};

    row_cache<R, L> rc;
    if constexpr (L > 0) load_rows<T, R, L>(n, rp, col, val, rc);
    double xr[R], rr[R], q[R];
    double loc = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        const double bi = i < n ? b[i] : 0.0;
        xr[j] = i < n ? x[i] : 0.0;
        loc += bi * bi;
    }
    const double bb = sum(loc);
    const double stop2 = tol * tol * bb;
    int32_t it = 0, restarts = 0, flag = kRunning;
    double rho = 0.0, tr2 = 0.0;

    // r = b - A x into rr[], returns r.r.  Every thread has passed the
    // reduction's barrier when it returns, so p may be rewritten afterwards.
    auto residual = [&]() {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * T;
            if (i < n) p[i] = xr[j];
        }
        __syncthreads();
        rows_product<T, R, L>(n, rp, col, val, rc, p, q);
        double l = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * T;
            rr[j] = i < n ? b[i] - q[j] : 0.0;
            l += rr[j] * rr[j];
        }
        return sum(l);
    };

    if (!std::isfinite(bb)) {
        flag = kBreakdown;
    } else if (bb == 0.0) {
#pragma unroll
        for (int j = 0; j < R; ++j) xr[j] = 0.0;
        flag = kConverged;
    } else {
        rho = residual();
        for (;;) {
            if (!std::isfinite(rho)) {
                flag = kBreakdown;
                break;
            }
            // p = r
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int32_t i = threadIdx.x + j * T;
                if (i < n) p[i] = rr[j];
            }
            __syncthreads();
            while (rho > stop2 && it < maxit) {
                rows_product<T, R, L>(n, rp, col, val, rc, p, q);
                double l = 0.0;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * T;
                    if (i < n) l += p[i] * q[j];
                }
                const double pq = sum(l);
                ++it;
                if (!(pq > 0.0)) {
                    flag = std::isnan(pq) ? kBreakdown : kNotSpd;
                    break;
                }
                const double alpha = rho / pq;
                l = 0.0;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * T;
                    if (i < n) {
                        xr[j] = xr[j] + alpha * p[i];
                        rr[j] = rr[j] - alpha * q[j];
                        l += rr[j] * rr[j];
                    }
                }
                const double rho_new = sum(l);
                if (!std::isfinite(rho_new)) {
                    flag = kBreakdown;
                    break;
                }
                if (rho_new <= stop2) {
                    rho = rho_new;
                    break;
                }
                const double beta = rho_new / rho;
                rho = rho_new;
#pragma unroll
                for (int j = 0; j < R; ++j) {
                    const int32_t i = threadIdx.x + j * T;
                    if (i < n) p[i] = rr[j] + beta * p[i];
                }
                __syncthreads();
            }
            if (flag != kRunning) break;
            if (!(rho <= stop2)) {
                flag = kMaxIter;
                break;
            }
            // the true residual decides; a miss restarts from x
            __syncthreads();  // every thread is done with p before x overwrites it
            tr2 = residual();
            if (std::sqrt(tr2) <= tol * std::sqrt(bb)) {
                flag = kConverged;
                break;
            }
            if (restarts == 2 || it >= maxit) {
                flag = kMaxIter;
                break;
            }
            ++restarts;
            rho = tr2;
            __syncthreads();
        }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        if (i < n) x[i] = xr[j];
    }
    if (flag != kConverged || bb == 0.0) {
        // the true residual was not formed on this exit
        __syncthreads();
        tr2 = bb == 0.0 ? 0.0 : residual();
    }
    if (threadIdx.x == 0) {
        out->bb = bb;
        out->rr = rho;
        out->tr2 = tr2;
        out->iters = it;
        out->flag = flag;
        out->restarts = restarts;
    }
}

template <int R, int L>
hipError_t launch_small(hipStream_t s, int32_t n, const int32_t *rp, const int32_t *col,
                        const double *val, const double *b, double *x, double tol, int32_t maxit,
                        small_cg_result *out) {
    small_cg_kernel<kSmallT, R, L><<<1, kSmallT, (size_t)n * sizeof(double), s>>>(
        n, rp, col, val, b, x, tol, maxit, out);
    return hipGetLastError();
}

// R rows per thread; rows of at most LMAX entries are kept in registers
// (LMAX is what fits the register budget of a 1024-thread workgroup next to
// R), longer ones are read from memory every iteration.
template <int R, int LMAX>
hipError_t launch_small_r(hipStream_t s, int32_t n, int64_t max_len, const int32_t *rp,
                          const int32_t *col, const double *val, const double *b, double *x,
                          double tol, int32_t maxit, small_cg_result *out) {
    if (max_len <= LMAX) return launch_small<R, LMAX>(s, n, rp, col, val, b, x, tol, maxit, out);
    return launch_small<R, 0>(s, n, rp, col, val, b, x, tol, maxit, out);
}

}  // namespace

int64_t small_cg_max_rows() {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return 0;
    // p in dynamic LDS plus the reduction slots (static)
    const int64_t by_lds = ((int64_t)lds - 2 * (kSmallT / kWave) * 8 - 64) / 8;
    const int64_t by_regs = (int64_t)kSmallT * 8;
    return by_lds < by_regs ? by_lds : by_regs;
}

hipError_t small_cg(hipStream_t s, int64_t n, int64_t max_len, const int32_t *rp,
                    const int32_t *col, const double *val, const double *b, double *x, double tol,
                    int32_t maxit, small_cg_result *out) {
    if (n <= 0 || n > small_cg_max_rows()) return hipErrorInvalidValue;
    const int32_t m = (int32_t)n;
    if (n <= kSmallT)
        return launch_small_r<1, 16>(s, m, max_len, rp, col, val, b, x, tol, maxit, out);
    if (n <= 2 * kSmallT)
        return launch_small_r<2, 8>(s, m, max_len, rp, col, val, b, x, tol, maxit, out);
    if (n <= 4 * kSmallT)
        return launch_small_r<4, 5>(s, m, max_len, rp, col, val, b, x, tol, maxit, out);
    return launch_small_r<8, 3>(s, m, max_len, rp, col, val, b, x, tol, maxit, out);
}

}  // namespace gko
