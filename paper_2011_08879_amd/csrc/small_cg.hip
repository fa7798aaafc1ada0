// CG on a single workgroup for systems whose direction vector fits in LDS.
//
// For small systems the multi-kernel CG is bound by launch and grid-wide
// reduction latency, not by memory: a 4096-row 2D Laplacian moves about
// 0.7 MB per iteration.  Here the whole solve is one launch on one compute
// unit.  Thread t owns rows t, t+T, t+2T, ...; the solution, residual and
// A p of its rows stay in registers, and only the direction p (gathered by
// the product) lives in LDS.  An iteration costs three workgroup barriers.
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
        v = subwarp<kWave>::reduce_sum(v);
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

// s_j = (A v)_i for the thread's rows i = tid + j T, v in LDS.
template <int T, int R>
__device__ inline void rows_product(int32_t n, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col,
                                    const double *__restrict__ val, const double *v,
                                    double (&s)[R]) {
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        double a = 0.0;
        if (i < n)
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k) a += val[k] * v[col[k]];
        s[j] = a;
    }
}

template <int T, int R>
__global__ __launch_bounds__(T) void small_cg_kernel(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ val,
                                                     const double *__restrict__ b,
                                                     double *__restrict__ x, double tol,
                                                     int32_t maxit, small_cg_result *out) {
    extern __shared__ double p[];  // n: the direction (x while a residual is formed)
    __shared__ double slots[2][T / kWave];
    wg_reducer<T> sum{slots};

    double xr[R], rr[R], br[R], q[R];
    double loc = 0.0;
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int32_t i = threadIdx.x + j * T;
        br[j] = i < n ? b[i] : 0.0;
        xr[j] = i < n ? x[i] : 0.0;
        loc += br[j] * br[j];
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
        rows_product<T, R>(n, rp, col, val, p, q);
        double l = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int32_t i = threadIdx.x + j * T;
            rr[j] = i < n ? br[j] - q[j] : 0.0;
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
                rows_product<T, R>(n, rp, col, val, p, q);
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

template <int R>
hipError_t launch_small(hipStream_t s, int32_t n, const int32_t *rp, const int32_t *col,
                        const double *val, const double *b, double *x, double tol, int32_t maxit,
                        small_cg_result *out) {
    small_cg_kernel<kSmallT, R><<<1, kSmallT, (size_t)n * sizeof(double), s>>>(
        n, rp, col, val, b, x, tol, maxit, out);
    return hipGetLastError();
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

hipError_t small_cg(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                    const double *val, const double *b, double *x, double tol, int32_t maxit,
                    small_cg_result *out) {
    if (n <= 0 || n > small_cg_max_rows()) return hipErrorInvalidValue;
    const int32_t m = (int32_t)n;
    if (n <= kSmallT) return launch_small<1>(s, m, rp, col, val, b, x, tol, maxit, out);
    if (n <= 2 * kSmallT) return launch_small<2>(s, m, rp, col, val, b, x, tol, maxit, out);
    if (n <= 4 * kSmallT) return launch_small<4>(s, m, rp, col, val, b, x, tol, maxit, out);
    return launch_small<8>(s, m, rp, col, val, b, x, tol, maxit, out);
}

}  // namespace gko
