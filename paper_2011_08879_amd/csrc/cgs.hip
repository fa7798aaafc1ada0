// CGS, conjugate gradients squared (Sonneveld 1989; Saad, Iterative Methods,
// Alg. 7.5), unpreconditioned, FP64, shadow residual rhat = r0.  Per
// iteration two SpMVs by the format's own kernel and four vector kernels;
// the scalars stay in device memory (krylov_scalars), every reduction ends
// in an op that applies the recurrence's scalar step:
//   t = A p;  alpha = rho / (t.rhat)                        [cgs_alpha]
//   q = u - alpha t;  w = u + q;  x += alpha w              [cgs_qwx]
//   t = A w;  r -= alpha t;  r.r, rho' = r.rhat; beta      [cgs_update]
//   u = r + beta q;  p = u + beta (q + beta p)             [cgs_direction]
#include <cmath>

#include "device.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"
#include "solver_state.hpp"
#include "krylov_ops.hpp"

namespace gko {

namespace {

constexpr int kB = kRedBlock;

// Start: totals r.r, b.b; rho = r.rhat = r.r.
struct cgs_init_op {
    krylov_scalars *sc;
    double tol;
    __device__ bool skip() const { return false; }
    __device__ void operator()(const double *o) const {
        sc->rho = o[0];
        sc->rr = o[0];
        sc->bb = o[1];
        sc->stop2 = tol * tol * o[1];
        if (!std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[0] <= sc->stop2) sc->done = kConverged;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else sc->done = kRunning;
    }
};


// After r -= alpha A (u + q): totals r.r, r.rhat; convergence, then beta.
struct cgs_update_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->iter += 1;
        sc->rr = o[0];
        if (!std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[0] <= sc->stop2) sc->done = kConverged;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else if (!(fabs(o[1]) >= 1e-300)) sc->done = kBreakdown;
        else {
            sc->beta = o[1] / sc->rho;
            sc->rho = o[1];
        }
    }
};

__global__ __launch_bounds__(kB) void cgs_init_kernel(int64_t n, const double *__restrict__ b,
                                                      const double *__restrict__ r,
                                                      double *__restrict__ rh,
                                                      double *__restrict__ p,
                                                      double *__restrict__ u, double tol,
                                                      krylov_scalars *sc, red_args ra) {
    double a_rr = 0.0, a_bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double ri = r[i];
        rh[i] = ri;
        p[i] = ri;
        u[i] = ri;
        a_rr += ri * ri;
        a_bb += b[i] * b[i];
    }
    double v[2] = {a_rr, a_bb};
    grid_sum_apply<kB, 2>(v, ra, cgs_init_op{sc, tol});
}

__global__ __launch_bounds__(kB) void cgs_alpha_kernel(int64_t n, const double *__restrict__ t,
                                                       const double *__restrict__ rh,
                                                       krylov_scalars *sc, red_args ra) {
    if (sc->done) return;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        a += t[i] * rh[i];
    double v[1] = {a};
    grid_sum_apply<kB, 1>(v, ra, cgs_alpha_op{sc});
}

__global__ __launch_bounds__(kB) void cgs_qwx_kernel(int64_t n, const double *__restrict__ u,
                                                     const double *__restrict__ t,
                                                     double *__restrict__ q,
                                                     double *__restrict__ w,
                                                     double *__restrict__ x,
                                                     const krylov_scalars *sc) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double ui = u[i];
        const double qi = ui - alpha * t[i];
        const double wi = ui + qi;
        q[i] = qi;
        w[i] = wi;
        x[i] = x[i] + alpha * wi;
    }
}

__global__ __launch_bounds__(kB) void cgs_update_kernel(int64_t n, double *__restrict__ r,
                                                        const double *__restrict__ t,
                                                        const double *__restrict__ rh,
                                                        krylov_scalars *sc, red_args ra) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    double a_rr = 0.0, a_rho = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double ri = r[i] - alpha * t[i];
        r[i] = ri;
        a_rr += ri * ri;
        a_rho += ri * rh[i];
    }
    double v[2] = {a_rr, a_rho};
    grid_sum_apply<kB, 2>(v, ra, cgs_update_op{sc});
}

__global__ __launch_bounds__(kB) void cgs_direction_kernel(int64_t n, const double *__restrict__ r,
                                                           const double *__restrict__ q,
                                                           double *__restrict__ u,
                                                           double *__restrict__ p,
                                                           const krylov_scalars *sc) {
    if (sc->done) return;
    const double beta = sc->beta;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double qi = q[i];
        const double ui = r[i] + beta * qi;
        u[i] = ui;
        p[i] = ui + beta * (qi + beta * p[i]);
    }
}

}  // namespace

hipError_t cgs_init(hipStream_t s, int64_t n, const void *b, const void *r, void *rh, void *p,
                    void *u, double tol, krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    cgs_init_kernel<<<g, kB, 0, s>>>(n, static_cast<const double *>(b),
                                     static_cast<const double *>(r), static_cast<double *>(rh),
                                     static_cast<double *>(p), static_cast<double *>(u), tol, sc,
                                     ra);
    return red_finish<2>(s, g, ra, cgs_init_op{sc, tol});
}

hipError_t cgs_alpha(hipStream_t s, int64_t n, const void *t, const void *rh, krylov_scalars *sc,
                     double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    cgs_alpha_kernel<<<g, kB, 0, s>>>(n, static_cast<const double *>(t),
                                      static_cast<const double *>(rh), sc, ra);
    return red_finish<1>(s, g, ra, cgs_alpha_op{sc});
}

hipError_t cgs_qwx(hipStream_t s, int64_t n, const void *u, const void *t, void *q, void *w,
                   void *x, const krylov_scalars *sc) {
    cgs_qwx_kernel<<<stream_blocks(n), kB, 0, s>>>(
        n, static_cast<const double *>(u), static_cast<const double *>(t), static_cast<double *>(q),
        static_cast<double *>(w), static_cast<double *>(x), sc);
    return hipGetLastError();
}

hipError_t cgs_update(hipStream_t s, int64_t n, void *r, const void *t, const void *rh,
                      krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    cgs_update_kernel<<<g, kB, 0, s>>>(n, static_cast<double *>(r), static_cast<const double *>(t),
                                       static_cast<const double *>(rh), sc, ra);
    return red_finish<2>(s, g, ra, cgs_update_op{sc});
}

hipError_t cgs_direction(hipStream_t s, int64_t n, const void *r, const void *q, void *u, void *p,
                         const krylov_scalars *sc) {
    cgs_direction_kernel<<<stream_blocks(n), kB, 0, s>>>(
        n, static_cast<const double *>(r), static_cast<const double *>(q), static_cast<double *>(u),
        static_cast<double *>(p), sc);
    return hipGetLastError();
}

}  // namespace gko
