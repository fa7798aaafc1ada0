// Vector kernels of the Krylov solvers: dot/norm reductions and the fused
// step kernels of CG (with optional block-Jacobi) and BiCGSTAB.
//
// The paper's solvers are memory bound (Sec. 6.2), so each step is fused to
// touch every vector as few times as possible, and the scalars of the
// recurrences (alpha, beta, rho, ...) never leave the GPU: the last block of
// each deterministic grid reduction updates them in device memory, and every
// kernel returns immediately once the solver is flagged done.  Reductions
// always accumulate in FP64, also for FP32 vectors.
#include <climits>
#include <cmath>

#include "csr_rows.hpp"
#include "device.hpp"
#include "ell_rows.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"
#include "solver_state.hpp"
#include "krylov_ops.hpp"

namespace gko {

constexpr int kB = kRedBlock;  // 256 threads, one row per thread per tile

// Grid of a fused product over n rows (or row pairs), one per thread.
static int fused_blocks(int64_t n) {
    int64_t g = (n + kB - 1) / kB;
    if (g > kFusedMaxBlocks) g = kFusedMaxBlocks;
    return g < 1 ? 1 : (int)g;
}

int stream_blocks(int64_t n) { return fused_blocks(n); }

int reduction_blocks(int64_t n) {
    int64_t g = (n + kB - 1) / kB;
    if (g > kMaxReductionBlocks) g = kMaxReductionBlocks;
    if (g < 1) g = 1;
    return (int)g;
}

// ------------------------------------------------------------------ finishing operations
// What the totals of each reduction update, applied once per launch (by the
// last block or by the finalize kernel).  skip() repeats the early-exit test
// of the kernel whose partials are being summed.
struct dot_op {
    double *result;
    bool sq;
    __device__ bool skip() const { return false; }
    __device__ void operator()(const double *o) const { *result = sq ? sqrt(o[0]) : o[0]; }
};

// CG start: totals r.z, r.r, b.b.
struct cg_init_op {
    krylov_scalars *sc;
    double tol;
    __device__ bool skip() const { return false; }
    __device__ void operator()(const double *o) const {
        sc->rho = o[0];
        sc->rr = o[1];
        sc->bb = o[2];
        sc->stop2 = tol * tol * o[2];
        if (!std::isfinite(o[1]) || !std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[1] <= sc->stop2) sc->done = kConverged;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else sc->done = kRunning;
    }
};

// alpha = rho / p.q; p.q <= 0 means A is not SPD.
struct cg_alpha_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        const double pq = o[0];
        sc->aux = pq;
        if (!(pq > 0.0)) {
            sc->done = std::isnan(pq) ? kBreakdown : kNotSpd;
            sc->iter += 1;
        } else {
            sc->alpha = sc->rho / pq;
        }
    }
};

// After the update: totals r.z, r.r (and, for flexible CG, z.(r - r_old));
// convergence test, then beta: r.z / rho (Fletcher-Reeves, CG) or
// z.(r - r_old) / rho (Polak-Ribiere, flexible CG).
struct cg_update_op {
    krylov_scalars *sc;
    bool flex;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->iter += 1;
        sc->rr = o[1];
        if (!std::isfinite(o[1]) || !std::isfinite(o[0])) {
            sc->done = kBreakdown;
        } else if (o[1] <= sc->stop2) {
            sc->done = kConverged;
        } else {
            sc->beta = (flex ? o[2] : o[0]) / sc->rho;
            sc->rho = o[0];
            if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        }
    }
};

// BiCGSTAB start: totals r.r, b.b.
struct bicg_init_op {
    krylov_scalars *sc;
    double tol;
    __device__ bool skip() const { return false; }
    __device__ void operator()(const double *o) const {
        sc->rho = o[0];
        sc->rr = o[0];
        sc->bb = o[1];
        sc->stop2 = tol * tol * o[1];
        sc->rho_old = sc->alpha = sc->omega = 1.0;
        sc->half = 0;
        if (!std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[0] <= sc->stop2) sc->done = kConverged;
        else if (!(fabs(o[0]) >= 1e-300)) sc->done = kBreakdown;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else {
            sc->beta = (sc->rho / sc->rho_old) * (sc->alpha / sc->omega);
            sc->done = kRunning;
        }
    }
};

// alpha = rho / (rhat.v)
struct bicg_alpha_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->aux = o[0];
        if (!(fabs(o[0]) >= 1e-300)) sc->done = kBreakdown;
        else sc->alpha = sc->rho / o[0];
    }
};

// s.s: converging here finishes at the half step.
struct bicg_s_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->iter += 1;
        if (!std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[0] <= sc->stop2) {
            sc->half = 1;
            sc->rr = o[0];
        }
    }
};

// omega = (t.s) / (t.t)
struct bicg_omega_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0 || sc->half != 0; }
    __device__ void operator()(const double *o) const {
        sc->aux = o[1];
        if (!(o[1] >= 1e-300)) sc->done = kBreakdown;
        else sc->omega = o[0] / o[1];
    }
};

// After the update: totals r.r and the next rho = rhat.r.
struct bicg_update_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        if (sc->half) {
            sc->done = kConverged;
            return;
        }
        sc->rr = o[0];
        if (!std::isfinite(o[0])) sc->done = kBreakdown;
        else if (o[0] <= sc->stop2) sc->done = kConverged;
        else if (sc->omega == 0.0) sc->done = kBreakdown;
        else {
            sc->rho_old = sc->rho;
            sc->rho = o[1];
            if (!(fabs(o[1]) >= 1e-300)) sc->done = kBreakdown;
            else {
                sc->beta = (sc->rho / sc->rho_old) * (sc->alpha / sc->omega);
                if (sc->iter >= sc->maxit) sc->done = kMaxIter;
            }
        }
    }
};

// ------------------------------------------------------------------ dot / norm
template <typename V>
__global__ __launch_bounds__(kB) void dot_kernel(int64_t n, const V *__restrict__ x,
                                                 const V *__restrict__ y, red_args ra, dot_op op) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        s += (double)x[i] * (double)y[i];
    double v[1] = {s};
    grid_sum_apply<kB, 1>(v, ra, op);
}

hipError_t dot(hipStream_t s, vt t, int64_t n, const void *x, const void *y, double *result,
               double *partials, unsigned *ticket, bool sqrt_result) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    const dot_op op{result, sqrt_result};
    if (t == vt::f64)
        dot_kernel<double><<<g, kB, 0, s>>>(n, static_cast<const double *>(x),
                                            static_cast<const double *>(y), ra, op);
    else
        dot_kernel<float><<<g, kB, 0, s>>>(n, static_cast<const float *>(x),
                                           static_cast<const float *>(y), ra, op);
    return red_finish<1>(s, g, ra, op);
}

// ------------------------------------------------------------------ scalars
__global__ void scalars_reset_kernel(krylov_scalars *sc, int32_t maxit) {
    sc->rho = sc->rho_old = sc->alpha = sc->beta = sc->omega = 0.0;
    sc->rr = sc->bb = sc->stop2 = sc->aux = 0.0;
    sc->iter = 0;
    sc->maxit = maxit;
    sc->done = kRunning;
    sc->half = 0;
}

hipError_t scalars_reset(hipStream_t s, krylov_scalars *sc, int32_t maxit) {
    scalars_reset_kernel<<<1, 1, 0, s>>>(sc, maxit);
    return hipGetLastError();
}

// ------------------------------------------------------------------ block-Jacobi apply
// z_i = sum_j D_b^{-1}[i mod bs][j] r_{b*bs + j}, j ascending, for the tile
// of 256 rows starting at `base`, with entry (i, j) of a symmetric inverse
// block read from its packed upper triangle (the (min, max) entry).  The
// tile's packed blocks (contiguous because BS divides 256) and residuals are
// staged in LDS with coalesced loads.  Slots of a short last block beyond n
// are zero in `inv`.
template <int BS>
constexpr int bj_packed() { return BS * (BS + 1) / 2; }

template <typename V, int BS>
__device__ inline V bj_tile_apply(int64_t n, int64_t base, V ri, const V *__restrict__ inv,
                                  V *r_lds, V *inv_lds) {
    constexpr int P = bj_packed<BS>();
    const int tid = threadIdx.x;
    r_lds[tid] = ri;
    const int64_t nb = (n + BS - 1) / BS;
    const int64_t off = (base / BS) * P;
    for (int t = tid; t < (kB / BS) * P; t += kB)
        inv_lds[t] = (off + t < nb * P) ? inv[off + t] : V(0);
    __syncthreads();
    V z = V(0);
    const int i = tid % BS, b0 = tid - i;
    const V *D = inv_lds + (tid / BS) * P;
    const int row_i = i * BS - i * (i - 1) / 2 - i;  // packed (i, j) = row_i + j, j >= i
#pragma unroll
    for (int j = 0; j < BS; ++j) {
        const int idx = j >= i ? row_i + j : j * BS - j * (j - 1) / 2 - j + i;
        z += D[idx] * r_lds[b0 + j];
    }
    __syncthreads();
    return z;
}

// ------------------------------------------------------------------ CG
// Start (or restart) from r = b - A x: z = M^-1 r, p = z, rho = r.z, rr = r.r,
// bb = b.b; flags convergence at zero iterations.
template <typename V, int BS>
__global__ __launch_bounds__(kB) void cg_init_kernel(int64_t n, const V *__restrict__ b,
                                                     const V *__restrict__ r, V *__restrict__ z,
                                                     V *__restrict__ p, const V *__restrict__ inv,
                                                     double tol, krylov_scalars *sc,
                                                     red_args ra) {
    __shared__ V r_lds[BS > 0 ? kB : 1];
    __shared__ V inv_lds[BS > 0 ? kB / (BS > 0 ? BS : 1) * bj_packed<BS>() : 1];
    double a_rz = 0.0, a_rr = 0.0, a_bb = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kB; base < n; base += (int64_t)gridDim.x * kB) {
        const int64_t i = base + threadIdx.x;
        const V ri = i < n ? r[i] : V(0);
        V zi = ri;
        if constexpr (BS > 0) zi = bj_tile_apply<V, BS>(n, base, ri, inv, r_lds, inv_lds);
        if (i < n) {
            if constexpr (BS > 0) z[i] = zi;
            p[i] = zi;
            const double bi = (double)b[i];
            a_rz += (double)ri * (double)zi;
            a_rr += (double)ri * (double)ri;
            a_bb += bi * bi;
        }
    }
    double v[3] = {a_rz, a_rr, a_bb};
    grid_sum_apply<kB, 3>(v, ra, cg_init_op{sc, tol});
}

// ------------------------------------------------------------------ fused products
// out = A in by a format's SpMV row sums, with the sums a Krylov step needs
// next formed in the same pass and finished by the step's reduction op.
// What is summed is a policy:
//   pq_dot     in.out                  (CG: p.q)
//   aux_dot    aux.out                 (BiCGSTAB: rhat.v; CGS: t.rhat)
//   omega_dot  out.in and out.out      (BiCGSTAB: t.s and t.t)
template <typename V, typename Op>
struct pq_dot {
    static constexpr int NV = 1;
    Op op;
    __device__ bool skip() const { return op.skip(); }
    __device__ void add(double (&a)[NV], int64_t, V in, V out) const {
        a[0] += (double)in * (double)out;
    }
};
template <typename V, typename Op>
struct aux_dot {
    static constexpr int NV = 1;
    const V *aux;
    Op op;
    __device__ bool skip() const { return op.skip(); }
    __device__ void add(double (&a)[NV], int64_t i, V, V out) const {
        a[0] += (double)aux[i] * (double)out;
    }
};
template <typename V, typename Op>
struct omega_dot {
    static constexpr int NV = 2;
    Op op;
    __device__ bool skip() const { return op.skip(); }
    __device__ void add(double (&a)[NV], int64_t, V in, V out) const {
        a[0] += (double)out * (double)in;
        a[1] += (double)out * (double)out;
    }
};

// CSR, a subwarp of W lanes per U rows (as in the plain SpMV).
template <typename V, int W, typename P>
__global__ __launch_bounds__(kB) void fused_csr_kernel(int64_t n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const V *__restrict__ val,
                                                       const V *__restrict__ in, V *__restrict__ out,
                                                       P pol, red_args ra) {
    if (pol.skip()) return;
    constexpr int U = csr_shape<W>::U;
    constexpr int RPB = kB / W * U;
    const int lane = threadIdx.x % W;
    double acc[P::NV] = {};
    for (int64_t g0 = (int64_t)blockIdx.x * RPB; g0 < n; g0 += (int64_t)gridDim.x * RPB) {
        const int64_t row0 = g0 + (int64_t)(threadIdx.x / W) * U;
        if (row0 < n) {  // uniform across the subwarp
            V s[U];
            csr_rows_sum<V, W, U>(n, row0, lane, rp, col, val, in, s, INT_MAX);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t r = row0 + u;
                if ((W >= U ? lane == u : lane == 0) && r < n) {
                    out[r] = s[u];
                    pol.add(acc, r, in[r], s[u]);
                }
            }
        }
    }
    grid_sum_apply<kB, P::NV>(acc, ra, pol.op);
}

// CSR with G lanes per row and the entries staged through LDS (short regular
// rows, as in the plain SpMV); the workgroup strides over tiles of kB / G
// rows, and the first lane of each row stores it and adds its terms.
template <typename V, typename P, int G>
__global__ __launch_bounds__(kRowThreadBlock) void fused_csr_rowthread_kernel(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ in, V *__restrict__ out, P pol, red_args ra) {
    static_assert(kRowThreadBlock == kB, "one reduction block shape");
    constexpr int64_t RT = kB / G;
    __shared__ rowthread_lds<V> L;
    if (pol.skip()) return;
    double acc[P::NV] = {};
    // up to kXcdRowsMax rows, each round of the grid stride gives each XCD
    // one contiguous range of rows
    for (int64_t r0 = row_block_order(n) * RT; r0 < n; r0 += (int64_t)gridDim.x * RT) {
        const V s = csr_rowthread_sum<V, G>(n, r0, rp, col, val, in, L);
        const int64_t i = r0 + threadIdx.x / G;
        if (i < n && threadIdx.x % G == 0) {
            out[i] = s;
            pol.add(acc, i, in[i], s);
        }
    }
    grid_sum_apply<kB, P::NV>(acc, ra, pol.op);
}

// ELL, two adjacent rows per thread (as in the plain SpMV).
template <typename V, typename P>
__global__ __launch_bounds__(kB) void fused_ell_kernel(int64_t n, int64_t K, int64_t ld,
                                                       const int32_t *__restrict__ ecol,
                                                       const V *__restrict__ eval,
                                                       const V *__restrict__ in, V *__restrict__ out,
                                                       P pol, red_args ra) {
    if (pol.skip()) return;
    double acc[P::NV] = {};
    // workgroup order as in the plain SpMV (row_block_order)
    for (int64_t i = 2 * (row_block_order(n) * kB + threadIdx.x); i < n;
         i += 2 * (int64_t)gridDim.x * kB) {
        V s0, s1;
        ell_pair_rows(K, ld, i, ecol, eval, in, s0, s1);
        out[i] = s0;
        pol.add(acc, i, in[i], s0);
        if (i + 1 < n) {
            out[i + 1] = s1;
            pol.add(acc, i + 1, in[i + 1], s1);
        }
    }
    grid_sum_apply<kB, P::NV>(acc, ra, pol.op);
}

// SELL-P: a row per thread, a slice per wavefront (the grid-stride step is a
// multiple of the slice size).  Matrices with wide slices do not come here.
// STRIDE: the grid is smaller than the row count.  Without the grid-stride
// loop the FP64 kernel needs 40 VGPRs instead of 92 (8 waves per SIMD
// instead of 5).
template <typename V, typename P, bool STRIDE>
__global__ __launch_bounds__(kB) void fused_sellp_kernel(int64_t n, const int64_t *__restrict__ sets,
                                                         const int32_t *__restrict__ scol,
                                                         const V *__restrict__ sval,
                                                         const V *__restrict__ in,
                                                         V *__restrict__ out, P pol, red_args ra) {
    static_assert(kB % kSellpSlice == 0, "whole slices per workgroup");
    if (pol.skip()) return;
    double acc[P::NV] = {};
    int64_t i = row_block_order(n) * kB + threadIdx.x;
    if constexpr (STRIDE) {
        for (; i < n; i += (int64_t)gridDim.x * kB) {
            const V s0 = sellp_row(i, sets, scol, sval, in);
            out[i] = s0;
            pol.add(acc, i, in[i], s0);
        }
    } else if (i < n) {
        const V s0 = sellp_row(i, sets, scol, sval, in);
        out[i] = s0;
        pol.add(acc, i, in[i], s0);
    }
    grid_sum_apply<kB, P::NV>(acc, ra, pol.op);
}

// p.q after a SpMV done by a format's own kernel.
template <typename V>
__global__ __launch_bounds__(kB) void cg_pq_kernel(int64_t n, const V *__restrict__ p,
                                                   const V *__restrict__ q, krylov_scalars *sc,
                                                   red_args ra) {
    if (sc->done) return;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        acc += (double)p[i] * (double)q[i];
    double v[1] = {acc};
    grid_sum_apply<kB, 1>(v, ra, cg_alpha_op{sc});
}

// x += alpha p; r -= alpha q; z = M^-1 r; rho' = r.z; rr = r.r; then beta.
template <typename V, int BS, bool FLEX>
__global__ __launch_bounds__(kB) void cg_update_kernel(int64_t n, V *__restrict__ x,
                                                       V *__restrict__ r, V *__restrict__ z,
                                                       const V *__restrict__ p,
                                                       const V *__restrict__ q,
                                                       const V *__restrict__ inv,
                                                       krylov_scalars *sc, red_args ra) {
    __shared__ V r_lds[BS > 0 ? kB : 1];
    __shared__ V inv_lds[BS > 0 ? kB / (BS > 0 ? BS : 1) * bj_packed<BS>() : 1];
    if (sc->done) return;
    const double alpha = sc->alpha;
    double a_rz = 0.0, a_rr = 0.0, a_zt = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kB; base < n; base += (int64_t)gridDim.x * kB) {
        const int64_t i = base + threadIdx.x;
        V ri = V(0), ro = V(0);
        if (i < n) {
            x[i] = (V)((double)x[i] + alpha * (double)p[i]);
            ro = r[i];
            ri = (V)((double)ro - alpha * (double)q[i]);
            r[i] = ri;
        }
        V zi = ri;
        if constexpr (BS > 0) zi = bj_tile_apply<V, BS>(n, base, ri, inv, r_lds, inv_lds);
        if (i < n) {
            if constexpr (BS > 0) z[i] = zi;
            a_rz += (double)ri * (double)zi;
            a_rr += (double)ri * (double)ri;
            if constexpr (FLEX) a_zt += (double)zi * ((double)ri - (double)ro);
        }
    }
    if constexpr (FLEX) {
        double v[3] = {a_rz, a_rr, a_zt};
        grid_sum_apply<kB, 3>(v, ra, cg_update_op{sc, true});
    } else {
        double v[2] = {a_rz, a_rr};
        grid_sum_apply<kB, 2>(v, ra, cg_update_op{sc, false});
    }
}

// p = z + beta p  (z = r without a preconditioner).
template <typename V>
__global__ __launch_bounds__(kB) void cg_direction_kernel(int64_t n, const V *__restrict__ z,
                                                          V *__restrict__ p,
                                                          const krylov_scalars *sc) {
    if (sc->done) return;
    const double beta = sc->beta;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        p[i] = (V)((double)z[i] + beta * (double)p[i]);
}

template <typename V>
static hipError_t launch_cg_init(hipStream_t s, int64_t n, const void *b, const void *r, void *z,
                                 void *p, const void *inv, int bs, double tol, krylov_scalars *sc,
                                 double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    const V *B = static_cast<const V *>(b), *R = static_cast<const V *>(r);
    V *Z = static_cast<V *>(z), *P = static_cast<V *>(p);
    const V *I = static_cast<const V *>(inv);
    switch (bs) {
        case 0: cg_init_kernel<V, 0><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        case 1: cg_init_kernel<V, 1><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        case 2: cg_init_kernel<V, 2><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        case 4: cg_init_kernel<V, 4><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        case 8: cg_init_kernel<V, 8><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        case 16: cg_init_kernel<V, 16><<<g, kB, 0, s>>>(n, B, R, Z, P, I, tol, sc, ra); break;
        default: return hipErrorInvalidValue;
    }
    return red_finish<3>(s, g, ra, cg_init_op{sc, tol});
}

hipError_t cg_init(hipStream_t s, vt t, int64_t n, const void *b, const void *r, void *z, void *p,
                   const void *inv, int bs, double tol, krylov_scalars *sc, double *partials,
                   unsigned *ticket) {
    return t == vt::f64 ? launch_cg_init<double>(s, n, b, r, z, p, inv, bs, tol, sc, partials, ticket)
                        : launch_cg_init<float>(s, n, b, r, z, p, inv, bs, tol, sc, partials, ticket);
}

template <typename V, int W, typename P>
static hipError_t launch_fused_csr_w(hipStream_t s, const fused_matrix &A, const V *in, V *out,
                                     const P &pol, double *partials, unsigned *ticket) {
    constexpr int RPB = kB / W * csr_shape<W>::U;
    int64_t g = (A.n + RPB - 1) / RPB;
    if (g > kFusedMaxBlocks) g = kFusedMaxBlocks;
    if (g < 1) g = 1;
    const red_args ra = red_for((int)g, partials, ticket);
    fused_csr_kernel<V, W, P><<<(unsigned)g, kB, 0, s>>>(
        A.n, A.rp, A.col, static_cast<const V *>(A.val), in, out, pol, ra);
    return red_finish<P::NV>(s, (int)g, ra, pol.op);
}

template <typename V, typename P>
static hipError_t launch_fused(hipStream_t s, const fused_matrix &A, const void *in_, void *out_,
                               const P &pol, double *partials, unsigned *ticket) {
    static_assert(P::NV <= kFusedMaxSums, "the partials scratch holds kFusedMaxSums per block");
    const V *in = static_cast<const V *>(in_);
    V *out = static_cast<V *>(out_);
    if (A.format == fused_matrix::ell) {
        const int g = fused_blocks((A.n + 1) / 2);
        const red_args ra = red_for(g, partials, ticket);
        fused_ell_kernel<V, P><<<g, kB, 0, s>>>(A.n, A.K, A.ld, A.ecol,
                                                static_cast<const V *>(A.eval), in, out, pol, ra);
        return red_finish<P::NV>(s, g, ra, pol.op);
    }
    if (A.format == fused_matrix::sellp) {
        const int g = fused_blocks(A.n);
        const red_args ra = red_for(g, partials, ticket);
        if ((int64_t)g * kB >= A.n)
            fused_sellp_kernel<V, P, false><<<g, kB, 0, s>>>(
                A.n, A.sets, A.scol, static_cast<const V *>(A.sval), in, out, pol, ra);
        else
            fused_sellp_kernel<V, P, true><<<g, kB, 0, s>>>(
                A.n, A.sets, A.scol, static_cast<const V *>(A.sval), in, out, pol, ra);
        return red_finish<P::NV>(s, g, ra, pol.op);
    }
    if (A.w == kCsrRowThread) {
        if (A.lanes != 1 && A.lanes != 4 && A.lanes != 8) return hipErrorInvalidValue;
        // one block per tile of kB / lanes rows, at most kFusedMaxBlocks
        const int g = fused_blocks(A.n * A.lanes);
        const red_args ra = red_for(g, partials, ticket);
        if (A.lanes == 8)
            fused_csr_rowthread_kernel<V, P, 8><<<g, kB, 0, s>>>(
                A.n, A.rp, A.col, static_cast<const V *>(A.val), in, out, pol, ra);
        else if (A.lanes == 4)
            fused_csr_rowthread_kernel<V, P, 4><<<g, kB, 0, s>>>(
                A.n, A.rp, A.col, static_cast<const V *>(A.val), in, out, pol, ra);
        else
            fused_csr_rowthread_kernel<V, P, 1><<<g, kB, 0, s>>>(
                A.n, A.rp, A.col, static_cast<const V *>(A.val), in, out, pol, ra);
        return red_finish<P::NV>(s, g, ra, pol.op);
    }
    switch (A.w) {
        case 1: return launch_fused_csr_w<V, 1>(s, A, in, out, pol, partials, ticket);
        case 2: return launch_fused_csr_w<V, 2>(s, A, in, out, pol, partials, ticket);
        case 4: return launch_fused_csr_w<V, 4>(s, A, in, out, pol, partials, ticket);
        case 8: return launch_fused_csr_w<V, 8>(s, A, in, out, pol, partials, ticket);
        case 16: return launch_fused_csr_w<V, 16>(s, A, in, out, pol, partials, ticket);
        case 32: return launch_fused_csr_w<V, 32>(s, A, in, out, pol, partials, ticket);
        case 64: return launch_fused_csr_w<V, 64>(s, A, in, out, pol, partials, ticket);
        default: return hipErrorInvalidValue;
    }
}

hipError_t cg_spmv(hipStream_t s, const fused_matrix &A, const void *p, void *q, krylov_scalars *sc,
                   double *partials, unsigned *ticket) {
    if (A.t == vt::f64)
        return launch_fused<double>(s, A, p, q, pq_dot<double, cg_alpha_op>{cg_alpha_op{sc}},
                                    partials, ticket);
    return launch_fused<float>(s, A, p, q, pq_dot<float, cg_alpha_op>{cg_alpha_op{sc}}, partials,
                               ticket);
}

hipError_t bicg_spmv_alpha(hipStream_t s, const fused_matrix &A, const void *p, void *v,
                           const void *rh, krylov_scalars *sc, double *partials, unsigned *ticket) {
    if (A.t != vt::f64) return hipErrorInvalidValue;
    const aux_dot<double, bicg_alpha_op> pol{static_cast<const double *>(rh), bicg_alpha_op{sc}};
    return launch_fused<double>(s, A, p, v, pol, partials, ticket);
}

hipError_t bicg_spmv_omega(hipStream_t s, const fused_matrix &A, const void *sv, void *t,
                           krylov_scalars *sc, double *partials, unsigned *ticket) {
    if (A.t != vt::f64) return hipErrorInvalidValue;
    return launch_fused<double>(s, A, sv, t, omega_dot<double, bicg_omega_op>{bicg_omega_op{sc}},
                                partials, ticket);
}

hipError_t cgs_spmv_alpha(hipStream_t s, const fused_matrix &A, const void *p, void *t,
                          const void *rh, krylov_scalars *sc, double *partials, unsigned *ticket) {
    if (A.t != vt::f64) return hipErrorInvalidValue;
    const aux_dot<double, cgs_alpha_op> pol{static_cast<const double *>(rh), cgs_alpha_op{sc}};
    return launch_fused<double>(s, A, p, t, pol, partials, ticket);
}

hipError_t cg_pq(hipStream_t s, vt t, int64_t n, const void *p, const void *q, krylov_scalars *sc,
                 double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    if (t == vt::f64)
        cg_pq_kernel<double><<<g, kB, 0, s>>>(n, static_cast<const double *>(p),
                                              static_cast<const double *>(q), sc, ra);
    else
        cg_pq_kernel<float><<<g, kB, 0, s>>>(n, static_cast<const float *>(p),
                                             static_cast<const float *>(q), sc, ra);
    return red_finish<1>(s, g, ra, cg_alpha_op{sc});
}

template <typename V, bool FLEX>
static hipError_t launch_cg_update(hipStream_t s, int64_t n, void *x, void *r, void *z,
                                   const void *p, const void *q, const void *inv, int bs,
                                   krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    V *X = static_cast<V *>(x), *R = static_cast<V *>(r), *Z = static_cast<V *>(z);
    const V *P = static_cast<const V *>(p), *Q = static_cast<const V *>(q);
    const V *I = static_cast<const V *>(inv);
    switch (bs) {
        case 0: cg_update_kernel<V, 0, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        case 1: cg_update_kernel<V, 1, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        case 2: cg_update_kernel<V, 2, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        case 4: cg_update_kernel<V, 4, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        case 8: cg_update_kernel<V, 8, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        case 16: cg_update_kernel<V, 16, FLEX><<<g, kB, 0, s>>>(n, X, R, Z, P, Q, I, sc, ra); break;
        default: return hipErrorInvalidValue;
    }
    if constexpr (FLEX) return red_finish<3>(s, g, ra, cg_update_op{sc, true});
    return red_finish<2>(s, g, ra, cg_update_op{sc, false});
}

hipError_t cg_update(hipStream_t s, vt t, int64_t n, void *x, void *r, void *z, const void *p,
                     const void *q, const void *inv, int bs, krylov_scalars *sc, double *partials,
                     unsigned *ticket, bool flexible) {
    if (flexible)
        return t == vt::f64
                   ? launch_cg_update<double, true>(s, n, x, r, z, p, q, inv, bs, sc, partials, ticket)
                   : launch_cg_update<float, true>(s, n, x, r, z, p, q, inv, bs, sc, partials, ticket);
    return t == vt::f64
               ? launch_cg_update<double, false>(s, n, x, r, z, p, q, inv, bs, sc, partials, ticket)
               : launch_cg_update<float, false>(s, n, x, r, z, p, q, inv, bs, sc, partials, ticket);
}

hipError_t cg_direction(hipStream_t s, vt t, int64_t n, const void *z, void *p,
                        const krylov_scalars *sc) {
    const int g = stream_blocks(n);
    if (t == vt::f64)
        cg_direction_kernel<double><<<g, kB, 0, s>>>(n, static_cast<const double *>(z),
                                                     static_cast<double *>(p), sc);
    else
        cg_direction_kernel<float><<<g, kB, 0, s>>>(n, static_cast<const float *>(z),
                                                    static_cast<float *>(p), sc);
    return hipGetLastError();
}

// ------------------------------------------------------------------ pipelined CG
// Ghysels and Vanroose's pipelined (P)CG: u = M^-1 r and w = A u are carried
// by recurrences, so an iteration is one product n = A m (m = M^-1 w) and one
// fused vector kernel whose single reduction (gamma = r.u, delta = w.u, r.r)
// yields the next alpha and beta.  Without a preconditioner u = r, m = w and
// q = s, and the kernel carries the four vectors z, s, p, w besides x, r.

// alpha and beta of the step that follows the sums gamma, delta:
// first step beta = 0, alpha = gamma / delta; then beta = gamma / gamma_old,
// alpha = gamma / (delta - beta gamma / alpha_old).  The denominator is
// p.Ap in exact arithmetic, <= 0 means A is not SPD.
__device__ inline void pipe_next(krylov_scalars *sc, double gamma, double delta, bool first) {
    const double beta = first ? 0.0 : gamma / sc->rho;
    const double den = first ? delta : delta - beta * gamma / sc->alpha;
    sc->aux = den;
    if (!(den > 0.0)) {
        sc->done = std::isnan(den) ? kBreakdown : kNotSpd;
        sc->iter += 1;
        return;
    }
    sc->beta = beta;
    sc->alpha = gamma / den;
    sc->rho = gamma;
}

// Start: totals gamma, delta, r.r, b.b.
struct pipe_init_op {
    krylov_scalars *sc;
    double tol;
    __device__ bool skip() const { return false; }
    __device__ void operator()(const double *o) const {
        sc->rr = o[2];
        sc->bb = o[3];
        sc->stop2 = tol * tol * o[3];
        if (!std::isfinite(o[2]) || !std::isfinite(o[0]) || !std::isfinite(o[1])) sc->done = kBreakdown;
        else if (o[2] <= sc->stop2) sc->done = kConverged;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else {
            sc->done = kRunning;
            pipe_next(sc, o[0], o[1], true);
        }
    }
};

// After an update: totals gamma, delta, r.r.
struct pipe_update_op {
    krylov_scalars *sc;
    __device__ bool skip() const { return sc->done != 0; }
    __device__ void operator()(const double *o) const {
        sc->iter += 1;
        sc->rr = o[2];
        if (!std::isfinite(o[2]) || !std::isfinite(o[0]) || !std::isfinite(o[1])) sc->done = kBreakdown;
        else if (o[2] <= sc->stop2) sc->done = kConverged;
        else if (sc->iter >= sc->maxit) sc->done = kMaxIter;
        else pipe_next(sc, o[0], o[1], false);
    }
};

// u = M^-1 r (preconditioned start only).
template <typename V, int BS>
__global__ __launch_bounds__(kB) void pipe_precond_kernel(int64_t n, const V *__restrict__ r,
                                                          V *__restrict__ u,
                                                          const V *__restrict__ inv) {
    __shared__ V r_lds[kB];
    __shared__ V inv_lds[kB / BS * bj_packed<BS>()];
    for (int64_t base = (int64_t)blockIdx.x * kB; base < n; base += (int64_t)gridDim.x * kB) {
        const int64_t i = base + threadIdx.x;
        const V ri = i < n ? r[i] : V(0);
        const V ui = bj_tile_apply<V, BS>(n, base, ri, inv, r_lds, inv_lds);
        if (i < n) u[i] = ui;
    }
}

// Start, after w = A u: m = M^-1 w, and the sums gamma, delta, r.r, b.b.
template <typename V, int BS>
__global__ __launch_bounds__(kB) void pipe_init_kernel(int64_t n, const V *__restrict__ b,
                                                       const V *__restrict__ r,
                                                       const V *__restrict__ u,
                                                       const V *__restrict__ w, V *__restrict__ m,
                                                       const V *__restrict__ inv, double tol,
                                                       krylov_scalars *sc, red_args ra) {
    __shared__ V r_lds[BS > 0 ? kB : 1];
    __shared__ V inv_lds[BS > 0 ? kB / (BS > 0 ? BS : 1) * bj_packed<BS>() : 1];
    double a_g = 0.0, a_d = 0.0, a_rr = 0.0, a_bb = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kB; base < n; base += (int64_t)gridDim.x * kB) {
        const int64_t i = base + threadIdx.x;
        const V wi = i < n ? w[i] : V(0);
        V mi = wi;
        if constexpr (BS > 0) mi = bj_tile_apply<V, BS>(n, base, wi, inv, r_lds, inv_lds);
        if (i < n) {
            if constexpr (BS > 0) m[i] = mi;
            const double ri = (double)r[i], ui = (double)u[i], bi = (double)b[i];
            a_g += ri * ui;
            a_d += (double)wi * ui;
            a_rr += ri * ri;
            a_bb += bi * bi;
        }
    }
    double v[4] = {a_g, a_d, a_rr, a_bb};
    grid_sum_apply<kB, 4>(v, ra, pipe_init_op{sc, tol});
}

// One iteration after n = A m:
//   z = n + beta z; q = m + beta q; s = w + beta s; p = u + beta p;
//   x += alpha p; r -= alpha s; u -= alpha q; w -= alpha z; m = M^-1 w;
// then gamma = r.u, delta = w.u, r.r.  BS = 0: u = r, m = w, q = s.
template <typename V, int BS>
__global__ __launch_bounds__(kB) void pipe_update_kernel(
    int64_t n, const V *__restrict__ nv, V *__restrict__ z, V *__restrict__ q, V *__restrict__ s,
    V *__restrict__ p, V *__restrict__ x, V *__restrict__ r, V *__restrict__ u, V *__restrict__ w,
    V *__restrict__ m, const V *__restrict__ inv, krylov_scalars *sc, red_args ra) {
    __shared__ V r_lds[BS > 0 ? kB : 1];
    __shared__ V inv_lds[BS > 0 ? kB / (BS > 0 ? BS : 1) * bj_packed<BS>() : 1];
    if (sc->done) return;
    const double alpha = sc->alpha, beta = sc->beta;
    double a_g = 0.0, a_d = 0.0, a_rr = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kB; base < n; base += (int64_t)gridDim.x * kB) {
        const int64_t i = base + threadIdx.x;
        V wi = V(0), ri = V(0), ui = V(0);
        if (i < n) {
            const double zi = (double)nv[i] + beta * (double)z[i];
            const double si = (double)w[i] + beta * (double)s[i];
            z[i] = (V)zi;
            s[i] = (V)si;
            if constexpr (BS > 0) {
                const double qi = (double)m[i] + beta * (double)q[i];
                const double pi = (double)u[i] + beta * (double)p[i];
                q[i] = (V)qi;
                p[i] = (V)pi;
                x[i] = (V)((double)x[i] + alpha * (double)(V)pi);
                ri = (V)((double)r[i] - alpha * (double)(V)si);
                ui = (V)((double)u[i] - alpha * (double)(V)qi);
                u[i] = ui;
            } else {
                const double pi = (double)r[i] + beta * (double)p[i];
                p[i] = (V)pi;
                x[i] = (V)((double)x[i] + alpha * (double)(V)pi);
                ri = (V)((double)r[i] - alpha * (double)(V)si);
                ui = ri;
            }
            r[i] = ri;
            wi = (V)((double)w[i] - alpha * (double)(V)zi);
            w[i] = wi;
        }
        if constexpr (BS > 0) {
            const V mi = bj_tile_apply<V, BS>(n, base, wi, inv, r_lds, inv_lds);
            if (i < n) m[i] = mi;
        }
        if (i < n) {
            a_g += (double)ri * (double)ui;
            a_d += (double)wi * (double)ui;
            a_rr += (double)ri * (double)ri;
        }
    }
    double v[3] = {a_g, a_d, a_rr};
    grid_sum_apply<kB, 3>(v, ra, pipe_update_op{sc});
}

template <typename V>
static hipError_t launch_pipe_init(hipStream_t s, int64_t n, const void *b, const void *r, void *u,
                                   const void *w, void *m, const void *inv, int bs, double tol,
                                   krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    const V *B = static_cast<const V *>(b), *R = static_cast<const V *>(r);
    const V *U = static_cast<const V *>(u), *W = static_cast<const V *>(w);
    V *M = static_cast<V *>(m);
    const V *I = static_cast<const V *>(inv);
    switch (bs) {
        case 0: pipe_init_kernel<V, 0><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        case 1: pipe_init_kernel<V, 1><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        case 2: pipe_init_kernel<V, 2><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        case 4: pipe_init_kernel<V, 4><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        case 8: pipe_init_kernel<V, 8><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        case 16: pipe_init_kernel<V, 16><<<g, kB, 0, s>>>(n, B, R, U, W, M, I, tol, sc, ra); break;
        default: return hipErrorInvalidValue;
    }
    return red_finish<4>(s, g, ra, pipe_init_op{sc, tol});
}

template <typename V>
static hipError_t launch_pipe_precond(hipStream_t s, int64_t n, const void *r, void *u,
                                      const void *inv, int bs) {
    const int g = reduction_blocks(n);
    const V *R = static_cast<const V *>(r), *I = static_cast<const V *>(inv);
    V *U = static_cast<V *>(u);
    switch (bs) {
        case 1: pipe_precond_kernel<V, 1><<<g, kB, 0, s>>>(n, R, U, I); break;
        case 2: pipe_precond_kernel<V, 2><<<g, kB, 0, s>>>(n, R, U, I); break;
        case 4: pipe_precond_kernel<V, 4><<<g, kB, 0, s>>>(n, R, U, I); break;
        case 8: pipe_precond_kernel<V, 8><<<g, kB, 0, s>>>(n, R, U, I); break;
        case 16: pipe_precond_kernel<V, 16><<<g, kB, 0, s>>>(n, R, U, I); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename V>
static hipError_t launch_pipe_update(hipStream_t st, int64_t n, const pipe_vectors &v,
                                     const void *inv, int bs, krylov_scalars *sc,
                                     double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    const V *N = static_cast<const V *>(v.n), *I = static_cast<const V *>(inv);
    V *Z = static_cast<V *>(v.z), *Q = static_cast<V *>(v.q), *S = static_cast<V *>(v.s);
    V *P = static_cast<V *>(v.p), *X = static_cast<V *>(v.x), *R = static_cast<V *>(v.r);
    V *U = static_cast<V *>(v.u), *W = static_cast<V *>(v.w), *M = static_cast<V *>(v.m);
    switch (bs) {
        case 0: pipe_update_kernel<V, 0><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        case 1: pipe_update_kernel<V, 1><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        case 2: pipe_update_kernel<V, 2><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        case 4: pipe_update_kernel<V, 4><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        case 8: pipe_update_kernel<V, 8><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        case 16: pipe_update_kernel<V, 16><<<g, kB, 0, st>>>(n, N, Z, Q, S, P, X, R, U, W, M, I, sc, ra); break;
        default: return hipErrorInvalidValue;
    }
    return red_finish<3>(st, g, ra, pipe_update_op{sc});
}

hipError_t pipe_precond(hipStream_t s, vt t, int64_t n, const void *r, void *u, const void *inv,
                        int bs) {
    return t == vt::f64 ? launch_pipe_precond<double>(s, n, r, u, inv, bs)
                        : launch_pipe_precond<float>(s, n, r, u, inv, bs);
}

hipError_t pipe_init(hipStream_t s, vt t, int64_t n, const void *b, const void *r, void *u,
                     const void *w, void *m, const void *inv, int bs, double tol,
                     krylov_scalars *sc, double *partials, unsigned *ticket) {
    return t == vt::f64
               ? launch_pipe_init<double>(s, n, b, r, u, w, m, inv, bs, tol, sc, partials, ticket)
               : launch_pipe_init<float>(s, n, b, r, u, w, m, inv, bs, tol, sc, partials, ticket);
}

hipError_t pipe_update(hipStream_t s, vt t, int64_t n, const pipe_vectors &v, const void *inv,
                       int bs, krylov_scalars *sc, double *partials, unsigned *ticket) {
    return t == vt::f64 ? launch_pipe_update<double>(s, n, v, inv, bs, sc, partials, ticket)
                        : launch_pipe_update<float>(s, n, v, inv, bs, sc, partials, ticket);
}

// ------------------------------------------------------------------ BiCGSTAB (FP64)
// Start from r = b - A x: rhat = r, p = v = 0, rho = rhat.r, bb = b.b,
// rho_old = alpha = omega = 1, so the first direction is p = r.
__global__ __launch_bounds__(kB) void bicg_init_kernel(int64_t n, const double *__restrict__ b,
                                                       const double *__restrict__ r,
                                                       double *__restrict__ rh,
                                                       double *__restrict__ p,
                                                       double *__restrict__ v, double tol,
                                                       krylov_scalars *sc, red_args ra) {
    double a_rr = 0.0, a_bb = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double ri = r[i];
        rh[i] = ri;
        p[i] = 0.0;
        v[i] = 0.0;
        a_rr += ri * ri;
        a_bb += b[i] * b[i];
    }
    double vv[2] = {a_rr, a_bb};
    grid_sum_apply<kB, 2>(vv, ra, bicg_init_op{sc, tol});
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(kB) void bicg_p_kernel(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ p,
                                                    const krylov_scalars *sc) {
    if (sc->done) return;
    const double beta = sc->beta, omega = sc->omega;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// alpha = rho / (rhat.v)
__global__ __launch_bounds__(kB) void bicg_alpha_kernel(int64_t n, const double *__restrict__ rh,
                                                        const double *__restrict__ v,
                                                        krylov_scalars *sc, red_args ra) {
    if (sc->done) return;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
        a += rh[i] * v[i];
    double vv[1] = {a};
    grid_sum_apply<kB, 1>(vv, ra, bicg_alpha_op{sc});
}

// s = r - alpha v, with s.s: converging here finishes at the half step.
__global__ __launch_bounds__(kB) void bicg_s_kernel(int64_t n, const double *__restrict__ r,
                                                    const double *__restrict__ v,
                                                    double *__restrict__ s, krylov_scalars *sc,
                                                    red_args ra) {
    if (sc->done) return;
    const double alpha = sc->alpha;
    double a = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        const double si = r[i] - alpha * v[i];
        s[i] = si;
        a += si * si;
    }
    double vv[1] = {a};
    grid_sum_apply<kB, 1>(vv, ra, bicg_s_op{sc});
}

// omega = (t.s) / (t.t)
__global__ __launch_bounds__(kB) void bicg_omega_kernel(int64_t n, const double *__restrict__ t,
                                                        const double *__restrict__ s,
                                                        krylov_scalars *sc, red_args ra) {
    if (sc->done || sc->half) return;
    double a_ts = 0.0, a_tt = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        a_ts += t[i] * s[i];
        a_tt += t[i] * t[i];
    }
    double vv[2] = {a_ts, a_tt};
    grid_sum_apply<kB, 2>(vv, ra, bicg_omega_op{sc});
}

// x += alpha p + omega s; r = s - omega t; then rr and the next rho = rhat.r.
// At the half step only x += alpha p.
__global__ __launch_bounds__(kB) void bicg_update_kernel(int64_t n, double *__restrict__ x,
                                                         double *__restrict__ r,
                                                         const double *__restrict__ rh,
                                                         const double *__restrict__ p,
                                                         const double *__restrict__ s,
                                                         const double *__restrict__ t,
                                                         krylov_scalars *sc, red_args ra) {
    if (sc->done) return;
    const bool half = sc->half != 0;
    const double alpha = sc->alpha, omega = sc->omega;
    double a_rr = 0.0, a_rho = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
        if (half) {
            x[i] = x[i] + alpha * p[i];
        } else {
            x[i] = x[i] + alpha * p[i] + omega * s[i];
            const double ri = s[i] - omega * t[i];
            r[i] = ri;
            a_rr += ri * ri;
            a_rho += rh[i] * ri;
        }
    }
    double vv[2] = {a_rr, a_rho};
    grid_sum_apply<kB, 2>(vv, ra, bicg_update_op{sc});
}

static inline const double *cd(const void *p) { return static_cast<const double *>(p); }
static inline double *md(void *p) { return static_cast<double *>(p); }

hipError_t bicg_init(hipStream_t st, int64_t n, const void *b, const void *r, void *rh, void *p,
                     void *v, double tol, krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    bicg_init_kernel<<<g, kB, 0, st>>>(n, cd(b), cd(r), md(rh), md(p), md(v), tol,
                                                        sc, ra);
    return red_finish<2>(st, g, ra, bicg_init_op{sc, tol});
}

hipError_t bicg_p(hipStream_t st, int64_t n, const void *r, const void *v, void *p,
                  const krylov_scalars *sc) {
    bicg_p_kernel<<<stream_blocks(n), kB, 0, st>>>(n, cd(r), cd(v), md(p), sc);
    return hipGetLastError();
}

hipError_t bicg_alpha(hipStream_t st, int64_t n, const void *rh, const void *v, krylov_scalars *sc,
                      double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    bicg_alpha_kernel<<<g, kB, 0, st>>>(n, cd(rh), cd(v), sc, ra);
    return red_finish<1>(st, g, ra, bicg_alpha_op{sc});
}

hipError_t bicg_s(hipStream_t st, int64_t n, const void *r, const void *v, void *s,
                  krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    bicg_s_kernel<<<g, kB, 0, st>>>(n, cd(r), cd(v), md(s), sc, ra);
    return red_finish<1>(st, g, ra, bicg_s_op{sc});
}

hipError_t bicg_omega(hipStream_t st, int64_t n, const void *t, const void *s, krylov_scalars *sc,
                      double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    bicg_omega_kernel<<<g, kB, 0, st>>>(n, cd(t), cd(s), sc, ra);
    return red_finish<2>(st, g, ra, bicg_omega_op{sc});
}

hipError_t bicg_update(hipStream_t st, int64_t n, void *x, void *r, const void *rh, const void *p,
                       const void *s, const void *t, krylov_scalars *sc, double *partials, unsigned *ticket) {
    const int g = reduction_blocks(n);
    const red_args ra = red_for(g, partials, ticket);
    bicg_update_kernel<<<g, kB, 0, st>>>(n, md(x), md(r), cd(rh), cd(p), cd(s),
                                                          cd(t), sc, ra);
    return red_finish<2>(st, g, ra, bicg_update_op{sc});
}

// ------------------------------------------------------------------ mixed-precision helpers
// rt = fp32(r / ||r||) with ||r|| read from device memory.
__global__ void scaled_cast_kernel(int64_t n, const double *__restrict__ r,
                                   const double *__restrict__ norm, float *__restrict__ rt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rt[i] = (float)(r[i] / *norm);
}

hipError_t scaled_cast(hipStream_t s, int64_t n, const double *r, const double *norm, float *rt) {
    if (n == 0) return hipSuccess;
    scaled_cast_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, r, norm, rt);
    return hipGetLastError();
}

// x += ||r|| * fp64(d)
__global__ void refine_update_kernel(int64_t n, double *__restrict__ x, const double *__restrict__ norm,
                                     const float *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] + *norm * (double)d[i];
}

hipError_t refine_update(hipStream_t s, int64_t n, double *x, const double *norm, const float *d) {
    if (n == 0) return hipSuccess;
    refine_update_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, x, norm, d);
    return hipGetLastError();
}

template <typename V>
__global__ void fill_kernel(int64_t n, V *__restrict__ y, V v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

hipError_t fill_zero(hipStream_t s, vt t, int64_t n, void *y) {
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 255) / 256);
    if (t == vt::f64) fill_kernel<double><<<g, 256, 0, s>>>(n, static_cast<double *>(y), 0.0);
    else fill_kernel<float><<<g, 256, 0, s>>>(n, static_cast<float *>(y), 0.0f);
    return hipGetLastError();
}

}  // namespace gko
