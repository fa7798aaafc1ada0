// Host-side launchers of the solver step kernels (see blas1.hip, precond.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "solver_state.hpp"

namespace gko {

hipError_t scalars_reset(hipStream_t s, krylov_scalars *sc, int32_t maxit);

// Single-workgroup CG for small FP64 CSR systems (small_cg.hip): the whole
// solve in one launch.  x: initial guess in, solution out.
struct small_cg_result {
    double bb;         // b.b
    double rr;         // recursive r.r at exit
    double tr2;        // true ||b - A x||^2 at exit
    int32_t iters;     // iterations over all restarts
    int32_t flag;      // solver_flag
    int32_t restarts;  // true-residual restarts
    int32_t pad;
};
// Largest n the device's LDS allows (0 when the device cannot be queried).
int64_t small_cg_max_rows();
// max_len: longest row; rows up to a small bound are kept in registers.
hipError_t small_cg(hipStream_t s, int64_t n, int64_t max_len, const int32_t *rp,
                    const int32_t *col, const double *val, const double *b, double *x, double tol,
                    int32_t maxit, small_cg_result *out);

// CG / PCG.  bs = 0: no preconditioner (z aliases r); bs in {1,2,4,8,16}:
// block-Jacobi with the packed upper triangles `inv` of the explicit inverse
// blocks (values of type t, bj_pack_upper layout).
hipError_t cg_init(hipStream_t s, vt t, int64_t n, const void *b, const void *r, void *z, void *p,
                   const void *inv, int bs, double tol, krylov_scalars *sc, double *partials,
                   unsigned *ticket);
// A matrix as the fused products read it (out = A in together with the
// sums a Krylov step needs next): CSR without long rows, ELL (or HYB with an
// empty tail) or SELL-P without wide slices, in value type t.
struct fused_matrix {
    enum kind { csr = 0, ell = 1, sellp = 2 };
    kind format = csr;
    vt t = vt::f64;
    int64_t n = 0;
    const int32_t *rp = nullptr, *col = nullptr;  // CSR
    const void *val = nullptr;
    int w = 0;                                    // CSR kernel (see csr_kernel_width)
    int lanes = 1;                                // its lanes per row (csr_row_lanes)
    int64_t K = 0, ld = 0;                        // ELL
    const int32_t *ecol = nullptr;
    const void *eval = nullptr;
    const int64_t *sets = nullptr;                // SELL-P
    const int32_t *scol = nullptr;
    const void *sval = nullptr;
};
// The fused products take partials of kFusedMaxSums * kFusedMaxBlocks doubles.
// CG: q = A p with p.q, then alpha (or NOT_SPD).
hipError_t cg_spmv(hipStream_t s, const fused_matrix &A, const void *p, void *q, krylov_scalars *sc,
                   double *partials, unsigned *ticket);
// BiCGSTAB: v = A p with rhat.v, then alpha; t = A s with t.s and t.t, then
// omega.  CGS: t = A p with t.rhat, then alpha.  FP64 only.
hipError_t bicg_spmv_alpha(hipStream_t s, const fused_matrix &A, const void *p, void *v,
                           const void *rh, krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t bicg_spmv_omega(hipStream_t s, const fused_matrix &A, const void *sv, void *t,
                           krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t cgs_spmv_alpha(hipStream_t s, const fused_matrix &A, const void *p, void *t,
                          const void *rh, krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t cg_pq(hipStream_t s, vt t, int64_t n, const void *p, const void *q, krylov_scalars *sc,
                 double *partials, unsigned *ticket);
// flexible: beta = z.(r - r_old) / rho (flexible CG) instead of r.z / rho.
hipError_t cg_update(hipStream_t s, vt t, int64_t n, void *x, void *r, void *z, const void *p,
                     const void *q, const void *inv, int bs, krylov_scalars *sc, double *partials,
                     unsigned *ticket, bool flexible);
hipError_t cg_direction(hipStream_t s, vt t, int64_t n, const void *z, void *p,
                        const krylov_scalars *sc);

// Pipelined (P)CG (Ghysels and Vanroose).  Start from r = b - A x:
// pipe_precond (u = M^-1 r, preconditioned only), w = A u by the format's
// SpMV, pipe_init (m = M^-1 w and the first alpha); then per iteration
// n = A m by the format's SpMV and pipe_update.  bs = 0: u aliases r, m
// aliases w and q aliases s (pass the same pointers).
struct pipe_vectors {
    const void *n;
    void *z, *q, *s, *p, *x, *r, *u, *w, *m;
};
hipError_t pipe_precond(hipStream_t s, vt t, int64_t n, const void *r, void *u, const void *inv,
                        int bs);
hipError_t pipe_init(hipStream_t s, vt t, int64_t n, const void *b, const void *r, void *u,
                     const void *w, void *m, const void *inv, int bs, double tol,
                     krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t pipe_update(hipStream_t s, vt t, int64_t n, const pipe_vectors &v, const void *inv,
                       int bs, krylov_scalars *sc, double *partials, unsigned *ticket);

// BiCGSTAB (FP64).
hipError_t bicg_init(hipStream_t st, int64_t n, const void *b, const void *r, void *rh, void *p,
                     void *v, double tol, krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t bicg_p(hipStream_t st, int64_t n, const void *r, const void *v, void *p,
                  const krylov_scalars *sc);
hipError_t bicg_alpha(hipStream_t st, int64_t n, const void *rh, const void *v, krylov_scalars *sc,
                      double *partials, unsigned *ticket);
hipError_t bicg_s(hipStream_t st, int64_t n, const void *r, const void *v, void *s,
                  krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t bicg_omega(hipStream_t st, int64_t n, const void *t, const void *s, krylov_scalars *sc,
                      double *partials, unsigned *ticket);
hipError_t bicg_update(hipStream_t st, int64_t n, void *x, void *r, const void *rh, const void *p,
                       const void *s, const void *t, krylov_scalars *sc, double *partials,
                       unsigned *ticket);

// CGS (FP64, unpreconditioned; cgs.hip).  init from r = b - A x: rhat = p =
// u = r, rho = r.r; then per iteration t = A p, cgs_alpha, cgs_qwx, t = A w,
// cgs_update, cgs_direction.
hipError_t cgs_init(hipStream_t s, int64_t n, const void *b, const void *r, void *rh, void *p,
                    void *u, double tol, krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t cgs_alpha(hipStream_t s, int64_t n, const void *t, const void *rh, krylov_scalars *sc,
                     double *partials, unsigned *ticket);
hipError_t cgs_qwx(hipStream_t s, int64_t n, const void *u, const void *t, void *q, void *w,
                   void *x, const krylov_scalars *sc);
hipError_t cgs_update(hipStream_t s, int64_t n, void *r, const void *t, const void *rh,
                      krylov_scalars *sc, double *partials, unsigned *ticket);
hipError_t cgs_direction(hipStream_t s, int64_t n, const void *r, const void *q, void *u, void *p,
                         const krylov_scalars *sc);

// Restarted GMRES (FP64, unpreconditioned; gmres.hip).  The host computes
// v0 = b - A x into basis slot 0, calls gmres_cycle_start, then for each step
// j writes w = A v_j into slot j+1 and calls gmres_arnoldi_step, and closes
// the cycle with gmres_cycle_end (x += V_k y).  Flags and scalars live in
// gmres_state; every kernel of a closed cycle returns at once.
constexpr int kGmresMaxKrylov = 128;   // largest restart length
constexpr int kGmresSmallKrylov = 64;  // largest restart length of the one-workgroup solve
constexpr int kGmresMaxBlocks = 2048;  // grid of the multi-vector passes (1024: 12% slower)
struct gmres_state {
    double stop;        // tol * ||b||
    double beta;        // ||b - A x|| at the cycle start
    double est;         // |g_{j+1}|: residual norm of the cycle's least-squares solution
    double hn;          // h_{j+1,j} (the next basis vector's scale)
    double ww;          // w.w after the first Gram-Schmidt round
    int32_t iter;       // Arnoldi steps over all cycles
    int32_t maxit;
    int32_t k;          // columns of the current cycle
    int32_t cycles;
    int32_t done;       // solver_flag of the solve
    int32_t cycle_done; // the current cycle has ended
    int32_t reorth;     // step asked for a second Gram-Schmidt round
    int32_t reorths;    // steps that took a second round
};
struct gmres_work {
    double *partials;      // gmres_partial_elems(n, m)
    double *dot1, *dot2;   // m + 2 each
    double *upd1, *upd2;   // 1 each
    double *hcol;          // m + 1
    double *H;             // (m + 1) * m, row-major
    double *cs, *sn;       // m each
    double *g;             // m + 1
    double *y;             // m
};
int64_t gmres_ld(int64_t n);   // leading dimension of the basis
int64_t gmres_partial_elems(int64_t n, int m);
hipError_t gmres_cycle_start(hipStream_t s, int64_t n, double *V, gmres_state *st,
                             const gmres_work &wk);
hipError_t gmres_arnoldi_step(hipStream_t s, int64_t n, int m, int j, double *V, int64_t ldv,
                              gmres_state *st, const gmres_work &wk);
hipError_t gmres_cycle_end(hipStream_t s, int64_t n, int m, const double *V, int64_t ldv, double *x,
                           gmres_state *st, const gmres_work &wk);
// The whole solve of a small CSR system (n <= gmres_small_max_rows(), m <=
// kGmresSmallKrylov) in one launch of one workgroup, from x (in/out), with
// the basis in V ((m + 1) ldv doubles).  out: iter, cycles, reorths, done,
// est, beta, k as the multi-kernel path leaves them in gmres_state.
int64_t gmres_small_max_rows();
hipError_t gmres_small(hipStream_t s, int64_t n, int m, const int32_t *rp, const int32_t *col,
                       const double *val, const double *b, double *x, double *V, int64_t ldv,
                       double stop, int maxit, gmres_state *out);

// Mixed precision helpers.
hipError_t scaled_cast(hipStream_t s, int64_t n, const double *r, const double *norm, float *rt);
hipError_t refine_update(hipStream_t s, int64_t n, double *x, const double *norm, const float *d);
hipError_t fill_zero(hipStream_t s, vt t, int64_t n, void *y);

// Block-Jacobi: explicit FP64 inverses of the bs x bs diagonal blocks
// (Gauss-Jordan, partial pivoting), one bs*bs row-major slot per block.
// err: device int, set to 1 on a zero pivot.
hipError_t bj_invert(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                     const double *val, int bs, double *inv, int *err);
// The solvers apply the upper triangles of the inverse blocks: the inverse
// of a symmetric block is symmetric, so z = D^-1 r reads bs (bs + 1) / 2
// values per block instead of bs^2 (row by row, see precond.hip).
hipError_t bj_pack_upper(hipStream_t s, int64_t nb, int bs, const double *full, double *packed);

}  // namespace gko
