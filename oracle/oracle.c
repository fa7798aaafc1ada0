/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * Plain, serial, obviously correct CPU implementations of what the GPU
 * library computes.  Only the test suite, the smoke check and the bench's
 * CPU-baseline leg load this file.  It shares no code with the GPU path.
 * Compiled with -O2 -ffp-contract=off: every multiply and add rounds
 * separately, in the order written.
 *
 * The paper (Sec. 6.1) fixes the operation SpMV y = A x and its cost model
 * (memory bound: 16 bytes per COO entry, 12 per CSR entry, 2 flops each), and
 * (Sec. 6.2) that its Krylov solvers are memory bound and generate their
 * subspace with SpMV.  It does not spell out kernels or solvers; the
 * definitions below are the textbook ones, named at each function.
 *
 * Status codes: 0 ok, 6 not converged, 7 breakdown, 8 not SPD, 1 bad input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_BAD 1
#define ORC_NOT_CONVERGED 6
#define ORC_BREAKDOWN 7
#define ORC_NOT_SPD 8

/* ======================================================================
 * SpMV (Sec. 6.1): y <- alpha * A x + beta * y, A in CSR.
 * Entries of a row are summed in ascending storage order.  beta == 0 means
 * y is not read (BLAS convention), so NaN in y does not propagate.
 * ====================================================================== */
void orc_csr_spmv(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                  const double *x, double alpha, double beta, double *y) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s = s + v[k] * x[ci[k]];
        y[i] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[i];
    }
}

/* Magnitude used for SpMV error bounds:
 * absy_i = |alpha| * sum_k |a_ik| |x_k| + |beta| |y_i|  (y_i term dropped if beta == 0).
 * The rounding error of any summation order is bounded by gamma_len * absy_i
 * (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1). */
void orc_csr_spmv_absbound(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                           const double *x, double alpha, double beta, const double *y,
                           double *absy) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s = s + fabs(v[k]) * fabs(x[ci[k]]);
        absy[i] = fabs(alpha) * s + (beta == 0.0 ? 0.0 : fabs(beta) * fabs(y[i]));
    }
}

/* Error-free transformations (Knuth TwoSum; TwoProduct with a correctly
 * rounded fma), used by the compensated dot product Dot2 of Ogita, Rump and
 * Oishi, "Accurate sum and dot product", SIAM J. Sci. Comput. 2005. */
static void two_sum(double a, double b, double *s, double *e) {
    double x = a + b;
    double z = x - a;
    *e = (a - (x - z)) + (b - z);
    *s = x;
}

static void two_prod(double a, double b, double *p, double *e) {
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* Row sums of A x computed as if in twice the working precision (Dot2),
 * then y <- alpha*s + beta*y with the final combination also compensated.
 * A near-exact reference for pinning the plain SpMV's own error. */
void orc_csr_spmv_dot2(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                       const double *x, double alpha, double beta, double *y) {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0, c = 0.0, p, e, q;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            two_prod(v[k], x[ci[k]], &p, &e);
            two_sum(s, p, &s, &q);
            c = c + (q + e);
        }
        double hi = s + c;          /* row sum, nearly exact */
        double lo = c - (hi - s);
        double r, re, t, te;
        two_prod(alpha, hi, &r, &re);
        re = re + alpha * lo;
        if (beta != 0.0) {
            two_prod(beta, y[i], &t, &te);
            two_sum(r, t, &r, &q);
            re = re + (q + te);
        }
        y[i] = r + re;
    }
}

/* ======================================================================
 * Format conversions.  The layouts are this library's own definitions:
 *  COO : row-major sorted triplets (row[k], col[k], val[k]) in CSR order.
 *  ELL : width K, leading dimension ld (>= n); slot (j, i) at j*ld + i holds
 *        the j-th entry of row i, or padding col = -1, val = +0.0.
 *  HYB : ELL(K) holding the first min(len_i, K) entries of each row, and a
 *        COO tail holding the remaining entries in row-major order.
 * ====================================================================== */
void orc_csr_to_coo(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int32_t *row, int32_t *col, double *val) {
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
            row[k] = (int32_t)i;
            col[k] = ci[k];
            val[k] = v[k];
        }
}

int32_t orc_max_row_len(int64_t n, const int32_t *rp) {
    int32_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] - rp[i] > m) m = rp[i + 1] - rp[i];
    return m;
}

static void ell_fill(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     int32_t K, int64_t ld, int32_t *ecol, double *eval) {
    for (int64_t j = 0; j < K; ++j)
        for (int64_t i = 0; i < ld; ++i) {
            int64_t len = (i < n) ? rp[i + 1] - rp[i] : 0;
            if (j < len) {
                ecol[j * ld + i] = ci[rp[i] + j];
                eval[j * ld + i] = v[rp[i] + j];
            } else {
                ecol[j * ld + i] = -1;
                eval[j * ld + i] = 0.0;
            }
        }
}

void orc_csr_to_ell(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int32_t K, int64_t ld, int32_t *ecol, double *eval) {
    ell_fill(n, rp, ci, v, K, ld, ecol, eval);
}

/* HYB split width: the K minimising the bytes one SpMV streams,
 *   cost(K) = n*K*(value_bytes + 4) + (value_bytes + 8) * sum_i max(0, len_i - K),
 * over K in [0, max_len]; ties go to the smaller K.  Evaluated by brute force. */
int32_t orc_hyb_width(int64_t n, const int32_t *rp, int32_t value_bytes) {
    int32_t maxlen = orc_max_row_len(n, rp);
    int32_t best = 0;
    int64_t best_cost = -1;
    for (int32_t K = 0; K <= maxlen; ++K) {
        int64_t tail = 0;
        for (int64_t i = 0; i < n; ++i) {
            int64_t len = rp[i + 1] - rp[i];
            if (len > K) tail += len - K;
        }
        int64_t cost = n * (int64_t)K * (value_bytes + 4) + (int64_t)(value_bytes + 8) * tail;
        if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = K; }
    }
    return best;
}

int64_t orc_hyb_tail_nnz(int64_t n, const int32_t *rp, int32_t K) {
    int64_t tail = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t len = rp[i + 1] - rp[i];
        if (len > K) tail += len - K;
    }
    return tail;
}

void orc_csr_to_hyb(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    int32_t K, int64_t ld, int32_t *ecol, double *eval,
                    int32_t *trow, int32_t *tcol, double *tval) {
    ell_fill(n, rp, ci, v, K, ld, ecol, eval);
    int64_t t = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = rp[i] + K; k < rp[i + 1]; ++k) {
            trow[t] = (int32_t)i;
            tcol[t] = ci[k];
            tval[t] = v[k];
            ++t;
        }
}

/* COO (row-major sorted) back to CSR: count, prefix sum, copy. */
void orc_coo_to_csr(int64_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                    const double *val, int32_t *rp, int32_t *ci, double *v) {
    for (int64_t i = 0; i <= n; ++i) rp[i] = 0;
    for (int64_t k = 0; k < nnz; ++k) rp[row[k] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    for (int64_t k = 0; k < nnz; ++k) { ci[k] = col[k]; v[k] = val[k]; }
}

/* ELL (and HYB = ELL + COO tail) back to CSR: padding (col = -1) dropped. */
void orc_hyb_to_csr(int64_t n, int32_t K, int64_t ld, const int32_t *ecol, const double *eval,
                    int64_t tnnz, const int32_t *trow, const int32_t *tcol, const double *tval,
                    int32_t *rp, int32_t *ci, double *v) {
    int64_t k = 0, t = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < K; ++j)
            if (ecol[j * ld + i] >= 0) { ci[k] = ecol[j * ld + i]; v[k] = eval[j * ld + i]; ++k; }
        while (t < tnnz && trow[t] == i) { ci[k] = tcol[t]; v[k] = tval[t]; ++k; ++t; }
        rp[i + 1] = (int32_t)k;
    }
}

/* SELL-P, the sliced ELL format with padding (Anzt, Tomov and Dongarra,
 * "Implementing a sparse matrix vector product for the SELL-C/SELL-C-sigma
 * formats on NVIDIA GPUs", 2014), without row sorting and with stride
 * factor 1: rows are grouped in slices of C consecutive rows; slice s is
 * padded to its own width w_s (its longest row) and stored column-major
 * inside the slice.  Slot (j, r) of slice s -- the j-th entry of row
 * i = s*C + r -- is at sets[s] + j*C + r, with sets[0] = 0 and
 * sets[s+1] = sets[s] + w_s*C.  Padding (and rows i >= n of the last slice)
 * is col = -1, val = +0.0.  Returns the number of slots, sets[nslices]. */
int64_t orc_sellp_layout(int64_t n, const int32_t *rp, int32_t C, int32_t *widths, int64_t *sets) {
    const int64_t ns = (n + C - 1) / C;
    sets[0] = 0;
    for (int64_t s = 0; s < ns; ++s) {
        int32_t w = 0;
        for (int64_t i = s * C; i < (s + 1) * C && i < n; ++i)
            if (rp[i + 1] - rp[i] > w) w = rp[i + 1] - rp[i];
        widths[s] = w;
        sets[s + 1] = sets[s] + (int64_t)w * C;
    }
    return sets[ns];
}

void orc_csr_to_sellp(int64_t n, const int32_t *rp, const int32_t *ci, const double *v, int32_t C,
                      const int32_t *widths, const int64_t *sets, int32_t *scol, double *sval) {
    const int64_t ns = (n + C - 1) / C;
    for (int64_t s = 0; s < ns; ++s)
        for (int64_t j = 0; j < widths[s]; ++j)
            for (int64_t r = 0; r < C; ++r) {
                const int64_t i = s * C + r, slot = sets[s] + j * C + r;
                const int64_t len = i < n ? rp[i + 1] - rp[i] : 0;
                if (j < len) {
                    scol[slot] = ci[rp[i] + j];
                    sval[slot] = v[rp[i] + j];
                } else {
                    scol[slot] = -1;
                    sval[slot] = 0.0;
                }
            }
}

/* SELL-P back to CSR: padding dropped, entries of a row in slot order. */
void orc_sellp_to_csr(int64_t n, int32_t C, const int32_t *widths, const int64_t *sets,
                      const int32_t *scol, const double *sval, int32_t *rp, int32_t *ci, double *v) {
    int64_t k = 0;
    rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s = i / C, r = i % C;
        for (int64_t j = 0; j < widths[s]; ++j) {
            const int64_t slot = sets[s] + j * C + r;
            if (scol[slot] >= 0) { ci[k] = scol[slot]; v[k] = sval[slot]; ++k; }
        }
        rp[i + 1] = (int32_t)k;
    }
}

/* ======================================================================
 * Dot products and norms: serial ascending sums.
 * ====================================================================== */
double orc_dot(int64_t n, const double *x, const double *y) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + x[i] * y[i];
    return s;
}

double orc_norm2(int64_t n, const double *x) { return sqrt(orc_dot(n, x, x)); }

/* ======================================================================
 * Block-Jacobi preconditioner with uniform blocks of bs consecutive rows
 * (the last block is short when bs does not divide n).  Each diagonal block
 * D_k = A[blk, blk] is inverted explicitly by Gauss-Jordan elimination with
 * partial pivoting (ties keep the smaller row index).  inv holds one bs*bs
 * row-major slot per block; a short block uses the top-left corner.
 * Returns ORC_BREAKDOWN on a zero pivot.
 * ====================================================================== */
int orc_bj_invert(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                  int32_t bs, double *inv) {
    int64_t nb = (n + bs - 1) / bs;
    double *a = (double *)malloc(sizeof(double) * bs * bs);
    double *e = (double *)malloc(sizeof(double) * bs * bs);
    int rc = ORC_OK;
    for (int64_t b = 0; b < nb && rc == ORC_OK; ++b) {
        int64_t r0 = b * bs;
        int m = (int)((r0 + bs <= n) ? bs : n - r0);
        for (int i = 0; i < bs * bs; ++i) { a[i] = 0.0; e[i] = 0.0; }
        for (int i = 0; i < m; ++i) {
            e[i * bs + i] = 1.0;
            for (int64_t k = rp[r0 + i]; k < rp[r0 + i + 1]; ++k) {
                int64_t c = ci[k];
                if (c >= r0 && c < r0 + m) a[i * bs + (c - r0)] = v[k];
            }
        }
        for (int c = 0; c < m; ++c) {
            int piv = c;
            for (int r = c + 1; r < m; ++r)
                if (fabs(a[r * bs + c]) > fabs(a[piv * bs + c])) piv = r;
            if (a[piv * bs + c] == 0.0) { rc = ORC_BREAKDOWN; break; }
            if (piv != c)
                for (int j = 0; j < m; ++j) {
                    double t = a[c * bs + j]; a[c * bs + j] = a[piv * bs + j]; a[piv * bs + j] = t;
                    t = e[c * bs + j]; e[c * bs + j] = e[piv * bs + j]; e[piv * bs + j] = t;
                }
            double d = a[c * bs + c];
            for (int j = 0; j < m; ++j) { a[c * bs + j] = a[c * bs + j] / d; e[c * bs + j] = e[c * bs + j] / d; }
            for (int r = 0; r < m; ++r) {
                if (r == c) continue;
                double f = a[r * bs + c];
                if (f == 0.0) continue;
                for (int j = 0; j < m; ++j) {
                    a[r * bs + j] = a[r * bs + j] - f * a[c * bs + j];
                    e[r * bs + j] = e[r * bs + j] - f * e[c * bs + j];
                }
            }
        }
        for (int i = 0; i < bs * bs; ++i) inv[b * bs * bs + i] = e[i];
    }
    free(a);
    free(e);
    return rc;
}

/* z_blk = D_k^{-1} r_blk, each row an ascending dot over the block. */
void orc_bj_apply(int64_t n, int32_t bs, const double *inv, const double *r, double *z) {
    int64_t nb = (n + bs - 1) / bs;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t r0 = b * bs;
        int m = (int)((r0 + bs <= n) ? bs : n - r0);
        for (int i = 0; i < m; ++i) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) s = s + inv[b * bs * bs + i * bs + j] * r[r0 + j];
            z[r0 + i] = s;
        }
    }
}

/* ======================================================================
 * Conjugate gradients, optionally preconditioned (Hestenes and Stiefel 1952;
 * Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Alg. 9.1):
 *   r = b - A x;  z = M^{-1} r;  p = z;  rho = r.z
 *   repeat: q = A p;  alpha = rho / (p.q);  x += alpha p;  r -= alpha q;
 *           stop when ||r||_2 <= tol ||b||_2;
 *           z = M^{-1} r;  rho' = r.z;  beta = rho'/rho;  p = z + beta p.
 * p.q <= 0 means A is not SPD.  When the recursive residual meets tol, the
 * true residual b - A x is checked; if it does not meet tol the iteration is
 * restarted from the current x (at most twice).  ||b|| = 0 gives x = 0.
 * out[0] = iterations, out[1] = final recursive ||r||/||b||,
 * out[2] = true ||b - A x||/||b||, out[3] = restarts.
 * ====================================================================== */
int orc_cg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
           const double *b, double *x, double tol, int32_t maxit,
           const double *bj_inv, int32_t bs, double *out) {
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0, restarts = 0;
    double bnorm = orc_norm2(n, b), rnorm = 0.0, tnorm = 0.0;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (;;) {
        /* (re)start: r = b - A x, z = M^{-1} r, p = z */
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
        rnorm = orc_norm2(n, r);
        int conv = rnorm <= tol * bnorm;
        if (!conv) {
            if (bj_inv) orc_bj_apply(n, bs, bj_inv, r, z);
            else for (int64_t i = 0; i < n; ++i) z[i] = r[i];
            for (int64_t i = 0; i < n; ++i) p[i] = z[i];
            double rho = orc_dot(n, r, z);
            while (it < maxit) {
                orc_csr_spmv(n, rp, ci, v, p, 1.0, 0.0, q);
                double pq = orc_dot(n, p, q);
                if (!(pq > 0.0)) { rc = isnan(pq) ? ORC_BREAKDOWN : ORC_NOT_SPD; ++it; goto done; }
                double alpha = rho / pq;
                for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
                for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
                ++it;
                rnorm = orc_norm2(n, r);
                if (isnan(rnorm) || isinf(rnorm)) { rc = ORC_BREAKDOWN; goto done; }
                if (rnorm <= tol * bnorm) { conv = 1; break; }
                if (bj_inv) orc_bj_apply(n, bs, bj_inv, r, z);
                else for (int64_t i = 0; i < n; ++i) z[i] = r[i];
                double rho_new = orc_dot(n, r, z);
                double beta = rho_new / rho;
                rho = rho_new;
                for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            }
        }
        if (!conv) { rc = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        if (tnorm <= tol * bnorm) { rc = ORC_OK; break; }
        if (restarts == 2 || it >= maxit) { rc = ORC_NOT_CONVERGED; break; }
        ++restarts;
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        out[0] = it;
        out[1] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? tnorm / bnorm : 0.0;
        out[3] = restarts;
    }
    free(r); free(z); free(p); free(q);
    return rc;
}

/* ======================================================================
 * BiCGSTAB (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992;
 * Saad Alg. 7.7), unpreconditioned, shadow residual rhat = r0:
 *   rho = rhat.r;  beta = (rho/rho_old)(alpha/omega);  p = r + beta(p - omega v)
 *   v = A p;  alpha = rho/(rhat.v);  s = r - alpha v  (stop: x += alpha p)
 *   t = A s;  omega = (t.s)/(t.t);  x += alpha p + omega s;  r = s - omega t.
 * Breakdown when |rho|, |rhat.v| or t.t falls below 1e-300, or omega == 0.
 * out[0] = iterations, out[1] = recursive relres, out[2] = true relres.
 * ====================================================================== */
int orc_bicgstab(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 const double *b, double *x, double tol, int32_t maxit, double *out) {
    double *r = (double *)calloc(n, sizeof(double));
    double *rh = (double *)calloc(n, sizeof(double));
    double *p = (double *)calloc(n, sizeof(double));
    double *vv = (double *)calloc(n, sizeof(double));
    double *s = (double *)calloc(n, sizeof(double));
    double *t = (double *)calloc(n, sizeof(double));
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0;
    double bnorm = orc_norm2(n, b), rnorm;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        rnorm = 0.0;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
    for (int64_t i = 0; i < n; ++i) rh[i] = r[i];
    rnorm = orc_norm2(n, r);
    if (rnorm <= tol * bnorm) { rc = ORC_OK; goto done; }
    double rho_old = 1.0, alpha = 1.0, omega = 1.0;
    while (it < maxit) {
        double rho = orc_dot(n, rh, r);
        if (!(fabs(rho) >= 1e-300)) { rc = ORC_BREAKDOWN; goto done; }
        double beta = (rho / rho_old) * (alpha / omega);
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * vv[i]);
        orc_csr_spmv(n, rp, ci, v, p, 1.0, 0.0, vv);
        double rv = orc_dot(n, rh, vv);
        if (!(fabs(rv) >= 1e-300)) { rc = ORC_BREAKDOWN; goto done; }
        alpha = rho / rv;
        for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * vv[i];
        ++it;
        double snorm = orc_norm2(n, s);
        if (snorm <= tol * bnorm) {
            for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
            rnorm = snorm;
            rc = ORC_OK;
            goto done;
        }
        orc_csr_spmv(n, rp, ci, v, s, 1.0, 0.0, t);
        double tt = orc_dot(n, t, t);
        if (!(tt >= 1e-300)) { rc = ORC_BREAKDOWN; goto done; }
        omega = orc_dot(n, t, s) / tt;
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i] + omega * s[i];
        for (int64_t i = 0; i < n; ++i) r[i] = s[i] - omega * t[i];
        rho_old = rho;
        rnorm = orc_norm2(n, r);
        if (isnan(rnorm)) { rc = ORC_BREAKDOWN; goto done; }
        if (rnorm <= tol * bnorm) { rc = ORC_OK; goto done; }
        if (omega == 0.0) { rc = ORC_BREAKDOWN; goto done; }
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) t[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, t);
        out[0] = it;
        out[1] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? orc_norm2(n, t) / bnorm : 0.0;
    }
    free(r); free(rh); free(p); free(vv); free(s); free(t);
    return rc;
}

/* ======================================================================
 * Pipelined preconditioned CG (Ghysels and Vanroose, Parallel Computing 40,
 * 2014): CG rearranged so that one global reduction per iteration (the dots
 * gamma = r.u, delta = w.u and r.r) can overlap the preconditioner and the
 * product.  With u = M^{-1} r and w = A u kept by recurrences:
 *   start: r = b - A x;  u = M^{-1} r;  w = A u
 *   repeat: gamma = r.u;  delta = w.u;  m = M^{-1} w;  n = A m;
 *           first step: beta = 0, alpha = gamma / delta;  later:
 *           beta = gamma / gamma_old, alpha = gamma / (delta - beta gamma / alpha_old)
 *           z = n + beta z;  q = m + beta q;  s = w + beta s;  p = u + beta p;
 *           x += alpha p;  r -= alpha s;  u -= alpha q;  w -= alpha z;
 *           stop when ||r||_2 <= tol ||b||_2.
 * The denominator of alpha is p.Ap in exact arithmetic: <= 0 means A is not
 * SPD.  In exact arithmetic the iterates are CG's.  True-residual check and
 * restarts (at most two) and the outputs as orc_cg.
 * ====================================================================== */
int orc_pipecg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
               const double *b, double *x, double tol, int32_t maxit,
               const double *bj_inv, int32_t bs, double *out) {
    double *r = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *u = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *w = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *m = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *nn = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *z = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *q = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *sv = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *p = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0, restarts = 0;
    double bnorm = orc_norm2(n, b), rnorm = 0.0, tnorm = 0.0;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (;;) {
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
        rnorm = orc_norm2(n, r);
        int conv = rnorm <= tol * bnorm;
        if (!conv) {
            if (bj_inv) orc_bj_apply(n, bs, bj_inv, r, u);
            else for (int64_t i = 0; i < n; ++i) u[i] = r[i];
            orc_csr_spmv(n, rp, ci, v, u, 1.0, 0.0, w);
            double gamma_old = 0.0, alpha_old = 0.0;
            int first = 1;
            while (it < maxit) {
                double gamma = orc_dot(n, r, u), delta = orc_dot(n, w, u);
                if (bj_inv) orc_bj_apply(n, bs, bj_inv, w, m);
                else for (int64_t i = 0; i < n; ++i) m[i] = w[i];
                orc_csr_spmv(n, rp, ci, v, m, 1.0, 0.0, nn);
                double alpha, beta, den;
                if (first) {
                    beta = 0.0;
                    den = delta;
                } else {
                    beta = gamma / gamma_old;
                    den = delta - beta * gamma / alpha_old;
                }
                if (!(den > 0.0)) { rc = isnan(den) ? ORC_BREAKDOWN : ORC_NOT_SPD; ++it; goto done; }
                alpha = gamma / den;
                for (int64_t i = 0; i < n; ++i) {
                    z[i] = nn[i] + beta * z[i];
                    q[i] = m[i] + beta * q[i];
                    sv[i] = w[i] + beta * sv[i];
                    p[i] = u[i] + beta * p[i];
                }
                for (int64_t i = 0; i < n; ++i) {
                    x[i] = x[i] + alpha * p[i];
                    r[i] = r[i] - alpha * sv[i];
                    u[i] = u[i] - alpha * q[i];
                    w[i] = w[i] - alpha * z[i];
                }
                ++it;
                first = 0;
                gamma_old = gamma;
                alpha_old = alpha;
                rnorm = orc_norm2(n, r);
                if (isnan(rnorm) || isinf(rnorm)) { rc = ORC_BREAKDOWN; goto done; }
                if (rnorm <= tol * bnorm) { conv = 1; break; }
            }
        }
        if (!conv) { rc = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        if (tnorm <= tol * bnorm) { rc = ORC_OK; break; }
        if (restarts == 2 || it >= maxit) { rc = ORC_NOT_CONVERGED; break; }
        ++restarts;
        /* the recurrences restart from scratch: z, q, s, p are multiplied by beta = 0 */
        for (int64_t i = 0; i < n; ++i) { z[i] = 0.0; q[i] = 0.0; sv[i] = 0.0; p[i] = 0.0; }
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        out[0] = it;
        out[1] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? tnorm / bnorm : 0.0;
        out[3] = restarts;
    }
    free(r); free(u); free(w); free(m); free(nn); free(z); free(q); free(sv); free(p);
    return rc;
}

/* ======================================================================
 * Flexible CG (Notay, SIAM J. Sci. Comput. 22, 2000, truncated to one
 * previous direction), optionally preconditioned.  CG with the
 * Polak-Ribiere coefficient
 *   beta = z_{k+1}.(r_{k+1} - r_k) / (z_k.r_k),
 * which keeps consecutive directions A-conjugate when the preconditioner is
 * not a fixed symmetric operator; with a fixed SPD preconditioner it equals
 * CG's beta in exact arithmetic (z_{k+1}.r_k = 0).  Stopping, true-residual
 * restarts and outputs as orc_cg.
 * ====================================================================== */
int orc_fcg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
            const double *b, double *x, double tol, int32_t maxit,
            const double *bj_inv, int32_t bs, double *out) {
    double *r = (double *)malloc(sizeof(double) * n);
    double *r_old = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0, restarts = 0;
    double bnorm = orc_norm2(n, b), rnorm = 0.0, tnorm = 0.0;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (;;) {
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
        rnorm = orc_norm2(n, r);
        int conv = rnorm <= tol * bnorm;
        if (!conv) {
            if (bj_inv) orc_bj_apply(n, bs, bj_inv, r, z);
            else for (int64_t i = 0; i < n; ++i) z[i] = r[i];
            for (int64_t i = 0; i < n; ++i) p[i] = z[i];
            double rho = orc_dot(n, r, z);
            while (it < maxit) {
                orc_csr_spmv(n, rp, ci, v, p, 1.0, 0.0, q);
                double pq = orc_dot(n, p, q);
                if (!(pq > 0.0)) { rc = isnan(pq) ? ORC_BREAKDOWN : ORC_NOT_SPD; ++it; goto done; }
                double alpha = rho / pq;
                for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
                for (int64_t i = 0; i < n; ++i) r_old[i] = r[i];
                for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
                ++it;
                rnorm = orc_norm2(n, r);
                if (isnan(rnorm) || isinf(rnorm)) { rc = ORC_BREAKDOWN; goto done; }
                if (rnorm <= tol * bnorm) { conv = 1; break; }
                if (bj_inv) orc_bj_apply(n, bs, bj_inv, r, z);
                else for (int64_t i = 0; i < n; ++i) z[i] = r[i];
                double rho_new = orc_dot(n, r, z);
                double zt = 0.0;   /* z_{k+1}.(r_{k+1} - r_k) */
                for (int64_t i = 0; i < n; ++i) zt += z[i] * (r[i] - r_old[i]);
                double beta = zt / rho;
                rho = rho_new;
                for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
            }
        }
        if (!conv) { rc = ORC_NOT_CONVERGED; break; }
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        if (tnorm <= tol * bnorm) { rc = ORC_OK; break; }
        if (restarts == 2 || it >= maxit) { rc = ORC_NOT_CONVERGED; break; }
        ++restarts;
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) q[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, q);
        tnorm = orc_norm2(n, q);
        out[0] = it;
        out[1] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? tnorm / bnorm : 0.0;
        out[3] = restarts;
    }
    free(r); free(r_old); free(z); free(p); free(q);
    return rc;
}

/* ======================================================================
 * CGS, conjugate gradients squared (Sonneveld, SIAM J. Sci. Stat. Comput.
 * 10, 1989; Saad Alg. 7.5), unpreconditioned, shadow residual rhat = r0:
 *   p = u = r0;  rho = r.rhat
 *   repeat: v = A p;  alpha = rho / (v.rhat);  q = u - alpha v;
 *           x += alpha (u + q);  r -= alpha A (u + q);
 *           stop when ||r||_2 <= tol ||b||_2;
 *           rho' = r.rhat;  beta = rho'/rho;  u = r + beta q;
 *           p = u + beta (q + beta p).
 * Breakdown when |rho| or |v.rhat| falls below 1e-300.
 * out[0] = iterations, out[1] = recursive relres, out[2] = true relres.
 * ====================================================================== */
int orc_cgs(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
            const double *b, double *x, double tol, int32_t maxit, double *out) {
    double *r = (double *)calloc(n, sizeof(double));
    double *rh = (double *)calloc(n, sizeof(double));
    double *p = (double *)calloc(n, sizeof(double));
    double *u = (double *)calloc(n, sizeof(double));
    double *q = (double *)calloc(n, sizeof(double));
    double *w = (double *)calloc(n, sizeof(double));
    double *t = (double *)calloc(n, sizeof(double));
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0;
    double bnorm = orc_norm2(n, b), rnorm = 0.0;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) r[i] = b[i];
    orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
    rnorm = orc_norm2(n, r);
    if (rnorm <= tol * bnorm) { rc = ORC_OK; goto done; }
    for (int64_t i = 0; i < n; ++i) { rh[i] = r[i]; p[i] = r[i]; u[i] = r[i]; }
    double rho = orc_dot(n, r, rh);
    while (it < maxit) {
        if (!(fabs(rho) >= 1e-300)) { rc = ORC_BREAKDOWN; goto done; }
        orc_csr_spmv(n, rp, ci, v, p, 1.0, 0.0, t);          /* t = A p */
        double vr = orc_dot(n, t, rh);
        if (!(fabs(vr) >= 1e-300)) { rc = ORC_BREAKDOWN; goto done; }
        double alpha = rho / vr;
        for (int64_t i = 0; i < n; ++i) q[i] = u[i] - alpha * t[i];
        for (int64_t i = 0; i < n; ++i) w[i] = u[i] + q[i];
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + alpha * w[i];
        orc_csr_spmv(n, rp, ci, v, w, 1.0, 0.0, t);          /* t = A (u + q) */
        for (int64_t i = 0; i < n; ++i) r[i] = r[i] - alpha * t[i];
        ++it;
        rnorm = orc_norm2(n, r);
        if (isnan(rnorm) || isinf(rnorm)) { rc = ORC_BREAKDOWN; goto done; }
        if (rnorm <= tol * bnorm) { rc = ORC_OK; goto done; }
        double rho_new = orc_dot(n, r, rh);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) u[i] = r[i] + beta * q[i];
        for (int64_t i = 0; i < n; ++i) p[i] = u[i] + beta * (q[i] + beta * p[i]);
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) t[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, t);
        out[0] = it;
        out[1] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? orc_norm2(n, t) / bnorm : 0.0;
    }
    free(r); free(rh); free(p); free(u); free(q); free(w); free(t);
    return rc;
}

/* ======================================================================
 * Restarted GMRES(m) (Saad and Schultz, SIAM J. Sci. Stat. Comput. 7, 1986;
 * Saad Alg. 6.9 with the Givens-rotation least-squares update of Sec. 6.5.3),
 * unpreconditioned.  A cycle: r = b - A x, beta = ||r||, v_0 = r / beta,
 * g = beta e_0; for j = 0, 1, ...: w = A v_j; modified Gram-Schmidt
 * h_ij = w.v_i, w -= h_ij v_i (i = 0..j); h_{j+1,j} = ||w||; the earlier
 * rotations applied to column j, then the rotation (c, s) with
 * c = h_jj / d, s = h_{j+1,j} / d, d = sqrt(h_jj^2 + h_{j+1,j}^2) that zeroes
 * h_{j+1,j}, applied to g (g_{j+1} = -s g_j, g_j = c g_j).  |g_{j+1}| is the
 * residual norm of the cycle's least-squares solution.  The cycle ends after
 * m steps, when |g_{j+1}| <= tol ||b||, when h_{j+1,j} = 0 (the Krylov space
 * is invariant) or at maxit; then R y = g (back substitution) and
 * x += sum_i y_i v_i.  The true residual starts the next cycle and decides
 * convergence.  out[0] = iterations (Arnoldi steps), out[1] = |g| / ||b|| of
 * the last step, out[2] = true relres, out[3] = cycles.
 * ====================================================================== */
int orc_gmres(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const double *b, double *x, double tol, int32_t maxit, int32_t m, double *out) {
    if (m < 1) return ORC_BAD;
    double *V = (double *)calloc((size_t)(m + 1) * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *H = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));  /* H[i*m + j] */
    double *cs = (double *)calloc(m, sizeof(double));
    double *sn = (double *)calloc(m, sizeof(double));
    double *g = (double *)calloc(m + 1, sizeof(double));
    double *y = (double *)calloc(m, sizeof(double));
    double *w = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    int rc = ORC_NOT_CONVERGED;
    int32_t it = 0, cycles = 0;
    double bnorm = orc_norm2(n, b), est = 0.0, tnorm = 0.0;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (;;) {
        for (int64_t i = 0; i < n; ++i) w[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, w);
        double beta = orc_norm2(n, w);
        tnorm = beta;
        if (isnan(beta) || isinf(beta)) { rc = ORC_BREAKDOWN; goto done; }
        if (beta <= tol * bnorm) { rc = ORC_OK; goto done; }
        if (it >= maxit) { rc = ORC_NOT_CONVERGED; goto done; }
        ++cycles;
        for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
        for (int j = 0; j <= m; ++j) g[j] = 0.0;
        g[0] = beta;
        int k = 0;   /* columns of this cycle */
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
            orc_csr_spmv(n, rp, ci, v, vj, 1.0, 0.0, w);
            for (int i = 0; i <= j; ++i) {
                const double *vi = V + (size_t)i * n;
                double h = orc_dot(n, w, vi);
                H[i * m + j] = h;
                for (int64_t l = 0; l < n; ++l) w[l] = w[l] - h * vi[l];
            }
            double hn = orc_norm2(n, w);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                double a = H[i * m + j], c = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a + sn[i] * c;
                H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[j * m + j];
            double d = sqrt(a * a + hn * hn);
            if (!(d > 0.0)) { rc = ORC_BREAKDOWN; goto done; }
            cs[j] = a / d;
            sn[j] = hn / d;
            H[j * m + j] = d;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++it;
            k = j + 1;
            est = fabs(g[j + 1]);
            if (isnan(est)) { rc = ORC_BREAKDOWN; goto done; }
            if (est <= tol * bnorm || hn == 0.0 || it >= maxit) break;
            for (int64_t l = 0; l < n; ++l) vn[l] = w[l] / hn;
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s = s - H[i * m + l] * y[l];
            y[i] = s / H[i * m + i];
        }
        for (int i = 0; i < k; ++i) {
            const double *vi = V + (size_t)i * n;
            for (int64_t l = 0; l < n; ++l) x[l] = x[l] + y[i] * vi[l];
        }
    }
done:
    if (out) {
        for (int64_t i = 0; i < n; ++i) w[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, w);
        out[0] = it;
        out[1] = bnorm > 0.0 ? est / bnorm : 0.0;
        out[2] = bnorm > 0.0 ? orc_norm2(n, w) / bnorm : 0.0;
        out[3] = cycles;
    }
    free(V); free(H); free(cs); free(sn); free(g); free(y); free(w);
    return rc;
}

/* ======================================================================
 * Mixed-precision iterative refinement around an FP32 inner PCG.
 * Outer loop in FP64:  r = b - A x;  stop when ||r|| <= tol ||b||;
 *   rt = fp32(r / ||r||);  solve A32 d = rt approximately;  x += ||r|| fp64(d).
 * Inner PCG (same steps as orc_cg) with FP32 matrix values, FP32 vectors and
 * FP32 block-Jacobi inverse (rounded from the FP64 one); SpMV rows summed in
 * FP32; dot products accumulate FP64 products of the FP32 data in FP64;
 * scalars alpha, beta are FP64 and each vector update is done in FP64 and
 * rounded once to FP32.  Inner stop: ||r_inner|| <= tau_k ||rt||, or
 * max_inner iterations, where step k asks only for the reduction still
 * missing (with a factor 2 of margin), but never less than inner_tol:
 *   tau_k = max(inner_tol, 0.5 tol ||b|| / ||r_k||).
 * Outer stop: converged, max_outer, or a residual that did not halve
 * (stagnation, -> not converged).  maxit caps the inner iterations summed
 * over all outer steps: step k may run at most min(max_inner, maxit - done)
 * of them, and a solve whose budget is spent stops as not converged.
 * out[0] = total inner iterations, out[1] = outer iterations,
 * out[2] = final true relres.  inner_counts (may be NULL; room for
 * max_outer entries) receives the inner iterations of each outer step.
 * ====================================================================== */
static void spmv_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *v,
                     const float *x, float *y) {
    for (int64_t i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s = s + v[k] * x[ci[k]];
        y[i] = s;
    }
}

static double dot_f32(int64_t n, const float *x, const float *y) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = s + (double)x[i] * (double)y[i];
    return s;
}

void orc_bj_apply_f32(int64_t n, int32_t bs, const float *inv, const float *r, float *z) {
    int64_t nb = (n + bs - 1) / bs;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t r0 = b * bs;
        int m = (int)((r0 + bs <= n) ? bs : n - r0);
        for (int i = 0; i < m; ++i) {
            float s = 0.0f;
            for (int j = 0; j < m; ++j) s = s + inv[b * bs * bs + i * bs + j] * r[r0 + j];
            z[r0 + i] = s;
        }
    }
}

/* Inner FP32 PCG on A32 d = rhs, d starts at 0. Returns iterations done;
 * *status gets ORC_OK, ORC_NOT_CONVERGED (max reached), ORC_NOT_SPD or ORC_BREAKDOWN. */
static int32_t pcg_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *v32,
                       const float *rhs, float *d, double tol, int32_t maxit,
                       const float *inv32, int32_t bs, float *r, float *z, float *p, float *q,
                       int *status) {
    for (int64_t i = 0; i < n; ++i) { d[i] = 0.0f; r[i] = rhs[i]; }
    double rn0 = sqrt(dot_f32(n, r, r));
    int32_t it = 0;
    *status = ORC_OK;
    if (rn0 == 0.0) return 0;
    if (inv32) orc_bj_apply_f32(n, bs, inv32, r, z); else memcpy(z, r, sizeof(float) * n);
    memcpy(p, z, sizeof(float) * n);
    double rho = dot_f32(n, r, z);
    while (it < maxit) {
        spmv_f32(n, rp, ci, v32, p, q);
        double pq = dot_f32(n, p, q);
        if (!(pq > 0.0)) { *status = isnan(pq) ? ORC_BREAKDOWN : ORC_NOT_SPD; return it + 1; }
        double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) d[i] = (float)((double)d[i] + alpha * (double)p[i]);
        for (int64_t i = 0; i < n; ++i) r[i] = (float)((double)r[i] - alpha * (double)q[i]);
        ++it;
        double rn = sqrt(dot_f32(n, r, r));
        if (isnan(rn)) { *status = ORC_BREAKDOWN; return it; }
        if (rn <= tol * rn0) return it;
        if (inv32) orc_bj_apply_f32(n, bs, inv32, r, z); else memcpy(z, r, sizeof(float) * n);
        double rho_new = dot_f32(n, r, z);
        double beta = rho_new / rho;
        rho = rho_new;
        for (int64_t i = 0; i < n; ++i) p[i] = (float)((double)z[i] + beta * (double)p[i]);
    }
    *status = ORC_NOT_CONVERGED;
    return it;
}

/* The inner solve on its own: FP32 PCG on A32 d = rhs from d = 0 to
 * ||r|| <= tol ||rhs|| or maxit iterations (inv32 may be NULL: no
 * preconditioner).  Returns the iterations done; *status as pcg_f32. */
int32_t orc_pcg_f32(int64_t n, const int32_t *rp, const int32_t *ci, const float *v32,
                    const float *rhs, float *d, double tol, int32_t maxit,
                    const float *inv32, int32_t bs, int32_t *status) {
    float *w = (float *)malloc(sizeof(float) * (size_t)(4 * n + 4));
    int st = ORC_OK;
    int32_t it = pcg_f32(n, rp, ci, v32, rhs, d, tol, maxit, inv32, bs, w, w + n, w + 2 * n,
                         w + 3 * n, &st);
    free(w);
    *status = st;
    return it;
}

int orc_ir_cg(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const double *b, double *x, double tol, int32_t max_outer,
              double inner_tol, int32_t max_inner, int32_t maxit, const double *bj_inv,
              int32_t bs, double *out, int32_t *inner_counts) {
    float *v32 = (float *)malloc(sizeof(float) * (size_t)rp[n]);
    float *inv32 = NULL;
    float *rt = (float *)malloc(sizeof(float) * n), *d = (float *)malloc(sizeof(float) * n);
    float *w1 = (float *)malloc(sizeof(float) * n), *w2 = (float *)malloc(sizeof(float) * n);
    float *w3 = (float *)malloc(sizeof(float) * n), *w4 = (float *)malloc(sizeof(float) * n);
    double *r = (double *)malloc(sizeof(double) * n);
    for (int64_t k = 0; k < rp[n]; ++k) v32[k] = (float)v[k];
    if (bj_inv) {
        int64_t nb = (n + bs - 1) / bs;
        inv32 = (float *)malloc(sizeof(float) * nb * bs * bs);
        for (int64_t k = 0; k < nb * bs * bs; ++k) inv32[k] = (float)bj_inv[k];
    }
    int rc = ORC_NOT_CONVERGED;
    int32_t outer = 0;
    int64_t inner_total = 0;
    double bnorm = orc_norm2(n, b), rnorm = 0.0, prev = INFINITY;
    if (!(bnorm > 0.0)) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        rc = (bnorm == 0.0) ? ORC_OK : ORC_BREAKDOWN;
        goto done;
    }
    for (;;) {
        for (int64_t i = 0; i < n; ++i) r[i] = b[i];
        orc_csr_spmv(n, rp, ci, v, x, -1.0, 1.0, r);
        rnorm = orc_norm2(n, r);
        if (isnan(rnorm)) { rc = ORC_BREAKDOWN; break; }
        if (rnorm <= tol * bnorm) { rc = ORC_OK; break; }
        if (outer >= max_outer || !(rnorm <= 0.5 * prev) || inner_total >= maxit) {
            rc = ORC_NOT_CONVERGED;
            break;
        }
        prev = rnorm;
        for (int64_t i = 0; i < n; ++i) rt[i] = (float)(r[i] / rnorm);
        double tau = 0.5 * (tol * bnorm / rnorm);
        if (tau < inner_tol) tau = inner_tol;
        int32_t cap = max_inner;
        if (maxit - inner_total < cap) cap = (int32_t)(maxit - inner_total);
        int st;
        int32_t done_k = pcg_f32(n, rp, ci, v32, rt, d, tau, cap, inv32, bs, w1, w2, w3, w4, &st);
        inner_total += done_k;
        if (inner_counts) inner_counts[outer] = done_k;
        if (st == ORC_NOT_SPD || st == ORC_BREAKDOWN) { rc = st; break; }
        for (int64_t i = 0; i < n; ++i) x[i] = x[i] + rnorm * (double)d[i];
        ++outer;
    }
done:
    if (out) {
        out[0] = (double)inner_total;
        out[1] = outer;
        out[2] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
    }
    free(v32); free(inv32); free(rt); free(d); free(w1); free(w2); free(w3); free(w4); free(r);
    return rc;
}

/* ======================================================================
 * Batched CG: independent systems, each solved by orc_cg (x0 = 0, no
 * preconditioner).  Systems are stored as concatenated local CSR:
 * system i has rows [row_off[i], row_off[i+1]), local row offsets at
 * rp_local[row_off[i] + i ...], entries [nnz_off[i], nnz_off[i+1]).
 * iters[i], relres[i] (true) are written; returns the worst status.
 * ====================================================================== */
int orc_batch_cg(int64_t nsys, const int64_t *row_off, const int64_t *nnz_off,
                 const int32_t *rp_local, const int32_t *ci, const double *v,
                 const double *b, double *x, double tol, int32_t maxit,
                 int32_t *iters, double *relres) {
    int worst = ORC_OK;
    for (int64_t s = 0; s < nsys; ++s) {
        int64_t m = row_off[s + 1] - row_off[s];
        const int32_t *rp = rp_local + row_off[s] + s;
        double out[4];
        for (int64_t i = 0; i < m; ++i) x[row_off[s] + i] = 0.0;
        int rc = orc_cg(m, rp, ci + nnz_off[s], v + nnz_off[s], b + row_off[s], x + row_off[s],
                        tol, maxit, NULL, 0, out);
        iters[s] = (int32_t)out[0];
        relres[s] = out[2];
        if (rc != ORC_OK && worst == ORC_OK) worst = rc;
    }
    return worst;
}

/* ======================================================================
 * Batched mixed-precision solve: each system by orc_ir_cg (no
 * preconditioner), the FP32 inner solves on the system's values rounded to
 * FP32 and the FP64 residual on the values as given.  For a batch stored in
 * FP32 the values passed here are those FP32 values, so the outer residual
 * refines towards the solution of the FP32-stored matrix.
 * iters[i] = total inner iterations, relres[i] = final true relres.
 * ====================================================================== */
int orc_batch_ir_cg(int64_t nsys, const int64_t *row_off, const int64_t *nnz_off,
                    const int32_t *rp_local, const int32_t *ci, const double *v,
                    const double *b, double *x, double tol, int32_t max_inner,
                    int32_t *iters, double *relres) {
    int worst = ORC_OK;
    for (int64_t s = 0; s < nsys; ++s) {
        int64_t m = row_off[s + 1] - row_off[s];
        const int32_t *rp = rp_local + row_off[s] + s;
        double out[3];
        for (int64_t i = 0; i < m; ++i) x[row_off[s] + i] = 0.0;
        int rc = orc_ir_cg(m, rp, ci + nnz_off[s], v + nnz_off[s], b + row_off[s], x + row_off[s],
                           tol, 20, 1e-5, max_inner, 20 * max_inner, NULL, 0, out, NULL);
        iters[s] = (int32_t)out[0];
        relres[s] = out[2];
        if (rc != ORC_OK && worst == ORC_OK) worst = rc;
    }
    return worst;
}
