/* Drives every oracle routine on small inputs, for a build of the oracle with
 * the address and undefined-behaviour sanitizers (host only).  Inputs: the
 * 2D 5-point Laplacian on a 9 x 7 grid, the same with a convection term
 * (nonsymmetric), and a pattern with empty rows and one long row for the
 * conversions.  Exits nonzero on a failed check; the sanitizers abort on any
 * out-of-bounds access, use of freed memory or undefined arithmetic. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_csr_spmv(int64_t, const int32_t *, const int32_t *, const double *, const double *,
                  double, double, double *);
void orc_csr_to_coo(int64_t, const int32_t *, const int32_t *, const double *, int32_t *,
                    int32_t *, double *);
int32_t orc_max_row_len(int64_t, const int32_t *);
void orc_csr_to_ell(int64_t, const int32_t *, const int32_t *, const double *, int32_t, int64_t,
                    int32_t *, double *);
int32_t orc_hyb_width(int64_t, const int32_t *, int32_t);
int64_t orc_hyb_tail_nnz(int64_t, const int32_t *, int32_t);
void orc_csr_to_hyb(int64_t, const int32_t *, const int32_t *, const double *, int32_t, int64_t,
                    int32_t *, double *, int32_t *, int32_t *, double *);
void orc_coo_to_csr(int64_t, int64_t, const int32_t *, const int32_t *, const double *, int32_t *,
                    int32_t *, double *);
void orc_hyb_to_csr(int64_t, int32_t, int64_t, const int32_t *, const double *, int64_t,
                    const int32_t *, const int32_t *, const double *, int32_t *, int32_t *,
                    double *);
int64_t orc_sellp_layout(int64_t, const int32_t *, int32_t, int32_t *, int64_t *);
void orc_csr_to_sellp(int64_t, const int32_t *, const int32_t *, const double *, int32_t,
                      const int32_t *, const int64_t *, int32_t *, double *);
void orc_sellp_to_csr(int64_t, int32_t, const int32_t *, const int64_t *, const int32_t *,
                      const double *, int32_t *, int32_t *, double *);
int orc_bj_invert(int64_t, const int32_t *, const int32_t *, const double *, int32_t, double *);
void orc_bj_apply(int64_t, int32_t, const double *, const double *, double *);
int orc_cg(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
           double, int32_t, const double *, int32_t, double *);
int orc_bicgstab(int64_t, const int32_t *, const int32_t *, const double *, const double *,
                 double *, double, int32_t, double *);
int orc_pipecg(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
               double, int32_t, const double *, int32_t, double *);
int orc_fcg(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
            double, int32_t, const double *, int32_t, double *);
int orc_cgs(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
            double, int32_t, double *);
int orc_gmres(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
              double, int32_t, int32_t, double *);
int orc_ir_cg(int64_t, const int32_t *, const int32_t *, const double *, const double *, double *,
              double, int32_t, double, int32_t, int32_t, const double *, int32_t, double *,
              int32_t *);
int32_t orc_pcg_f32(int64_t, const int32_t *, const int32_t *, const float *, const float *,
                    float *, double, int32_t, const float *, int32_t, int32_t *);
int orc_batch_cg(int64_t, const int64_t *, const int64_t *, const int32_t *, const int32_t *,
                 const double *, const double *, double *, double, int32_t, int32_t *, double *);
int orc_batch_ir_cg(int64_t, const int64_t *, const int64_t *, const int32_t *, const int32_t *,
                    const double *, const double *, double *, double, int32_t, int32_t *,
                    double *);
void orc_features(int64_t, int64_t, const int32_t *, const int32_t *, double *);
void orc_mlp_forward(int64_t, const double *, const double *, double *);
double orc_mlp_loss_grad(int64_t, const double *, const double *, const double *, const double *,
                         double *);
void orc_adam_step(int64_t, double *, const double *, double *, double *, int64_t, double, double,
                   double, double);

#define NX 9
#define NY 7
#define N (NX * NY)
#define N_PARAMS 6662
#define N_CLASSES 6
#define N_FEATURES 32

static int failures = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++failures;                                            \
        }                                                          \
    } while (0)

/* 5-point operator on the NX x NY grid: diagonal 4 (+ shift), west/east
 * -1 -/+ c, south/north -1. */
static int64_t grid(double c, int32_t *rp, int32_t *ci, double *v) {
    int64_t k = 0;
    for (int i = 0; i < N; ++i) {
        const int x = i % NX, y = i / NX;
        rp[i] = (int32_t)k;
        if (y > 0) { ci[k] = i - NX; v[k++] = -1.0; }
        if (x > 0) { ci[k] = i - 1; v[k++] = -1.0 - c; }
        ci[k] = i; v[k++] = 4.0;
        if (x < NX - 1) { ci[k] = i + 1; v[k++] = -1.0 + c; }
        if (y < NY - 1) { ci[k] = i + NX; v[k++] = -1.0; }
    }
    rp[N] = (int32_t)k;
    return k;
}

static int same_csr(int64_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    const int32_t *rp2, const int32_t *ci2, const double *v2) {
    if (memcmp(rp, rp2, (size_t)(n + 1) * 4)) return 0;
    return !memcmp(ci, ci2, (size_t)rp[n] * 4) && !memcmp(v, v2, (size_t)rp[n] * 8);
}

static void conversions(void) {
    /* 12 rows: empty rows 0, 5, 11; row 7 holds all 12 columns */
    enum { n = 12 };
    int32_t rp[n + 1], ci[64];
    double v[64];
    int64_t k = 0;
    for (int i = 0; i < n; ++i) {
        rp[i] = (int32_t)k;
        const int len = (i == 0 || i == 5 || i == 11) ? 0 : (i == 7 ? n : 1 + i % 3);
        for (int j = 0; j < len; ++j) {
            ci[k] = len == n ? j : (i + 2 * j) % n;
            v[k++] = 0.5 + i - j;
        }
        /* sort the row's columns (insertion sort; distinct by construction) */
        for (int64_t a = rp[i] + 1; a < k; ++a)
            for (int64_t b = a; b > rp[i] && ci[b - 1] > ci[b]; --b) {
                int32_t tc = ci[b]; ci[b] = ci[b - 1]; ci[b - 1] = tc;
                double tv = v[b]; v[b] = v[b - 1]; v[b - 1] = tv;
            }
    }
    rp[n] = (int32_t)k;
    const int64_t nnz = k;
    int32_t rp2[n + 1], ci2[64], row[64], col[64];
    double v2[64], val[64];

    orc_csr_to_coo(n, rp, ci, v, row, col, val);
    orc_coo_to_csr(n, nnz, row, col, val, rp2, ci2, v2);
    CHECK(same_csr(n, rp, ci, v, rp2, ci2, v2));

    const int32_t K = orc_max_row_len(n, rp);
    CHECK(K == n);
    const int64_t ld = 64;
    int32_t *ecol = malloc(sizeof(int32_t) * (size_t)(K * ld));
    double *eval = malloc(sizeof(double) * (size_t)(K * ld));
    orc_csr_to_ell(n, rp, ci, v, K, ld, ecol, eval);
    orc_hyb_to_csr(n, K, ld, ecol, eval, 0, NULL, NULL, NULL, rp2, ci2, v2);
    CHECK(same_csr(n, rp, ci, v, rp2, ci2, v2));
    free(ecol);
    free(eval);

    const int32_t Kh = orc_hyb_width(n, rp, 8);
    const int64_t tnnz = orc_hyb_tail_nnz(n, rp, Kh);
    int32_t *hcol = malloc(sizeof(int32_t) * (size_t)(Kh * ld + 1));
    double *hval = malloc(sizeof(double) * (size_t)(Kh * ld + 1));
    int32_t *trow = malloc(sizeof(int32_t) * (size_t)(tnnz + 1));
    int32_t *tcol = malloc(sizeof(int32_t) * (size_t)(tnnz + 1));
    double *tval = malloc(sizeof(double) * (size_t)(tnnz + 1));
    orc_csr_to_hyb(n, rp, ci, v, Kh, ld, hcol, hval, trow, tcol, tval);
    orc_hyb_to_csr(n, Kh, ld, hcol, hval, tnnz, trow, tcol, tval, rp2, ci2, v2);
    CHECK(same_csr(n, rp, ci, v, rp2, ci2, v2));
    free(hcol); free(hval); free(trow); free(tcol); free(tval);

    const int32_t C = 4;
    const int64_t ns = (n + C - 1) / C;
    int32_t widths[ns];
    int64_t sets[ns + 1];
    const int64_t slots = orc_sellp_layout(n, rp, C, widths, sets);
    CHECK(slots == sets[ns]);
    int32_t *scol = malloc(sizeof(int32_t) * (size_t)(slots + 1));
    double *sval = malloc(sizeof(double) * (size_t)(slots + 1));
    orc_csr_to_sellp(n, rp, ci, v, C, widths, sets, scol, sval);
    orc_sellp_to_csr(n, C, widths, sets, scol, sval, rp2, ci2, v2);
    CHECK(same_csr(n, rp, ci, v, rp2, ci2, v2));
    free(scol);
    free(sval);

    double x[n], y[n], f[N_FEATURES];
    for (int i = 0; i < n; ++i) x[i] = 1.0 - 0.1 * i;
    orc_csr_spmv(n, rp, ci, v, x, 1.0, 0.0, y);
    CHECK(y[0] == 0.0 && y[5] == 0.0 && y[11] == 0.0);
    orc_features(n, n, rp, ci, f);
    for (int j = 0; j < N_FEATURES; ++j) CHECK(isfinite(f[j]));
}

static void solvers(void) {
    int32_t rp[N + 1], ci[5 * N];
    double v[5 * N], b[N], x[N], out[4], xs[N];
    grid(0.0, rp, ci, v);
    for (int i = 0; i < N; ++i) xs[i] = sin(0.7 * i + 0.3);
    orc_csr_spmv(N, rp, ci, v, xs, 1.0, 0.0, b);

    double inv[((N + 7) / 8) * 64];
    CHECK(orc_bj_invert(N, rp, ci, v, 8, inv) == 0);
    double z[N];
    orc_bj_apply(N, 8, inv, b, z);

    memset(x, 0, sizeof x);
    CHECK(orc_cg(N, rp, ci, v, b, x, 1e-10, 500, NULL, 0, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_cg(N, rp, ci, v, b, x, 1e-10, 500, inv, 8, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_pipecg(N, rp, ci, v, b, x, 1e-10, 500, inv, 8, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_fcg(N, rp, ci, v, b, x, 1e-10, 500, inv, 8, out) == 0);
    memset(x, 0, sizeof x);
    {
        int32_t counts[20];
        float d32[N], b32[N], v32[5 * N];
        int32_t st;
        /* a budget of 3 inner iterations in total runs out before 1e-10 */
        CHECK(orc_ir_cg(N, rp, ci, v, b, x, 1e-10, 20, 1e-5, 1000, 3, inv, 8, out, counts) == 6);
        CHECK(out[0] <= 3);
        for (int i = 0; i < N; ++i) b32[i] = (float)b[i];
        for (int k = 0; k < rp[N]; ++k) v32[k] = (float)v[k];
        CHECK(orc_pcg_f32(N, rp, ci, v32, b32, d32, 1e-5, 500, NULL, 8, &st) > 0 && st == 0);
        memset(x, 0, sizeof x);
        CHECK(orc_ir_cg(N, rp, ci, v, b, x, 1e-10, 20, 1e-5, 1000, 20000, inv, 8, out, counts) == 0);
    }
    for (int i = 0; i < N; ++i) CHECK(fabs(x[i] - xs[i]) < 1e-6);

    /* nonsymmetric */
    grid(0.5, rp, ci, v);
    orc_csr_spmv(N, rp, ci, v, xs, 1.0, 0.0, b);
    memset(x, 0, sizeof x);
    CHECK(orc_bicgstab(N, rp, ci, v, b, x, 1e-10, 500, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_cgs(N, rp, ci, v, b, x, 1e-10, 500, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_gmres(N, rp, ci, v, b, x, 1e-10, 500, 10, out) == 0);
    memset(x, 0, sizeof x);
    CHECK(orc_gmres(N, rp, ci, v, b, x, 1e-10, 500, N + 5, out) == 0); /* m above n */
}

static void batch(void) {
    /* two systems: the Laplacian and a 1-row system */
    int32_t rp[N + 1], ci[5 * N];
    double v[5 * N];
    const int64_t nnz0 = grid(0.0, rp, ci, v);
    int64_t row_off[3] = {0, N, N + 1}, nnz_off[3] = {0, nnz0, nnz0 + 1};
    int32_t rpl[N + 3], cil[5 * N + 1];
    double vl[5 * N + 1], b[N + 1], x[N + 1], relres[2];
    int32_t iters[2];
    memcpy(rpl, rp, sizeof(int32_t) * (N + 1));
    rpl[N + 1] = 0;
    rpl[N + 2] = 1;
    memcpy(cil, ci, sizeof(int32_t) * (size_t)nnz0);
    memcpy(vl, v, sizeof(double) * (size_t)nnz0);
    cil[nnz0] = 0;
    vl[nnz0] = 2.0;
    for (int i = 0; i <= N; ++i) b[i] = 1.0 + 0.01 * i;
    CHECK(orc_batch_cg(2, row_off, nnz_off, rpl, cil, vl, b, x, 1e-10, 500, iters, relres) == 0);
    CHECK(fabs(x[N] - b[N] / 2.0) < 1e-12);
    CHECK(orc_batch_ir_cg(2, row_off, nnz_off, rpl, cil, vl, b, x, 1e-10, 500, iters, relres) == 0);
}

static void mlp(void) {
    enum { ns = 5 };
    double *P = malloc(sizeof(double) * N_PARAMS), *G = malloc(sizeof(double) * N_PARAMS);
    double *M = calloc(N_PARAMS, sizeof(double)), *V = calloc(N_PARAMS, sizeof(double));
    double X[ns * N_FEATURES], Y[ns * N_CLASSES], Mask[ns * N_CLASSES], O[ns * N_CLASSES];
    for (int i = 0; i < N_PARAMS; ++i) P[i] = 0.05 * sin(1.3 * i);
    for (int i = 0; i < ns * N_FEATURES; ++i) X[i] = cos(0.37 * i);
    for (int i = 0; i < ns * N_CLASSES; ++i) {
        Y[i] = 0.1 * (i % 4);
        Mask[i] = (i % 5) ? 1.0 : 0.0;
    }
    orc_mlp_forward(ns, P, X, O);
    const double loss = orc_mlp_loss_grad(ns, P, X, Y, Mask, G);
    CHECK(isfinite(loss));
    orc_adam_step(N_PARAMS, P, G, M, V, 1, 1e-3, 0.9, 0.999, 1e-8);
    free(P); free(G); free(M); free(V);
}

int main(void) {
    conversions();
    solvers();
    batch();
    mlp();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitize run ok\n");
    return 0;
}
