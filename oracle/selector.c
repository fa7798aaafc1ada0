/*
 * ORACLE -- test infrastructure, not part of the product.
 *
 * Serial FP64 reference of the learned format selector's arithmetic: the 32
 * structural features of a CSR matrix and the MLP 32 -> 64 -> 64 -> 6
 * (ReLU, ReLU, linear) with its masked mean-squared loss, the backward pass
 * and Adam (Kingma and Ba, ICLR 2015).  The paper has no selector; the
 * definitions are this library's (listed with the features below).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_hyb_width(int64_t n, const int32_t *rp, int32_t value_bytes);
int64_t orc_hyb_tail_nnz(int64_t n, const int32_t *rp, int32_t K);

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int has_entry(const int32_t *rp, const int32_t *ci, int64_t row, int32_t c) {
    int64_t lo = rp[row], hi = rp[row + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (ci[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo < rp[row + 1] && ci[lo] == c;
}

/* The 32 features, in order:
 *  0 log10 n            1 log10 max(nnz,1)     2 mean row length     3 std of lengths
 *  4 cv = std/mean      5 min length           6 max length          7 p50 length
 *  8 p90 length         9 p99 length          10 max/mean           11 frac empty rows
 * 12 frac rows len<=4  13 ELL pad n*max/nnz   14 Kh / mean (Kh = HYB width) 15 HYB tail / nnz
 * 16 Gini of lengths   17 entropy of the length distribution (natural log)
 * 18 frac of nnz in the top ceil(n/100) longest rows
 * 19 log10 CSR working set 12 nnz + 4(n+1) + 8 m + 8 n
 * 20 SELL-P padding: slots of 64-row slices (64 x the slice's longest row,
 *    summed over slices) / nnz
 * 21 m / n             22 mean |i-j| / m      23 max |i-j| / m     24 frac i == j
 * 25 frac |i-j| <= 1   26 frac |i-j| <= 64
 * 27 log10(1 + mean gap between consecutive columns of a row)
 * 28 frac of consecutive-column pairs with gap 1
 * 29 distinct 64-byte x segments (column / 8) per entry, summed over rows / nnz
 * 30 frac of entries (i,j) whose transpose (j,i) is stored (square matrices, else 0)
 * 31 log10(1 + mean column span max-min+1 over nonempty rows)
 * Percentile p: the smallest length L with #rows(len <= L) >= ceil(p n). */
void orc_features(int64_t n, int64_t m, const int32_t *rp, const int32_t *ci, double *f) {
    int64_t nnz = rp[n];
    int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    int64_t minl = n > 0 ? INT64_MAX : 0, maxl = 0, empty = 0, le4 = 0;
    double mean = n > 0 ? (double)nnz / (double)n : 0.0, var = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        len[i] = rp[i + 1] - rp[i];
        if (len[i] < minl) minl = len[i];
        if (len[i] > maxl) maxl = len[i];
        if (len[i] == 0) ++empty;
        if (len[i] <= 4) ++le4;
    }
    for (int64_t i = 0; i < n; ++i) var += ((double)len[i] - mean) * ((double)len[i] - mean);
    double sd = n > 0 ? sqrt(var / (double)n) : 0.0;
    qsort(len, (size_t)n, sizeof(int64_t), cmp_i64);
    /* ceil(p n) for p = 0.5, 0.9, 0.99 */
    int64_t q50 = (n * 50 + 99) / 100, q90 = (n * 90 + 99) / 100, q99 = (n * 99 + 99) / 100;
    double p50 = n ? (double)len[q50 > 0 ? q50 - 1 : 0] : 0;
    double p90 = n ? (double)len[q90 > 0 ? q90 - 1 : 0] : 0;
    double p99 = n ? (double)len[q99 > 0 ? q99 - 1 : 0] : 0;
    /* Gini: 2 sum_k k x_(k) / (n sum x) - (n+1)/n, ranks k = 1..n ascending */
    __int128 wsum = 0;
    for (int64_t k = 0; k < n; ++k) wsum += (__int128)(k + 1) * len[k];
    double gini = (n > 0 && nnz > 0) ? 2.0 * (double)wsum / ((double)n * (double)nnz) -
                                           (double)(n + 1) / (double)n : 0.0;
    double ent = 0.0;
    for (int64_t k = 0; k < n;) {
        int64_t j = k;
        while (j < n && len[j] == len[k]) ++j;
        double p = (double)(j - k) / (double)n;
        ent -= p * log(p);
        k = j;
    }
    int64_t top = (n + 99) / 100, topnnz = 0;
    for (int64_t k = 0; k < top && k < n; ++k) topnnz += len[n - 1 - k];
    int32_t K = orc_hyb_width(n, rp, 8);
    int64_t tail = orc_hyb_tail_nnz(n, rp, K);
    free(len);

    int64_t sabs = 0, mabs = 0, diag = 0, b1 = 0, b64 = 0, gaps = 0, pairs = 0, gap1 = 0;
    int64_t lines = 0, sym = 0, span = 0, nonempty = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = rp[i], e = rp[i + 1];
        if (e > b) {
            ++nonempty;
            span += (int64_t)ci[e - 1] - ci[b] + 1;
        }
        for (int64_t k = b; k < e; ++k) {
            int64_t d = (int64_t)ci[k] - i;
            if (d < 0) d = -d;
            sabs += d;
            if (d > mabs) mabs = d;
            if (d == 0) ++diag;
            if (d <= 1) ++b1;
            if (d <= 64) ++b64;
            if (k > b) {
                int64_t gp = (int64_t)ci[k] - ci[k - 1];
                gaps += gp;
                ++pairs;
                if (gp == 1) ++gap1;
            }
            if (k == b || ci[k] / 8 != ci[k - 1] / 8) ++lines;
            if (n == m && ci[k] < n && has_entry(rp, ci, ci[k], (int32_t)i)) ++sym;
        }
    }
    double dn = (double)n, dnz = nnz > 0 ? (double)nnz : 1.0, dm = m > 0 ? (double)m : 1.0;
    double ws = 12.0 * (double)nnz + 4.0 * (double)(n + 1) + 8.0 * (double)m + 8.0 * dn;
    int64_t sellp = 0;
    for (int64_t s0 = 0; s0 < n; s0 += 64) {
        int64_t w = 0;
        for (int64_t i = s0; i < s0 + 64 && i < n; ++i)
            if (rp[i + 1] - rp[i] > w) w = rp[i + 1] - rp[i];
        sellp += 64 * w;
    }
    f[0] = n > 0 ? log10(dn) : 0.0;
    f[1] = log10(nnz > 0 ? (double)nnz : 1.0);
    f[2] = mean;
    f[3] = sd;
    f[4] = mean > 0 ? sd / mean : 0.0;
    f[5] = (double)minl;
    f[6] = (double)maxl;
    f[7] = p50;
    f[8] = p90;
    f[9] = p99;
    f[10] = mean > 0 ? (double)maxl / mean : 0.0;
    f[11] = n > 0 ? (double)empty / dn : 0.0;
    f[12] = n > 0 ? (double)le4 / dn : 0.0;
    f[13] = nnz > 0 ? dn * (double)maxl / (double)nnz : 1.0;
    f[14] = mean > 0 ? (double)K / mean : 0.0;
    f[15] = (double)tail / dnz;
    f[16] = gini;
    f[17] = ent;
    f[18] = (double)topnnz / dnz;
    f[19] = log10(ws);
    f[20] = nnz > 0 ? (double)sellp / (double)nnz : 1.0;
    f[21] = n > 0 ? (double)m / dn : 0.0;
    f[22] = (double)sabs / dnz / dm;
    f[23] = (double)mabs / dm;
    f[24] = (double)diag / dnz;
    f[25] = (double)b1 / dnz;
    f[26] = (double)b64 / dnz;
    f[27] = log10(1.0 + (pairs > 0 ? (double)gaps / (double)pairs : 0.0));
    f[28] = pairs > 0 ? (double)gap1 / (double)pairs : 0.0;
    f[29] = (double)lines / dnz;
    f[30] = (n == m) ? (double)sym / dnz : 0.0;
    f[31] = log10(1.0 + (nonempty > 0 ? (double)span / (double)nonempty : 0.0));
}

/* ======================================================================
 * MLP 32 -> 64 -> 64 -> 6 (one output per SpMV format: CSR, CSR merge, COO,
 * ELL, HYB, SELL-P).  Parameters (6662), in order: W1[64][32], b1[64],
 * W2[64][64], b2[64], W3[6][64], b3[6] (row-major, out x in).
 *   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), o = W3 h2 + b3
 * Loss over a batch: L = sum_{s,f} mask[s][f] (o[s][f] - y[s][f])^2 / sum mask.
 * relu'(0) = 0.
 * ====================================================================== */
#define NI 32
#define NH 64
#define NO 6
#define NPARAM (NH * NI + NH + NH * NH + NH + NO * NH + NO)

static void mlp_forward1(const double *P, const double *x, double *h1, double *h2, double *o) {
    const double *W1 = P, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH;
    const double *W3 = b2 + NH, *b3 = W3 + NO * NH;
    for (int j = 0; j < NH; ++j) {
        double s = b1[j];
        for (int k = 0; k < NI; ++k) s = s + W1[j * NI + k] * x[k];
        h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < NH; ++j) {
        double s = b2[j];
        for (int k = 0; k < NH; ++k) s = s + W2[j * NH + k] * h1[k];
        h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int j = 0; j < NO; ++j) {
        double s = b3[j];
        for (int k = 0; k < NH; ++k) s = s + W3[j * NH + k] * h2[k];
        o[j] = s;
    }
}

void orc_mlp_forward(int64_t ns, const double *P, const double *X, double *O) {
    double h1[NH], h2[NH];
    for (int64_t s = 0; s < ns; ++s) mlp_forward1(P, X + s * NI, h1, h2, O + s * NO);
}

/* Loss and its gradient (NPARAM values) over the batch. */
double orc_mlp_loss_grad(int64_t ns, const double *P, const double *X, const double *Y,
                         const double *M, double *G) {
    const double *W2 = P + NH * NI + NH, *W3 = W2 + NH * NH + NH;
    double *gW1 = G, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH;
    double *gW3 = gb2 + NH, *gb3 = gW3 + NO * NH;
    for (int i = 0; i < NPARAM; ++i) G[i] = 0.0;
    double msum = 0.0, loss = 0.0;
    for (int64_t s = 0; s < ns * NO; ++s) msum = msum + M[s];
    if (msum == 0.0) return 0.0;
    double h1[NH], h2[NH], o[NO], dO[NO], dh2[NH], dh1[NH];
    for (int64_t s = 0; s < ns; ++s) {
        const double *x = X + s * NI;
        mlp_forward1(P, x, h1, h2, o);
        for (int j = 0; j < NO; ++j) {
            double d = o[j] - Y[s * NO + j];
            loss = loss + M[s * NO + j] * d * d;
            dO[j] = 2.0 * M[s * NO + j] * d / msum;
        }
        for (int j = 0; j < NO; ++j) {
            gb3[j] = gb3[j] + dO[j];
            for (int k = 0; k < NH; ++k) gW3[j * NH + k] = gW3[j * NH + k] + dO[j] * h2[k];
        }
        for (int k = 0; k < NH; ++k) {
            double s2 = 0.0;
            for (int j = 0; j < NO; ++j) s2 = s2 + W3[j * NH + k] * dO[j];
            dh2[k] = h2[k] > 0.0 ? s2 : 0.0;
        }
        for (int j = 0; j < NH; ++j) {
            gb2[j] = gb2[j] + dh2[j];
            for (int k = 0; k < NH; ++k) gW2[j * NH + k] = gW2[j * NH + k] + dh2[j] * h1[k];
        }
        for (int k = 0; k < NH; ++k) {
            double s1 = 0.0;
            for (int j = 0; j < NH; ++j) s1 = s1 + W2[j * NH + k] * dh2[j];
            dh1[k] = h1[k] > 0.0 ? s1 : 0.0;
        }
        for (int j = 0; j < NH; ++j) {
            gb1[j] = gb1[j] + dh1[j];
            for (int k = 0; k < NI; ++k) gW1[j * NI + k] = gW1[j * NI + k] + dh1[j] * x[k];
        }
    }
    return loss / msum;
}

/* t-th Adam step (t >= 1) on the parameters with gradient G. */
void orc_adam_step(int64_t np, double *P, const double *G, double *Mm, double *V, int64_t t,
                   double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        Mm[i] = b1 * Mm[i] + (1.0 - b1) * G[i];
        V[i] = b2 * V[i] + (1.0 - b2) * G[i] * G[i];
        double mh = Mm[i] / c1, vh = V[i] / c2;
        P[i] = P[i] - lr * mh / (sqrt(vh) + eps);
    }
}
