/*
 * Seeded synthetic input generators.
 *
 * This file holds no arithmetic of the method: it only draws random numbers
 * and lays out sparsity patterns and values in CSR (int32 row offsets, int32
 * column indices sorted ascending within a row, double values).  Both the
 * CPU oracle and the GPU library are fed from the arrays produced here.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), with the output mix
 * constants of its published reference implementation.  A stream is named by
 * (seed, k): its initial state is seed * 8 + k, k in [0, 8).
 *   uniform u in [0,1)   = (next() >> 11) * 2^-53
 *   U[lo,hi]             = lo + (hi - lo) * u
 *   integer in [0, m)    = high 64 bits of next() * m (multiply-shift)
 *   standard normal      = Box-Muller, sqrt(-2 ln(1-u1)) * cos(2 pi u2)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } sm64;

static void sm_init(sm64 *g, uint64_t seed, unsigned k) { g->s = seed * 8u + (uint64_t)k; }

static uint64_t sm_next(sm64 *g) {
    uint64_t z = (g->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double sm_u01(sm64 *g) { return (double)(sm_next(g) >> 11) * (1.0 / 9007199254740992.0); }

static uint64_t sm_below(sm64 *g, uint64_t m) {
    return (uint64_t)(((unsigned __int128)sm_next(g) * (unsigned __int128)m) >> 64);
}

static double sm_normal(sm64 *g) {
    double u1 = sm_u01(g), u2 = sm_u01(g);
    return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586 * u2);
}

uint64_t gen_splitmix64_first(uint64_t seed, unsigned k) {
    sm64 g; sm_init(&g, seed, k); return sm_next(&g);
}

/* out[i] = U[lo,hi] from stream (seed, 0). */
void gen_uniform(uint64_t seed, int64_t n, double lo, double hi, double *out) {
    sm64 g; sm_init(&g, seed, 0);
    for (int64_t i = 0; i < n; ++i) out[i] = lo + (hi - lo) * sm_u01(&g);
}

/* ------------------------------------------------------------------------
 * Structured grids.  Node (ix,iy,iz) has index ix + nx*(iy + ny*iz).
 * kind 0 = star (the 2d+1 point Laplacian: +-1 along each axis),
 * kind 1 = box  (all 3^d - 1 neighbours).  d counts the axes of extent > 1.
 * Diagonal = number of neighbours of an interior node, off-diagonals = -1,
 * neighbours outside the grid are dropped (Dirichlet boundary).
 * ------------------------------------------------------------------------ */
static int grid_dims(int64_t nx, int64_t ny, int64_t nz) {
    return (nx > 1) + (ny > 1) + (nz > 1);
}

static int offset_used(int kind, int dx, int dy, int dz, int64_t nx, int64_t ny, int64_t nz) {
    if (dx == 0 && dy == 0 && dz == 0) return 1;
    if ((dx && nx == 1) || (dy && ny == 1) || (dz && nz == 1)) return 0;
    if (kind == 0) return (dx != 0) + (dy != 0) + (dz != 0) == 1;
    return 1;
}

int64_t gen_grid_nnz(int64_t nx, int64_t ny, int64_t nz, int kind) {
    int64_t nnz = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                if (!offset_used(kind, dx, dy, dz, nx, ny, nz)) continue;
                nnz += (nx - (dx != 0)) * (ny - (dy != 0)) * (nz - (dz != 0));
            }
    return nnz;
}

void gen_grid_fill(int64_t nx, int64_t ny, int64_t nz, int kind,
                   int32_t *row_ptr, int32_t *col, double *val) {
    int d = grid_dims(nx, ny, nz);
    double diag = (kind == 0) ? 2.0 * d : (d == 1 ? 2.0 : d == 2 ? 8.0 : 26.0);
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t iz = 0; iz < nz; ++iz)
        for (int64_t iy = 0; iy < ny; ++iy)
            for (int64_t ix = 0; ix < nx; ++ix) {
                int64_t row = ix + nx * (iy + ny * iz);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            if (!offset_used(kind, dx, dy, dz, nx, ny, nz)) continue;
                            int64_t jx = ix + dx, jy = iy + dy, jz = iz + dz;
                            if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
                            col[k] = (int32_t)(jx + nx * (jy + ny * jz));
                            val[k] = (dx == 0 && dy == 0 && dz == 0) ? diag : -1.0;
                            ++k;
                        }
                row_ptr[row + 1] = (int32_t)k;
            }
}

/* 2D convection-diffusion on an N x N grid (nonsymmetric): diagonal 4,
 * west -1-c, east -1+c, south and north -1. */
void gen_convdiff2d_fill(int64_t N, double c, int32_t *row_ptr, int32_t *col, double *val) {
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t iy = 0; iy < N; ++iy)
        for (int64_t ix = 0; ix < N; ++ix) {
            int64_t i = ix + N * iy;
            if (iy > 0)     { col[k] = (int32_t)(i - N); val[k++] = -1.0; }
            if (ix > 0)     { col[k] = (int32_t)(i - 1); val[k++] = -1.0 - c; }
            col[k] = (int32_t)i; val[k++] = 4.0;
            if (ix < N - 1) { col[k] = (int32_t)(i + 1); val[k++] = -1.0 + c; }
            if (iy < N - 1) { col[k] = (int32_t)(i + N); val[k++] = -1.0; }
            row_ptr[i + 1] = (int32_t)k;
        }
}

/* ------------------------------------------------------------------------
 * Random matrices with given row lengths and distinct uniform columns.
 * ------------------------------------------------------------------------ */

/* Lognormal row lengths from stream (seed, 1):
 * len_i = clamp(round(exp(mu + sigma z)), min_len, max_len); afterwards the
 * first longest row is set to exactly max_len (if force_max != 0).
 * Returns the sum of lengths. */
int64_t gen_lognormal_lengths(uint64_t seed, int64_t n, double mu, double sigma,
                              int32_t min_len, int32_t max_len, int force_max, int32_t *len) {
    sm64 g; sm_init(&g, seed, 1);
    int64_t best = 0, total = 0;
    for (int64_t i = 0; i < n; ++i) {
        double l = nearbyint(exp(mu + sigma * sm_normal(&g)));
        if (!(l >= (double)min_len)) l = (double)min_len;
        if (l > (double)max_len) l = (double)max_len;
        len[i] = (int32_t)l;
        if (len[i] > len[best]) best = i;
    }
    if (force_max && n > 0) len[best] = max_len;
    for (int64_t i = 0; i < n; ++i) total += len[i];
    return total;
}

/* Uniform row lengths in [lo, hi] from stream (seed, 1). Returns the sum. */
int64_t gen_uniform_lengths(uint64_t seed, int64_t n, int32_t lo, int32_t hi, int32_t *len) {
    sm64 g; sm_init(&g, seed, 1);
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) {
        len[i] = lo + (int32_t)sm_below(&g, (uint64_t)(hi - lo + 1));
        total += len[i];
    }
    return total;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Row i gets len[i] distinct columns drawn uniformly from [0, n_cols) by
 * Floyd's sampling (stream (seed, 2)), sorted ascending; values U[-1,1]
 * from stream (seed, 3).  Requires len[i] <= n_cols.  Returns 0 on success. */
int gen_random_rows_fill(uint64_t seed, int64_t n, int64_t n_cols, const int32_t *len,
                         int32_t *row_ptr, int32_t *col, double *val) {
    sm64 gc, gv;
    sm_init(&gc, seed, 2);
    sm_init(&gv, seed, 3);
    unsigned char *mark = (unsigned char *)calloc((size_t)n_cols, 1);
    if (!mark) return 1;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t L = len[i];
        if (L > n_cols) { free(mark); return 2; }
        int32_t *c = col + k;
        for (int64_t j = n_cols - L, t = 0; j < n_cols; ++j, ++t) {
            int64_t r = (int64_t)sm_below(&gc, (uint64_t)(j + 1));
            if (mark[r]) r = j;
            mark[r] = 1;
            c[t] = (int32_t)r;
        }
        for (int64_t t = 0; t < L; ++t) mark[c[t]] = 0;
        qsort(c, (size_t)L, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < L; ++t) val[k + t] = -1.0 + 2.0 * sm_u01(&gv);
        k += L;
        row_ptr[i + 1] = (int32_t)k;
    }
    free(mark);
    return 0;
}

/* Banded random pattern: row i draws len[i] distinct columns from the
 * window [i - bw, i + bw] clipped to [0, n), always including i.  Columns
 * via Floyd's sampling on the window (stream (seed, 2)), values U[-1,1]
 * (stream (seed, 3)).  len[i] is clipped to the window size by the caller. */
int gen_banded_rows_fill(uint64_t seed, int64_t n, int64_t bw, const int32_t *len,
                         int32_t *row_ptr, int32_t *col, double *val) {
    sm64 gc, gv;
    sm_init(&gc, seed, 2);
    sm_init(&gv, seed, 3);
    unsigned char *mark = (unsigned char *)calloc((size_t)(2 * bw + 1), 1);
    if (!mark) return 1;
    int64_t k = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = i - bw < 0 ? 0 : i - bw;
        int64_t hi = i + bw >= n ? n - 1 : i + bw;
        int64_t W = hi - lo + 1;
        int64_t L = len[i];
        if (L > W || L < 1) { free(mark); return 2; }
        int32_t *c = col + k;
        /* the diagonal is always present; the other L-1 come from the W-1 others */
        int64_t dpos = i - lo;
        mark[dpos] = 1;
        c[0] = (int32_t)i;
        for (int64_t j = (W - 1) - (L - 1), t = 1; j < W - 1; ++j, ++t) {
            int64_t r = (int64_t)sm_below(&gc, (uint64_t)(j + 1));
            int64_t rr = r >= dpos ? r + 1 : r;   /* skip the diagonal slot */
            int64_t jj = j >= dpos ? j + 1 : j;
            if (mark[rr]) rr = jj;
            mark[rr] = 1;
            c[t] = (int32_t)(lo + rr);
        }
        for (int64_t t = 0; t < L; ++t) mark[c[t] - lo] = 0;
        qsort(c, (size_t)L, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < L; ++t) val[k + t] = -1.0 + 2.0 * sm_u01(&gv);
        k += L;
        row_ptr[i + 1] = (int32_t)k;
    }
    free(mark);
    return 0;
}

/* Block diagonal: consecutive dense blocks with sizes U{bmin..bmax} (stream
 * (seed, 1)), the last one truncated at n; values U[-1,1] (stream (seed, 3)).
 * Pass 1 (row_ptr == NULL) returns nnz; pass 2 fills. */
int64_t gen_blockdiag(uint64_t seed, int64_t n, int32_t bmin, int32_t bmax,
                      int32_t *row_ptr, int32_t *col, double *val) {
    sm64 gb, gv;
    sm_init(&gb, seed, 1);
    sm_init(&gv, seed, 3);
    int64_t start = 0, k = 0;
    if (row_ptr) row_ptr[0] = 0;
    while (start < n) {
        int64_t b = bmin + (int64_t)sm_below(&gb, (uint64_t)(bmax - bmin + 1));
        if (start + b > n) b = n - start;
        for (int64_t i = start; i < start + b; ++i) {
            if (row_ptr) {
                for (int64_t j = start; j < start + b; ++j) {
                    col[k] = (int32_t)j;
                    val[k] = -1.0 + 2.0 * sm_u01(&gv);
                    ++k;
                }
                row_ptr[i + 1] = (int32_t)k;
            } else {
                k += b;
            }
        }
        start += b;
    }
    return k;
}

/* ------------------------------------------------------------------------
 * Batches of small SPD systems.  System i of master seed S uses stream
 * (S * 2^32 + i, 0):  m = 32 + U{0..m_span-1};  pattern 5-point if u < 1/2
 * else 3-point;  shift s = U[0.1, 2];  then x* ~ U[-1,1] (m draws).
 *   3-point: tridiag(-1, 2+s, -1) of order m.
 *   5-point: grid width w = ceil(sqrt(m)), node j <-> (j mod w, j div w);
 *            j+-1 are neighbours when in the same grid row and in [0, m),
 *            j+-w when in [0, m); diagonal 4+s, neighbours -1.
 * ------------------------------------------------------------------------ */
static void batch_draw(uint64_t master, int64_t i, int32_t m_lo, int32_t m_hi,
                       int32_t *m, int32_t *pat, double *s, sm64 *g) {
    sm_init(g, (master << 32) + (uint64_t)i, 0);
    *m = m_lo + (int32_t)sm_below(g, (uint64_t)(m_hi - m_lo + 1));
    *pat = sm_u01(g) < 0.5 ? 5 : 3;
    *s = 0.1 + 1.9 * sm_u01(g);
}

static int32_t isqrt_ceil(int32_t m) {
    int32_t w = (int32_t)sqrt((double)m);
    while (w * w < m) ++w;
    while (w > 1 && (w - 1) * (w - 1) >= m) --w;
    return w;
}

static int64_t batch_nnz_of(int32_t m, int32_t pat) {
    if (pat == 3) return 3 * (int64_t)m - 2;
    int32_t w = isqrt_ceil(m);
    int64_t nnz = 0;
    for (int32_t j = 0; j < m; ++j) {
        nnz += 1;
        if (j % w > 0) nnz += 1;
        if (j % w < w - 1 && j + 1 < m) nnz += 1;
        if (j - w >= 0) nnz += 1;
        if (j + w < m) nnz += 1;
    }
    return nnz;
}

/* Pass 1: per-system sizes. */
void gen_batch_dims(uint64_t master, int64_t nsys, int32_t m_lo, int32_t m_hi,
                    int32_t *m_out, int64_t *nnz_out, int32_t *pat_out, double *shift_out) {
    for (int64_t i = 0; i < nsys; ++i) {
        sm64 g; int32_t m, pat; double s;
        batch_draw(master, i, m_lo, m_hi, &m, &pat, &s, &g);
        m_out[i] = m; pat_out[i] = pat; shift_out[i] = s;
        nnz_out[i] = batch_nnz_of(m, pat);
    }
}

/* Pass 2: concatenated local CSR (row_ptr_local has m_i + 1 entries per
 * system, stored at row_off[i] + i), values and x*. */
void gen_batch_fill(uint64_t master, int64_t nsys, int32_t m_lo, int32_t m_hi,
                    const int64_t *row_off, const int64_t *nnz_off,
                    int32_t *row_ptr_local, int32_t *col, double *val, double *xstar) {
    for (int64_t i = 0; i < nsys; ++i) {
        sm64 g; int32_t m, pat; double s;
        batch_draw(master, i, m_lo, m_hi, &m, &pat, &s, &g);
        int32_t *rp = row_ptr_local + row_off[i] + i;
        int32_t *c = col + nnz_off[i];
        double *v = val + nnz_off[i];
        int64_t k = 0;
        rp[0] = 0;
        if (pat == 3) {
            for (int32_t j = 0; j < m; ++j) {
                if (j > 0) { c[k] = j - 1; v[k++] = -1.0; }
                c[k] = j; v[k++] = 2.0 + s;
                if (j + 1 < m) { c[k] = j + 1; v[k++] = -1.0; }
                rp[j + 1] = (int32_t)k;
            }
        } else {
            int32_t w = isqrt_ceil(m);
            for (int32_t j = 0; j < m; ++j) {
                if (j - w >= 0) { c[k] = j - w; v[k++] = -1.0; }
                if (j % w > 0) { c[k] = j - 1; v[k++] = -1.0; }
                c[k] = j; v[k++] = 4.0 + s;
                if (j % w < w - 1 && j + 1 < m) { c[k] = j + 1; v[k++] = -1.0; }
                if (j + w < m) { c[k] = j + w; v[k++] = -1.0; }
                rp[j + 1] = (int32_t)k;
            }
        }
        double *xs = xstar + row_off[i];
        for (int32_t j = 0; j < m; ++j) xs[j] = -1.0 + 2.0 * sm_u01(&g);
    }
}
