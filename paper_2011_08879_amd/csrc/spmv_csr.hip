// SpMV for matrices stored in CSR: the row-parallel ("classical") kernel with
// a subwarp per row, and the load-balanced merge-path kernel.
//
// Both compute y <- alpha A x + beta y (Sec. 6.1); rows are independent, so
// the only cross-lane work is the per-row sum.  Memory bound: one streaming
// pass over col/val (s+4 bytes per entry), row_ptr once, x gathered, y once.
#include <climits>

#include "csr_rows.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace gko {

// ====================================================================== classical
// Rows longer than the subwarp threshold: one workgroup per row, four loads
// per thread in flight, a fixed-tree block sum.
constexpr int kLongBlock = 256;

template <typename V>
__device__ inline void csr_long_row(int32_t r, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col, const V *__restrict__ val,
                                    const V *__restrict__ x, V alpha, V beta, V *__restrict__ y,
                                    V *lds) {
    const int32_t b = rp[r], e = rp[r + 1];
    V s = V(0);
    for (int32_t k = b + threadIdx.x; k < e; k += 4 * kLongBlock) {
        int32_t cc[4];
        V vv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t kj = k + j * kLongBlock;
            cc[j] = kj < e ? load_stream(col + kj) : -1;
            vv[j] = kj < e ? load_stream(val + kj) : V(0);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (cc[j] >= 0) s += vv[j] * x[cc[j]];
    }
    s = block_sum<kLongBlock>(s, lds);
    if (threadIdx.x == 0) y[r] = (beta == V(0)) ? alpha * s : alpha * s + beta * y[r];
}

// A subwarp of W lanes owns U consecutive rows: consecutive lanes read
// consecutive entries, so a wave reads the entries of 64/W * U rows as
// contiguous stretches.  The loads of all U rows (offsets, then columns and
// values, then the x gathers) are issued before any is consumed, so each
// wave keeps U times more bytes in flight than a row-at-a-time loop; rows
// longer than W continue in a strided loop.  Each row is then summed by a
// subwarp butterfly.  W is a compile-time width chosen at run time from the
// mean row length, in the spirit of the run-time choice among precompiled
// subgroup widths in Sec. 5.
// Rows longer than long_t are listed in long_rows: the first n_long
// workgroups of the launch take one each (csr_long_row), the rest the
// subwarps, so both kinds of rows share one launch (lognormal rows with
// sigma 1.56: 118 + 88 us as two launches, 204 -> 192 us as one).
template <typename V, int W, int BLOCK>
__global__ __launch_bounds__(BLOCK) void spmv_csr_kernel(int64_t n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ col,
                                                         const V *__restrict__ val,
                                                         const V *__restrict__ x, V alpha, V beta,
                                                         V *__restrict__ y, int32_t long_t,
                                                         int64_t n_long,
                                                         const int32_t *__restrict__ long_rows) {
    static_assert(BLOCK == kLongBlock, "one workgroup shape for both kinds of rows");
    constexpr int U = csr_shape<W>::U;
    constexpr int SPB = BLOCK / W;
    if ((int64_t)blockIdx.x < n_long) {
        __shared__ V lds[kLongBlock / kWave];
        csr_long_row(long_rows[blockIdx.x], rp, col, val, x, alpha, beta, y, lds);
        return;
    }
    const int64_t blk = (int64_t)blockIdx.x - n_long;
    const int lane = threadIdx.x % W;
    const int64_t row0 = (blk * SPB + threadIdx.x / W) * U;
    if (row0 >= n) return;  // uniform across the subwarp
    V s[U];
    csr_rows_sum<V, W, U>(n, row0, lane, rp, col, val, x, s, long_t);
    // lane u stores row u (when the subwarp has fewer lanes than rows, lane 0 stores all)
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t r = row0 + u;
        if ((W >= U ? lane == u : lane == 0) && r < n && rp[r + 1] - rp[r] <= long_t)
            y[r] = (beta == V(0)) ? alpha * s[u] : alpha * s[u] + beta * y[r];
    }
}

// Row-per-thread CSR (csr_rowthread_sum with G lanes per row), chosen for
// short regular rows.
template <typename V, int G>
__global__ __launch_bounds__(kRowThreadBlock) void spmv_csr_rowthread_kernel(
    int64_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y) {
    __shared__ rowthread_lds<V> L;
    // up to kXcdRowsMax rows each XCD takes one contiguous range of rows, so
    // the x lines that neighbouring rows share are fetched into one L2
    const int64_t r0 = row_block_order(n) * (kRowThreadBlock / G);
    const V s = csr_rowthread_sum<V, G>(n, r0, rp, col, val, x, L);
    const int64_t i = r0 + threadIdx.x / G;
    if (i < n && threadIdx.x % G == 0) y[i] = (beta == V(0)) ? alpha * s : alpha * s + beta * y[i];
}

template <typename V, int G>
static hipError_t launch_csr_rowthread_g(hipStream_t s, int64_t n, const int32_t *rp,
                                         const int32_t *col, const void *val, const void *x,
                                         double alpha, double beta, void *y) {
    constexpr int64_t rows = kRowThreadBlock / G;
    spmv_csr_rowthread_kernel<V, G><<<dim3((unsigned)((n + rows - 1) / rows)),
                                      dim3(kRowThreadBlock), 0, s>>>(
        n, rp, col, static_cast<const V *>(val), static_cast<const V *>(x), (V)alpha, (V)beta,
        static_cast<V *>(y));
    return hipGetLastError();
}

template <typename V>
static hipError_t launch_csr_rowthread(hipStream_t s, int64_t n, const int32_t *rp,
                                       const int32_t *col, const void *val, const void *x,
                                       double alpha, double beta, void *y, int lanes) {
    switch (lanes) {
        case 1: return launch_csr_rowthread_g<V, 1>(s, n, rp, col, val, x, alpha, beta, y);
        case 2: return launch_csr_rowthread_g<V, 2>(s, n, rp, col, val, x, alpha, beta, y);
        case 4: return launch_csr_rowthread_g<V, 4>(s, n, rp, col, val, x, alpha, beta, y);
        case 8: return launch_csr_rowthread_g<V, 8>(s, n, rp, col, val, x, alpha, beta, y);
        default: return hipErrorInvalidValue;
    }
}

// The CSR kernel for a matrix, from its mean and longest row (measured on
// MI355X over 2D/3D stencils, banded, block-diagonal, uniform and lognormal
// random patterns, n = 0.5-4M):
//  * rows of at most 96 entries on average and 256 at most: the LDS-staged
//    row-per-thread kernel (csr_row_lanes lanes per row).  With one lane per
//    row against the subwarp kernel: 2D Laplacian 92 -> 34 us, banded mean 32
//    173 -> 107 us, banded mean 48 216 -> 173 us, lognormal rows with sigma
//    0.5 201 -> 180 us; with eight lanes per row (1M rows): banded mean 64
//    242 -> 189 us, block-diagonal mean 74 269 -> 202 us against the
//    quarter-mean subwarp;
//  * longer rows that are regular (longest <= 4 x mean): a subwarp of about
//    mean/4 lanes, four entries per lane (banded mean 64: 156 us with 64
//    lanes, 120 us with 16 lanes; block-diagonal mean 70: 164, 130 us);
//  * otherwise a subwarp of about mean lanes plus the long-row kernel
//    (lognormal rows with sigma 1.56: 223 us; a thread per row 910 us).
int csr_kernel_width(int64_t n, int64_t nnz, int64_t max_len) {
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    if (n > 0 && max_len <= kCsrRowThreadMaxLen && mean <= 96.0) return kCsrRowThread;
    const int w = csr_subwarp_width(n, nnz);
    if ((double)max_len <= 4.0 * mean) return w >= 4 ? w / 4 : 1;
    return w;
}

// Rows longer than this go to the workgroup-per-row kernel (for matrices
// with irregular rows, see csr_has_long_rows).  On the lognormal random
// matrix (mean 16, longest 10,000, 16-lane subwarps): threshold 512 223 us,
// 256 215 us, 128 208 us, 64 206 us.
int32_t csr_long_threshold(int w) { return 4 * w > 64 ? 4 * w : 64; }

// Lanes per row of the row-per-thread kernel, from the mean row length.
// Measured (FP64, us; 1 / 2 / 4 / 8 lanes): 2D Laplacian 2048^2 57 / 81 /
// 118 / 207, 3D Laplacian 160^3 75 / 102 / 134 / 210, lognormal rows of
// sigma 0.5 and mean 16 173 / 170 / 166 / 165, 27-point stencil 128^3 166 /
// 150 / 150 / 205, banded rows of mean 32 211 / 196 / 195 / 206, of mean 48
// 181 / 153 / 148 / 148 (8 lanes: 149 against 147 with 4 in a second run).
int csr_row_lanes(int64_t n, int64_t nnz) {
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    return mean >= 56.0 ? 8 : (mean >= 12.0 ? 4 : 1);
}

bool csr_has_long_rows(int64_t n, int64_t nnz, int64_t max_len, int w) {
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    return w != kCsrRowThread && (double)max_len > 4.0 * mean && max_len > csr_long_threshold(w);
}

__global__ void long_flag_kernel(int64_t n, const int32_t *__restrict__ rp, int32_t long_t,
                                 int32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = rp[i + 1] - rp[i] > long_t;
}

__global__ void long_scatter_kernel(int64_t n, const int32_t *__restrict__ flag,
                                    const int32_t *__restrict__ pos, int32_t *__restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) rows[pos[i]] = (int32_t)i;
}

hipError_t csr_long_flags(hipStream_t s, int64_t n, const int32_t *rp, int32_t long_t, int32_t *flag) {
    if (n == 0) return hipSuccess;
    long_flag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, rp, long_t, flag);
    return hipGetLastError();
}

hipError_t csr_long_scatter(hipStream_t s, int64_t n, const int32_t *flag, const int32_t *pos,
                            int32_t *rows) {
    if (n == 0) return hipSuccess;
    long_scatter_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(n, flag, pos, rows);
    return hipGetLastError();
}

int csr_subwarp_width(int64_t n, int64_t nnz) {
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    int w = 1;
    while (w < 64 && w < mean) w <<= 1;
    return w;
}

template <typename V, int W>
static hipError_t launch_csr_w(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                               const void *val, const void *x, double alpha, double beta, void *y,
                               int32_t long_t, int64_t n_long, const int32_t *long_rows) {
    constexpr int BLOCK = kLongBlock;
    constexpr int RPB = BLOCK / W * csr_shape<W>::U;
    const int64_t grid = n_long + (n + RPB - 1) / RPB;
    spmv_csr_kernel<V, W, BLOCK><<<dim3((unsigned)grid), dim3(BLOCK), 0, s>>>(
        n, rp, col, static_cast<const V *>(val), static_cast<const V *>(x), (V)alpha, (V)beta,
        static_cast<V *>(y), long_t, n_long, long_rows);
    return hipGetLastError();
}

template <typename V>
static hipError_t launch_csr(hipStream_t s, int64_t n, const int32_t *rp, const int32_t *col,
                             const void *val, const void *x, double alpha, double beta, void *y,
                             int w, int32_t long_t, int64_t n_long,
                             const int32_t *long_rows) {
    switch (w) {
        case 1: return launch_csr_w<V, 1>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 2: return launch_csr_w<V, 2>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 4: return launch_csr_w<V, 4>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 8: return launch_csr_w<V, 8>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 16: return launch_csr_w<V, 16>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 32: return launch_csr_w<V, 32>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        case 64: return launch_csr_w<V, 64>(s, n, rp, col, val, x, alpha, beta, y, long_t, n_long,
                                            long_rows);
        default: return hipErrorInvalidValue;
    }
}

hipError_t spmv_csr(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                    const void *val, const void *x, double alpha, double beta, void *y, int w,
                    int lanes, int64_t n_long, const int32_t *long_rows) {
    if (n == 0) return hipSuccess;
    if (w == kCsrRowThread)
        return t == vt::f64
                   ? launch_csr_rowthread<double>(s, n, rp, col, val, x, alpha, beta, y, lanes)
                   : launch_csr_rowthread<float>(s, n, rp, col, val, x, alpha, beta, y, lanes);
    const int32_t long_t = n_long > 0 ? csr_long_threshold(w) : INT_MAX;
    return t == vt::f64
               ? launch_csr<double>(s, n, rp, col, val, x, alpha, beta, y, w, long_t, n_long, long_rows)
               : launch_csr<float>(s, n, rp, col, val, x, alpha, beta, y, w, long_t, n_long, long_rows);
}

// ====================================================================== merge-path
// Merge-based SpMV (Merrill and Garland, SC'16): the sequence of n row ends
// merged with the nnz entries is cut into equal tiles of TILE items, one per
// workgroup, so work per workgroup does not depend on row lengths.  Tile
// starts are found once per matrix by a binary search along each diagonal
// (merge_partition).  Inside a tile the entries' products are staged in LDS
// with coalesced loads.  For regular rows the tile's rows are then summed in
// parallel, a few lanes per row; otherwise each thread walks IPT items of
// the merge sequentially, and rows that cross thread boundaries are combined
// by a segmented scan of the threads' carry-outs (a DPP scan inside each
// wave, then the wave totals), which keeps every thread's work equal however
// long the rows.  Tiles of 4 items per thread measured best (2048
// items 301 us, 1024 236 us, 512 275 us on the stencil, one workgroup per
// tile).  The staged products are padded by one slot per 8, so the threads'
// walks, which start about IPT entries apart, fall into different LDS banks.  Rows crossing tile boundaries
// leave a carry per tile, added by a second kernel in ascending tile order,
// so results are bitwise repeatable.
constexpr int kMergeBlock = 256;
constexpr int kMergeIpt = 4;
constexpr int kMergeTile = kMergeBlock * kMergeIpt;

int64_t merge_tiles(int64_t n, int64_t nnz) { return (n + nnz + kMergeTile - 1) / kMergeTile; }

// Coordinate on the merge path at diagonal d: rows completed i, entries consumed d - i.
__global__ void merge_partition_kernel(int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                       int32_t *__restrict__ part, int64_t tiles) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w > tiles) return;
    const int64_t d = (w * kMergeTile < n + nnz) ? w * kMergeTile : n + nnz;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < n ? d : n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)rp[mid + 1] <= d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    part[2 * w] = (int32_t)lo;
    part[2 * w + 1] = (int32_t)(d - lo);
}

hipError_t merge_partition(hipStream_t s, int64_t n, int64_t nnz, const int32_t *rp, int32_t *part) {
    const int64_t tiles = merge_tiles(n, nnz);
    const int64_t grid = (tiles + 1 + 255) / 256;
    merge_partition_kernel<<<dim3((unsigned)grid), dim3(256), 0, s>>>(n, nnz, rp, part, tiles);
    return hipGetLastError();
}


// What a workgroup fetches for one tile before it needs it: the tile's start
// on the merge path, its column indices and values (four per thread,
// coalesced) and its row ends.
template <typename V>
struct merge_tile_in {
    int32_t i0, k0, nrows, nk;
    int32_t c[kMergeIpt];
    V v[kMergeIpt];
    int32_t re[kMergeIpt + 1];
};

template <typename V>
__device__ inline void merge_fetch(int64_t w, int64_t n, const int32_t *__restrict__ rp,
                                   const int32_t *__restrict__ col, const V *__restrict__ val,
                                   const int32_t *__restrict__ part, merge_tile_in<V> &T) {
    const int tid = threadIdx.x;
    T.i0 = part[2 * w];
    T.k0 = part[2 * w + 1];
    T.nrows = part[2 * w + 2] - T.i0;
    T.nk = part[2 * w + 3] - T.k0;
#pragma unroll
    for (int j = 0; j < kMergeIpt; ++j) {
        const int t = tid + j * kMergeBlock;
        const bool ok = t < T.nk;
        T.c[j] = ok ? load_stream(col + T.k0 + t) : 0;
        T.v[j] = ok ? load_stream(val + T.k0 + t) : V(0);
    }
#pragma unroll
    for (int j = 0; j <= kMergeIpt; ++j) {
        const int t = tid + j * kMergeBlock;
        T.re[j] = (t <= T.nrows && (int64_t)T.i0 + t < n) ? rp[T.i0 + t + 1] - T.k0 : INT_MAX;
    }
}

// Sum over aligned groups of L lanes (L a power of two, 1..64, uniform
// across the wavefront), every lane getting its group's sum: xor butterfly.
template <typename V>
__device__ inline V subwarp_sum_any(V v, int L) {
    for (int b = 1; b < L; b <<= 1) v += __shfl_xor(v, b, kWave);
    return v;
}

// Persistent: as many workgroups as fit on the chip at once, each taking
// tiles w, w + grid, ...  While a workgroup walks tile w in LDS, the loads of
// its next tile are already in flight (the x gathers of tile w were issued
// first), so memory traffic does not stop during the LDS phase.  27-point
// stencil: 231 us with one workgroup per tile, 188 us persistent.
template <typename V, bool ROWS>
__global__ __launch_bounds__(kMergeBlock) void spmv_merge_kernel(
    int64_t n, int64_t tiles, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
    const V *__restrict__ val, const int32_t *__restrict__ part, const V *__restrict__ x, V alpha,
    V beta, V *__restrict__ y, int32_t *__restrict__ carry_row, V *__restrict__ carry_val) {
    __shared__ V prods[kMergeTile + kMergeTile / 8];  // entry t at t + t / 8
    __shared__ int32_t rend[kMergeTile + 1];
    // the walk's carry scan (ROWS = false)
    __shared__ int32_t s_row[ROWS ? 1 : kMergeBlock];
    __shared__ V s_val[ROWS ? 1 : kMergeBlock];
    __shared__ int32_t w_first[kMergeBlock / kWave], w_last[kMergeBlock / kWave];
    __shared__ V w_tot[kMergeBlock / kWave];

    const int tid = threadIdx.x;
    // The tiles are split over the XCDs in proportion to their workgroups,
    // in contiguous ranges (neighbouring tiles share x lines); the
    // workgroups of an XCD stride through its range.
    const int64_t G = gridDim.x, xcd = blockIdx.x % kXcds, q = G / kXcds, rq = G % kXcds;
    const int64_t gx = q + (xcd < rq ? 1 : 0);
    const int64_t p0 = xcd * q + (xcd < rq ? xcd : rq);
    const int64_t t_end = tiles * (p0 + gx) / G;
    int64_t w = tiles * p0 / G + blockIdx.x / kXcds;
    if (w >= t_end) return;
    merge_tile_in<V> cur;
    merge_fetch(w, n, rp, col, val, part, cur);
    for (; w < t_end; w += gx) {
        V pr[kMergeIpt];
#pragma unroll
        for (int j = 0; j < kMergeIpt; ++j) {
            const int t = tid + j * kMergeBlock;
            pr[j] = t < cur.nk ? cur.v[j] * x[cur.c[j]] : V(0);
        }
        const bool more = w + gx < t_end;
        merge_tile_in<V> nxt;
        if (more) merge_fetch(w + gx, n, rp, col, val, part, nxt);
        const int32_t i0 = cur.i0, nrows = cur.nrows, nk = cur.nk;
#pragma unroll
        for (int j = 0; j < kMergeIpt; ++j) {
            const int t = tid + j * kMergeBlock;
            if (t < nk) prods[t + (t >> 3)] = pr[j];
        }
#pragma unroll
        for (int j = 0; j <= kMergeIpt; ++j) {
            const int t = tid + j * kMergeBlock;
            if (t <= nrows) rend[t] = cur.re[j];
        }
        __syncthreads();

        if constexpr (ROWS) {
            // Rows of the tile in parallel: rows j = 0..nrows (the last one ends
            // in a later tile) get L lanes each, L the largest power of two with
            // L (nrows + 1) <= the workgroup (at most a wavefront); lane l sums
            // the row's staged products l, l + L, ... and the L lanes add their
            // sums by a xor butterfly.  Rows never straddle a wavefront.
            const int nr1 = nrows + 1;
            int L = 1;
            while (L < kWave && 2 * L * nr1 <= kMergeBlock) L *= 2;
            for (int j0 = 0; j0 < nr1; j0 += kMergeBlock / L) {
                const int j = j0 + tid / L, l = tid % L;
                V acc = V(0);
                if (j < nr1) {
                    const int kb = j == 0 ? 0 : rend[j - 1];
                    const int ke = j < nrows ? rend[j] : nk;
                    for (int k = kb + l; k < ke; k += L) acc += prods[k + (k >> 3)];
                }
                acc = subwarp_sum_any(acc, L);
                if (j < nr1 && l == 0) {
                    const int64_t r = (int64_t)i0 + j;
                    if (j < nrows) {
                        if (r < n) y[r] = (beta == V(0)) ? alpha * acc : alpha * acc + beta * y[r];
                    } else {
                        carry_row[w] = r < n ? (int32_t)r : -1;
                        carry_val[w] = acc;
                    }
                }
            }
            __syncthreads();  // prods and rend are rewritten for the next tile
        } else {
            const int total = nrows + nk;
            const int d = tid * kMergeIpt < total ? tid * kMergeIpt : total;
            int lo = d - nk > 0 ? d - nk : 0;
            int hi = d < nrows ? d : nrows;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (rend[mid] <= d - mid - 1) lo = mid + 1;
                else hi = mid;
            }
            int i = lo, k = d - lo;
            const int dend = d + kMergeIpt < total ? d + kMergeIpt : total;
            V acc = V(0);
            int first_row = -1;
            V first_val = V(0);
            for (int step = d; step < dend && i <= nrows; ++step) {
                if (k < rend[i] && k < nk) {
                    acc += prods[k + (k >> 3)];
                    ++k;
                } else {
                    const int64_t r = (int64_t)i0 + i;
                    if (first_row < 0) {
                        first_row = i;
                        first_val = acc;
                    } else if (r < n) {
                        y[r] = (beta == V(0)) ? alpha * acc : alpha * acc + beta * y[r];
                    }
                    acc = V(0);
                    ++i;
                }
            }
            V sv = acc;
            const int sr = i;
            wave_segmented_scan(sv, sr);
            const int wv = tid / kWave, ln = tid % kWave;
            if (ln == kWave - 1) { w_last[wv] = sr; w_tot[wv] = sv; }
            if (ln == 0) w_first[wv] = sr;
            __syncthreads();
            for (int q = wv - 1; q >= 0; --q) {
                if (w_last[q] != sr) break;
                sv += w_tot[q];
                if (w_first[q] != sr) break;
            }
            s_row[tid] = sr;
            s_val[tid] = sv;
            __syncthreads();
            if (first_row >= 0 && (int64_t)i0 + first_row < n) {
                V v = first_val;
                if (tid > 0) v += s_val[tid - 1];
                const int64_t r = (int64_t)i0 + first_row;
                y[r] = (beta == V(0)) ? alpha * v : alpha * v + beta * y[r];
            }
            if (tid == kMergeBlock - 1) {
                const int64_t r = (int64_t)i0 + s_row[tid];
                carry_row[w] = r < n ? (int32_t)r : -1;
                carry_val[w] = s_val[tid];
            }
        }
        if (more) cur = nxt;
    }
}

// Adds tile carries: the first tile of each run of tiles ending inside the
// same row sums the run in tile order and adds it to y.
template <typename V>
__global__ void merge_fixup_kernel(int64_t tiles, const int32_t *__restrict__ carry_row,
                                   const V *__restrict__ carry_val, V alpha, V *__restrict__ y) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= tiles) return;
    const int32_t r = carry_row[w];
    if (r < 0) return;
    if (w > 0 && carry_row[w - 1] == r) return;
    V s = carry_val[w];
    for (int64_t u = w + 1; u < tiles && carry_row[u] == r; ++u) s += carry_val[u];
    y[r] += alpha * s;
}

template <typename V, bool ROWS>
static hipError_t launch_merge(hipStream_t s, int64_t n, int64_t nnz, const int32_t *rp,
                               const int32_t *col, const void *val, const int32_t *part,
                               const void *x, double alpha, double beta, void *y,
                               int32_t *carry_row, void *carry_val) {
    const int64_t tiles = merge_tiles(n, nnz);
    // workgroups that fit on the device at once, per device
    static int resident_of[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    int &resident = resident_of[dev];
    if (!resident) {
        int cus = 0, per = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, spmv_merge_kernel<V, ROWS>, kMergeBlock, 0) !=
                hipSuccess)
            return hipErrorInvalidValue;
        resident = cus * (per > 0 ? per : 1);
    }
    const int64_t grid = tiles < resident ? tiles : resident;
    spmv_merge_kernel<V, ROWS><<<dim3((unsigned)grid), dim3(kMergeBlock), 0, s>>>(
        n, tiles, rp, col, static_cast<const V *>(val), part, static_cast<const V *>(x), (V)alpha,
        (V)beta, static_cast<V *>(y), carry_row, static_cast<V *>(carry_val));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    merge_fixup_kernel<V><<<dim3((unsigned)((tiles + 255) / 256)), dim3(256), 0, s>>>(
        tiles, carry_row, static_cast<const V *>(carry_val), (V)alpha, static_cast<V *>(y));
    return hipGetLastError();
}

hipError_t spmv_merge(hipStream_t s, vt t, int64_t n, int64_t nnz, const int32_t *rp,
                      const int32_t *col, const void *val, const int32_t *part, const void *x,
                      double alpha, double beta, void *y, int32_t *carry_row, void *carry_val,
                      bool rows) {
    if (n == 0) return hipSuccess;
    if (t == vt::f64)
        return rows ? launch_merge<double, true>(s, n, nnz, rp, col, val, part, x, alpha, beta, y,
                                                 carry_row, carry_val)
                    : launch_merge<double, false>(s, n, nnz, rp, col, val, part, x, alpha, beta, y,
                                                  carry_row, carry_val);
    return rows ? launch_merge<float, true>(s, n, nnz, rp, col, val, part, x, alpha, beta, y,
                                            carry_row, carry_val)
                : launch_merge<float, false>(s, n, nnz, rp, col, val, part, x, alpha, beta, y,
                                             carry_row, carry_val);
}

// Rows summed in parallel per tile for regular rows (longest <= 4 x mean);
// the merge walk otherwise.  27-point stencil 128^3: 190 -> 168 us; the
// lognormal random matrix (longest 10,000 against a mean of 16): walk 179
// us, rows in parallel 187 us.
bool merge_rows_parallel(int64_t n, int64_t nnz, int64_t max_len) {
    const double mean = n > 0 ? (double)nnz / (double)n : 0.0;
    return (double)max_len <= 4.0 * mean;
}

}  // namespace gko
