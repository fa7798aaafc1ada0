// Host-side launchers of the HIP kernels.  Plain pointers and sizes only;
// every launcher enqueues on the given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gko {

enum class vt { f64 = 0, f32 = 1 };  // value type of a kernel instance

inline size_t vsize(vt t) { return t == vt::f64 ? 8 : 4; }

// ------------------------------------------------------------------ SpMV
// CSR, a subwarp of w lanes per row (w a power of two <= 64).  Rows longer
// than csr_long_threshold(w) are listed in long_rows (n_long of them) and
// summed by a workgroup each.  w = kCsrRowThread: a thread per row with the
// entries staged through LDS and `lanes` lanes per row (for short rows of
// similar length, see csr_kernel_width and csr_row_lanes; no long rows then).
constexpr int kCsrRowThread = 0;
constexpr int64_t kCsrRowThreadMaxLen = 256;
// Power of two >= the mean row length, at most 64.
int csr_subwarp_width(int64_t n, int64_t nnz);
// The kernel for a matrix: kCsrRowThread or a subwarp width.
int csr_kernel_width(int64_t n, int64_t nnz, int64_t max_len);
// Lanes per row (1, 4 or 8) of the row-per-thread kernel.
int csr_row_lanes(int64_t n, int64_t nnz);
// Whether rows longer than csr_long_threshold(w) get the workgroup-per-row
// kernel: only for irregular rows (longest > 4 x mean).
bool csr_has_long_rows(int64_t n, int64_t nnz, int64_t max_len, int w);
int32_t csr_long_threshold(int w);
hipError_t spmv_csr(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                    const void *val, const void *x, double alpha, double beta, void *y, int w,
                    int lanes, int64_t n_long, const int32_t *long_rows);
// flag[i] = len_i > long_t; rows[pos[i]] = i for flagged rows (pos: exclusive scan of flag).
hipError_t csr_long_flags(hipStream_t s, int64_t n, const int32_t *rp, int32_t long_t, int32_t *flag);
hipError_t csr_long_scatter(hipStream_t s, int64_t n, const int32_t *flag, const int32_t *pos,
                            int32_t *rows);

// CSR merge-path: equal (rows + nonzeros) tiles per workgroup.
int64_t merge_tiles(int64_t n, int64_t nnz);
hipError_t merge_partition(hipStream_t s, int64_t n, int64_t nnz, const int32_t *rp,
                           int32_t *part /* 2*(tiles+1) */);
// carry_row: tiles int32, carry_val: tiles values of type t.  rows: sum each
// tile's rows in parallel (merge_rows_parallel) instead of the merge walk.
hipError_t spmv_merge(hipStream_t s, vt t, int64_t n, int64_t nnz, const int32_t *rp,
                      const int32_t *col, const void *val, const int32_t *part, const void *x,
                      double alpha, double beta, void *y, int32_t *carry_row, void *carry_val,
                      bool rows);
// Whether a matrix's merge tiles sum their rows in parallel: regular rows.
bool merge_rows_parallel(int64_t n, int64_t nnz, int64_t max_len);

// COO: equal nonzero chunks per wavefront.  accumulate: y += alpha A x, rows
// without entries untouched (used for the HYB tail).
int64_t coo_chunks(int64_t nnz);
// head/tail: coo_chunks(nnz) values of type t each.
hipError_t spmv_coo(hipStream_t s, vt t, int64_t n, int64_t nnz, const int32_t *row,
                    const int32_t *col, const void *val, const void *x, double alpha, double beta,
                    void *y, bool accumulate, void *head, void *tail);

// ELL: column-major slots, thread per row.
hipError_t spmv_ell(hipStream_t s, vt t, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                    const void *eval, const void *x, double alpha, double beta, void *y);

// SELL-P (sliced ELL with padding): rows in slices of kSellpSlice, slice s
// padded to its own longest row w_s and stored column-major inside the
// slice; slot (j, r) of slice s -- entry j of row s*kSellpSlice + r -- is at
// sets[s] + j*kSellpSlice + r, sets[s+1] = sets[s] + w_s*kSellpSlice.
// Padding (and rows >= n of the last slice): col = -1, val = +0.0.
constexpr int kSellpSlice = 64;
// Slices wider than kSellpWide (a few very long rows) are not walked by one
// wavefront: their slots are cut into work items of kSellpWideChunk columns
// (one wavefront each, partial sums per row), which a second kernel adds in
// item order.  wide: the n_wide slices (wide.slices), the [first, last) item
// range of each (wide.first, n_wide + 1 entries), the items as (slice,
// first column) pairs (wide.items, n_items of them) and partial-sum scratch
// of n_items * kSellpSlice values (wide.partial).
constexpr int64_t kSellpWide = 512;
constexpr int64_t kSellpWideChunk = 256;
struct sellp_wide {
    int64_t n_wide = 0, n_items = 0;
    const int32_t *slices = nullptr, *first = nullptr, *items = nullptr;
    void *partial = nullptr;
};
hipError_t spmv_sellp(hipStream_t s, vt t, int64_t n, const int64_t *sets, const int32_t *scol,
                      const void *sval, const void *x, double alpha, double beta, void *y,
                      const sellp_wide &wide);

// y <- beta * y (beta == 0: y <- 0 without reading y).
hipError_t scale(hipStream_t s, vt t, int64_t n, double beta, void *y);

// ------------------------------------------------------------------ conversions
// err: one device int, set nonzero on a violation (bit 1: row_ptr, 2: col range, 4: col order).
hipError_t validate_csr(hipStream_t s, int64_t n, int64_t m, int64_t nnz, const int32_t *rp,
                        const int32_t *col, int *err);
hipError_t narrow_row_ptr(hipStream_t s, int64_t n, const int64_t *rp64, int32_t *rp32, int *err);
hipError_t csr_rows(hipStream_t s, int64_t n, const int32_t *rp, int32_t *row);
hipError_t rows_to_ptr(hipStream_t s, int64_t n, int64_t nnz, const int32_t *row, int32_t *rp);
// maxlen: one device int, must be zero on entry.
hipError_t max_row_len(hipStream_t s, int64_t n, const int32_t *rp, int *maxlen);
// hist: maxlen+1 device ints, zero on entry.
hipError_t row_len_hist(hipStream_t s, int64_t n, const int32_t *rp, int *hist, int64_t maxlen);
// STREAM probe: op 0 c = a, op 1 c = a + sc * b (two roundings).
// y[i] = x[idx[i]] for i < n; x holds m doubles (an index outside reads 0).
// Requires 16-byte aligned idx and y and m * 8 < 2^31.
hipError_t gather_probe(hipStream_t s, int64_t n, const double *x, int64_t m, const int32_t *idx,
                        double *y);
hipError_t stream_op(hipStream_t s, int op, int64_t n, const double *a, const double *b, double sc,
                     double *c);
hipError_t csr_to_ell(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                      const void *val, int64_t K, int64_t ld, int32_t *ecol, void *eval);
// tail_ptr: n+1 offsets of the tail entries of each row (exclusive scan of max(0, len-K)).
hipError_t tail_lengths(hipStream_t s, int64_t n, const int32_t *rp, int64_t K, int32_t *len);
hipError_t csr_to_tail(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                       const void *val, int64_t K, const int32_t *tail_ptr, int32_t *trow,
                       int32_t *tcol, void *tval);
// lengths of rows stored as ELL (+ optional COO tail given by its row offsets).
hipError_t hyb_lengths(hipStream_t s, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                       const int32_t *tail_ptr, int32_t *len);
hipError_t hyb_to_csr(hipStream_t s, vt t, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                      const void *eval, const int32_t *tail_ptr, const int32_t *tcol,
                      const void *tval, const int32_t *rp, int32_t *col, void *val);
// SELL-P conversions: widths[s] = longest row of slice s; the slot arrays
// from CSR given sets; row lengths and CSR arrays back from the slots.
hipError_t sellp_widths(hipStream_t s, int64_t n, const int32_t *rp, int32_t *widths);
hipError_t csr_to_sellp(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                        const void *val, const int64_t *sets, int32_t *scol, void *sval);
hipError_t sellp_lengths(hipStream_t s, int64_t n, const int64_t *sets, const int32_t *scol,
                         int32_t *len);
hipError_t sellp_to_csr(hipStream_t s, vt t, int64_t n, const int64_t *sets, const int32_t *scol,
                        const void *sval, const int32_t *rp, int32_t *col, void *val);
// Exclusive scan of n int32 lengths into n+1 offsets; tmp: scan_tmp_elems(n) ints.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan(hipStream_t s, int64_t n, const int32_t *len, int32_t *out, int32_t *tmp);
hipError_t cast_values(hipStream_t s, vt from, vt to, int64_t n, const void *src, void *dst);

// ------------------------------------------------------------------ reductions
constexpr int kRedBlock = 256;
// Reduction kernels launch at most this many blocks (grid-stride loops
// beyond), so partial-sum scratch of NV * kMaxReductionBlocks doubles fits
// every launch of the vector kernels (the fused products below need
// kFusedMaxSums * kFusedMaxBlocks doubles).
constexpr int kMaxReductionBlocks = 2048;
// The CG products with p.q fused in launch a thread (or row pair) per row up
// to this many blocks, with one partial sum per block: a 2048-block
// grid-stride product ran 6% slower per CG iteration on the 7-point Poisson
// matrix 256^3 (SELL-P 609 -> 574 us, CSR 635 -> 597 us).
constexpr int kFusedMaxBlocks = 65536;
// A fused product forms at most this many sums per block, so its scratch is
// kFusedMaxSums * kFusedMaxBlocks doubles.
constexpr int kFusedMaxSums = 2;
int reduction_blocks(int64_t n);
// Grid of a vector kernel without a reduction: one element per thread up to
// kFusedMaxBlocks blocks of 256, grid-stride beyond.  Per iteration on the
// 3D Poisson matrix with 2^24 rows, against the 2048-block grid: CG 0.563 ->
// 0.549 ms (the direction update), BiCGSTAB 1.067 -> 1.055 ms (p update),
// CGS 1.089 -> 1.061 ms (q, w, x and direction updates); GMRES's scaling
// pass no faster.
int stream_blocks(int64_t n);
// result: one device double. partials: kMaxReductionBlocks doubles; ticket: zeroed uint.
hipError_t dot(hipStream_t s, vt t, int64_t n, const void *x, const void *y, double *result,
               double *partials, unsigned *ticket, bool sqrt_result);

}  // namespace gko
