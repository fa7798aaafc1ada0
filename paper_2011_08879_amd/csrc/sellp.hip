// SELL-P: SpMV and conversions.
//
// SELL-P (Anzt, Tomov and Dongarra 2014) pads each slice of kSellpSlice
// consecutive rows to that slice's longest row, instead of padding every row
// to the longest row of the matrix as ELL does: irregular matrices store far
// fewer padding slots, while the column-major slots inside a slice keep the
// coalesced, reduction-free access of ELL.  A slice of 64 rows is one
// wavefront (a row per thread) and a workgroup of 256 threads covers 4
// slices.  No row sorting, stride factor 1.  A slice made wide by a few very
// long rows is split into column chunks instead, so no single wavefront
// walks thousands of slots (one 10,000-entry row among lognormal rows of
// mean 16: 2.8 ms with one wavefront for its slice).
#include "device.hpp"
#include "ell_rows.hpp"
#include "kernels.hpp"

namespace gko {

namespace {

constexpr int kSellpBlock = 256;

inline unsigned blocks_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

template <typename V>
__global__ __launch_bounds__(kSellpBlock) void spmv_sellp_kernel(int64_t n,
                                                                 const int64_t *__restrict__ sets,
                                                                 const int32_t *__restrict__ scol,
                                                                 const V *__restrict__ sval,
                                                                 const V *__restrict__ x, V alpha,
                                                                 V beta, V *__restrict__ y) {
    // up to kXcdRowsMax rows each XCD takes one contiguous range of slices
    const int64_t i = row_block_order(n) * kSellpBlock + threadIdx.x;
    if (i >= n) return;
    const sellp_slice_of sl = sellp_slice(i, sets);
    if (sl.w > kSellpWide) return;  // the whole wavefront: the wide-slice kernels
    const V s0 = sellp_slots_sum(sl.base, sl.r, 0, sl.w, scol, sval, x);
    y[i] = (beta == V(0)) ? alpha * s0 : alpha * s0 + beta * y[i];
}

// Work item q of the wide slices: columns [j0, j0 + kSellpWideChunk) of
// slice s, a wavefront; partial[q * 64 + r] <- the partial sum of row r.
template <typename V>
__global__ __launch_bounds__(kSellpBlock) void sellp_wide_kernel(int64_t n_items,
                                                                 const int32_t *__restrict__ items,
                                                                 const int64_t *__restrict__ sets,
                                                                 const int32_t *__restrict__ scol,
                                                                 const V *__restrict__ sval,
                                                                 const V *__restrict__ x,
                                                                 V *__restrict__ partial) {
    const int64_t q = (int64_t)blockIdx.x * (kSellpBlock / kWave) + threadIdx.x / kWave;
    if (q >= n_items) return;  // a whole wavefront
    const int r = threadIdx.x % kWave;
    const int64_t sl = items[2 * q], j0 = items[2 * q + 1];
    const int64_t base = sets[sl], w = (sets[sl + 1] - base) / kSellpSlice;
    const int64_t j1 = j0 + kSellpWideChunk < w ? j0 + kSellpWideChunk : w;
    partial[q * kSellpSlice + r] = sellp_slots_sum(base, r, j0, j1, scol, sval, x);
}

// Wide slice q (a wavefront): row r's partials in item order, then y.
template <typename V>
__global__ __launch_bounds__(kSellpBlock) void sellp_wide_sum_kernel(
    int64_t n, int64_t n_wide, const int32_t *__restrict__ slices,
    const int32_t *__restrict__ first, const V *__restrict__ partial, V alpha, V beta,
    V *__restrict__ y) {
    const int64_t q = (int64_t)blockIdx.x * (kSellpBlock / kWave) + threadIdx.x / kWave;
    if (q >= n_wide) return;
    const int r = threadIdx.x % kWave;
    V s = V(0);
    for (int32_t t = first[q]; t < first[q + 1]; ++t) s += partial[(int64_t)t * kSellpSlice + r];
    const int64_t i = (int64_t)slices[q] * kSellpSlice + r;
    if (i < n) y[i] = (beta == V(0)) ? alpha * s : alpha * s + beta * y[i];
}

template <typename V>
hipError_t launch_sellp(hipStream_t s, int64_t n, const int64_t *sets, const int32_t *scol,
                        const void *sval, const void *x, double alpha, double beta, void *y,
                        const sellp_wide &wide) {
    const V *SV = static_cast<const V *>(sval), *X = static_cast<const V *>(x);
    V *Y = static_cast<V *>(y);
    spmv_sellp_kernel<V><<<blocks_for(n, kSellpBlock), kSellpBlock, 0, s>>>(
        n, sets, scol, SV, X, (V)alpha, (V)beta, Y);
    if (wide.n_wide == 0) return hipGetLastError();
    constexpr int WPB = kSellpBlock / kWave;
    V *P = static_cast<V *>(wide.partial);
    sellp_wide_kernel<V><<<blocks_for(wide.n_items, WPB), kSellpBlock, 0, s>>>(
        wide.n_items, wide.items, sets, scol, SV, X, P);
    sellp_wide_sum_kernel<V><<<blocks_for(wide.n_wide, WPB), kSellpBlock, 0, s>>>(
        n, wide.n_wide, wide.slices, wide.first, P, (V)alpha, (V)beta, Y);
    return hipGetLastError();
}

// ---------------------------------------------------------------- conversions
__global__ void sellp_widths_kernel(int64_t n, int64_t ns, const int32_t *__restrict__ rp,
                                    int32_t *__restrict__ widths) {
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= ns) return;
    const int64_t e = (sl + 1) * kSellpSlice < n ? (sl + 1) * kSellpSlice : n;
    int32_t w = 0;
    for (int64_t i = sl * kSellpSlice; i < e; ++i) {
        const int32_t l = rp[i + 1] - rp[i];
        w = l > w ? l : w;
    }
    widths[sl] = w;
}

// One thread per row of the padded slices (rows >= n write padding).
template <typename V>
__global__ void csr_to_sellp_kernel(int64_t n, int64_t rows, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col, const V *__restrict__ val,
                                    const int64_t *__restrict__ sets, int32_t *__restrict__ scol,
                                    V *__restrict__ sval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows) return;
    const int64_t sl = i / kSellpSlice, r = i - sl * kSellpSlice;
    const int64_t base = sets[sl] + r, w = (sets[sl + 1] - sets[sl]) / kSellpSlice;
    const int64_t b = i < n ? rp[i] : 0;
    const int64_t len = i < n ? rp[i + 1] - b : 0;
    for (int64_t j = 0; j < w; ++j) {
        const int64_t slot = base + j * kSellpSlice;
        scol[slot] = j < len ? col[b + j] : -1;
        sval[slot] = j < len ? val[b + j] : V(0);
    }
}

// A row's entries are its slots up to the first padding slot.
__global__ void sellp_len_kernel(int64_t n, const int64_t *__restrict__ sets,
                                 const int32_t *__restrict__ scol, int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t sl = i / kSellpSlice, r = i - sl * kSellpSlice;
    const int64_t base = sets[sl] + r, w = (sets[sl + 1] - sets[sl]) / kSellpSlice;
    int32_t l = 0;
    while (l < w && scol[base + l * kSellpSlice] >= 0) ++l;
    len[i] = l;
}

template <typename V>
__global__ void sellp_to_csr_kernel(int64_t n, const int64_t *__restrict__ sets,
                                    const int32_t *__restrict__ scol, const V *__restrict__ sval,
                                    const int32_t *__restrict__ rp, int32_t *__restrict__ col,
                                    V *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t sl = i / kSellpSlice, r = i - sl * kSellpSlice;
    const int64_t base = sets[sl] + r;
    const int64_t o = rp[i], len = rp[i + 1] - o;
    for (int64_t j = 0; j < len; ++j) {
        col[o + j] = scol[base + j * kSellpSlice];
        val[o + j] = sval[base + j * kSellpSlice];
    }
}

}  // namespace

hipError_t spmv_sellp(hipStream_t s, vt t, int64_t n, const int64_t *sets, const int32_t *scol,
                      const void *sval, const void *x, double alpha, double beta, void *y,
                      const sellp_wide &wide) {
    if (n == 0) return hipSuccess;
    return t == vt::f64 ? launch_sellp<double>(s, n, sets, scol, sval, x, alpha, beta, y, wide)
                        : launch_sellp<float>(s, n, sets, scol, sval, x, alpha, beta, y, wide);
}

hipError_t sellp_widths(hipStream_t s, int64_t n, const int32_t *rp, int32_t *widths) {
    const int64_t ns = (n + kSellpSlice - 1) / kSellpSlice;
    if (ns == 0) return hipSuccess;
    sellp_widths_kernel<<<blocks_for(ns, 256), 256, 0, s>>>(n, ns, rp, widths);
    return hipGetLastError();
}

hipError_t csr_to_sellp(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                        const void *val, const int64_t *sets, int32_t *scol, void *sval) {
    const int64_t rows = (n + kSellpSlice - 1) / kSellpSlice * kSellpSlice;
    if (rows == 0) return hipSuccess;
    if (t == vt::f64)
        csr_to_sellp_kernel<double><<<blocks_for(rows, 256), 256, 0, s>>>(
            n, rows, rp, col, static_cast<const double *>(val), sets, scol,
            static_cast<double *>(sval));
    else
        csr_to_sellp_kernel<float><<<blocks_for(rows, 256), 256, 0, s>>>(
            n, rows, rp, col, static_cast<const float *>(val), sets, scol,
            static_cast<float *>(sval));
    return hipGetLastError();
}

hipError_t sellp_lengths(hipStream_t s, int64_t n, const int64_t *sets, const int32_t *scol,
                         int32_t *len) {
    if (n == 0) return hipSuccess;
    sellp_len_kernel<<<blocks_for(n, 256), 256, 0, s>>>(n, sets, scol, len);
    return hipGetLastError();
}

hipError_t sellp_to_csr(hipStream_t s, vt t, int64_t n, const int64_t *sets, const int32_t *scol,
                        const void *sval, const int32_t *rp, int32_t *col, void *val) {
    if (n == 0) return hipSuccess;
    if (t == vt::f64)
        sellp_to_csr_kernel<double><<<blocks_for(n, 256), 256, 0, s>>>(
            n, sets, scol, static_cast<const double *>(sval), rp, col, static_cast<double *>(val));
    else
        sellp_to_csr_kernel<float><<<blocks_for(n, 256), 256, 0, s>>>(
            n, sets, scol, static_cast<const float *>(sval), rp, col, static_cast<float *>(val));
    return hipGetLastError();
}

}  // namespace gko
