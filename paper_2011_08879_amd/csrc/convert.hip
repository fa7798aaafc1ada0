// Format conversions and structure checks on the device.  All of it is
// integer bookkeeping and copies, so results are bit-exact by construction:
//   CSR -> COO : expand row offsets into row indices.
//   COO -> CSR : row_ptr[i] = first entry with row >= i (binary search).
//   CSR -> ELL : slot (j, i) at j*ld + i = j-th entry of row i, else padding
//                col = -1, val = +0.0.
//   CSR -> HYB : ELL of width K plus a COO tail with entries K.. of each row.
//   ELL/HYB -> CSR : per-row counts, exclusive scan, copy.
#include <climits>
#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace gko {

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ------------------------------------------------------------------ validation
__global__ void validate_csr_kernel(int64_t n, int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col, int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    if (i == 0 && rp[0] != 0) atomicOr(err, 1);
    if (i == n) {
        if ((int64_t)rp[n] != nnz) atomicOr(err, 1);
        return;
    }
    const int32_t b = rp[i], e = rp[i + 1];
    if (e < b || b < 0 || (int64_t)e > nnz) {
        atomicOr(err, 1);
        return;
    }
    int bad = 0;
    for (int32_t k = b; k < e; ++k) {
        const int32_t c = col[k];
        if (c < 0 || (int64_t)c >= m) bad |= 2;
        if (k > b && c <= col[k - 1]) bad |= 4;
    }
    if (bad) atomicOr(err, bad);
}

hipError_t validate_csr(hipStream_t s, int64_t n, int64_t m, int64_t nnz, const int32_t *rp,
                        const int32_t *col, int *err) {
    validate_csr_kernel<<<grid_for(n + 1, 256), 256, 0, s>>>(n, m, nnz, rp, col, err);
    return hipGetLastError();
}

__global__ void narrow_kernel(int64_t n, const int64_t *__restrict__ rp64, int32_t *__restrict__ rp32,
                              int *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    const int64_t v = rp64[i];
    if (v < 0 || v > INT_MAX) atomicOr(err, 1);
    rp32[i] = (int32_t)v;
}

hipError_t narrow_row_ptr(hipStream_t s, int64_t n, const int64_t *rp64, int32_t *rp32, int *err) {
    narrow_kernel<<<grid_for(n + 1, 256), 256, 0, s>>>(n, rp64, rp32, err);
    return hipGetLastError();
}

// ------------------------------------------------------------------ CSR <-> COO
// One wave per row: lanes write consecutive row indices.
__global__ void csr_rows_kernel(int64_t n, const int32_t *__restrict__ rp, int32_t *__restrict__ row) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const int lane = threadIdx.x % kWave;
    for (int32_t k = rp[i] + lane; k < rp[i + 1]; k += kWave) row[k] = (int32_t)i;
}

hipError_t csr_rows(hipStream_t s, int64_t n, const int32_t *rp, int32_t *row) {
    if (n == 0) return hipSuccess;
    csr_rows_kernel<<<grid_for(n, 4), 256, 0, s>>>(n, rp, row);
    return hipGetLastError();
}

__global__ void rows_to_ptr_kernel(int64_t n, int64_t nnz, const int32_t *__restrict__ row,
                                   int32_t *__restrict__ rp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    int64_t lo = 0, hi = nnz;  // first k with row[k] >= i
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (row[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    rp[i] = (int32_t)lo;
}

hipError_t rows_to_ptr(hipStream_t s, int64_t n, int64_t nnz, const int32_t *row, int32_t *rp) {
    rows_to_ptr_kernel<<<grid_for(n + 1, 256), 256, 0, s>>>(n, nnz, row, rp);
    return hipGetLastError();
}

// ------------------------------------------------------------------ row lengths
__global__ void max_len_kernel(int64_t n, const int32_t *__restrict__ rp, int *maxlen) {
    __shared__ int lds[256 / kWave];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int v = i < n ? rp[i + 1] - rp[i] : 0;
#pragma unroll
    for (int b = 1; b < kWave; b <<= 1) v = max(v, __shfl_xor(v, b));
    if ((threadIdx.x % kWave) == 0) lds[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) v = max(v, lds[w]);
        atomicMax(maxlen, v);
    }
}

hipError_t max_row_len(hipStream_t s, int64_t n, const int32_t *rp, int *maxlen) {
    if (n == 0) return hipSuccess;
    max_len_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, maxlen);
    return hipGetLastError();
}

// Row-length histogram.  Row lengths of structured matrices take few
// distinct values, so counting straight into global memory serialises on a
// handful of addresses; each block counts into LDS first (when the bins fit)
// and adds its nonzero bins once.
constexpr int kHistLdsBins = 8192;

__global__ void hist_lds_kernel(int64_t n, const int32_t *__restrict__ rp, int *hist, int nbins) {
    __shared__ int lh[kHistLdsBins];
    for (int t = threadIdx.x; t < nbins; t += blockDim.x) lh[t] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&lh[rp[i + 1] - rp[i]], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < nbins; t += blockDim.x)
        if (lh[t]) atomicAdd(hist + t, lh[t]);
}

__global__ void hist_kernel(int64_t n, const int32_t *__restrict__ rp, int *hist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(hist + (rp[i + 1] - rp[i]), 1);
}

hipError_t row_len_hist(hipStream_t s, int64_t n, const int32_t *rp, int *hist, int64_t maxlen) {
    if (n == 0) return hipSuccess;
    if (maxlen + 1 <= kHistLdsBins) {
        const unsigned g = grid_for(n, 256) < 1024 ? grid_for(n, 256) : 1024;
        hist_lds_kernel<<<g, 256, 0, s>>>(n, rp, hist, (int)(maxlen + 1));
    } else {
        hist_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, hist);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ STREAM probe
// Each thread moves one pair of doubles with 16-byte non-temporal loads and
// stores, the access shape that measured fastest on MI355X (about 6.6 TB/s
// for a 1 GiB copy, against 6.2 TB/s with one double per thread); an odd
// last element is handled by the thread of the last pair.  Arrays that are
// not all 16-byte aligned take the one-double-per-thread kernels.
typedef double dpair __attribute__((ext_vector_type(2)));

__global__ void stream_copy1_kernel(int64_t n, const double *__restrict__ a, double *__restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = a[i];
}

__global__ void stream_triad1_kernel(int64_t n, const double *__restrict__ a,
                                     const double *__restrict__ b, double sc, double *__restrict__ c) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = a[i] + sc * b[i];
}

__global__ void stream_copy_kernel(int64_t n, const double *__restrict__ a, double *__restrict__ c) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = n / 2;
    if (i < np) {
        const dpair v = __builtin_nontemporal_load(reinterpret_cast<const dpair *>(a) + i);
        __builtin_nontemporal_store(v, reinterpret_cast<dpair *>(c) + i);
    }
    if (i == np - (np > 0 ? 1 : 0) && (n & 1)) c[n - 1] = a[n - 1];
}

__global__ void stream_triad_kernel(int64_t n, const double *__restrict__ a,
                                    const double *__restrict__ b, double sc, double *__restrict__ c) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t np = n / 2;
    if (i < np) {
        const dpair va = __builtin_nontemporal_load(reinterpret_cast<const dpair *>(a) + i);
        const dpair vb = __builtin_nontemporal_load(reinterpret_cast<const dpair *>(b) + i);
        dpair r;
        r.x = va.x + sc * vb.x;
        r.y = va.y + sc * vb.y;
        __builtin_nontemporal_store(r, reinterpret_cast<dpair *>(c) + i);
    }
    if (i == np - (np > 0 ? 1 : 0) && (n & 1)) c[n - 1] = a[n - 1] + sc * b[n - 1];
}

hipError_t stream_op(hipStream_t s, int op, int64_t n, const double *a, const double *b, double sc,
                     double *c) {
    if (n == 0) return hipSuccess;
    const uintptr_t bits = (uintptr_t)a | (uintptr_t)c | (op == 0 ? 0 : (uintptr_t)b);
    if (bits & 15) {
        if (op == 0) stream_copy1_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, a, c);
        else stream_triad1_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, a, b, sc, c);
        return hipGetLastError();
    }
    const int64_t threads = n / 2 > 0 ? n / 2 : 1;
    if (op == 0) stream_copy_kernel<<<grid_for(threads, 256), 256, 0, s>>>(n, a, c);
    else stream_triad_kernel<<<grid_for(threads, 256), 256, 0, s>>>(n, a, b, sc, c);
    return hipGetLastError();
}

// Random-gather probe: y[i] = x[idx[i]].  A wavefront takes 256 consecutive
// elements as two runs of 128, each lane two adjacent elements per run, so
// every index load (8 bytes a lane) and every store (16 bytes a lane) covers
// one contiguous range; the four gathers are issued before any result is
// used.  x is read through a buffer resource of m doubles, so an index
// outside [0, m) reads 0 instead of faulting.  Index and output streams are
// non-temporal, so the L2 holds x the way an SpMV's gathers do.
typedef int32_t probe_i2 __attribute__((ext_vector_type(2)));
typedef double probe_d2 __attribute__((ext_vector_type(2)));
constexpr int kProbeBlock = 256;

__device__ inline double probe_gather(__amdgpu_buffer_rsrc_t rx, int32_t c) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rx, c * 8, 0, 0));
}

__global__ __launch_bounds__(kProbeBlock) void gather_probe_kernel(
    int64_t n, const double *__restrict__ x, int64_t m, const int32_t *__restrict__ idx,
    double *__restrict__ y) {
    const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
        (void *)x, (short)0, (int)(m * 8 < INT_MAX ? m * 8 : INT_MAX), 0x00020000);
    const int64_t wave = ((int64_t)blockIdx.x * kProbeBlock + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t i0 = wave * 256 + 2 * lane, i1 = i0 + 128;
    if (wave * 256 + 256 <= n) {
        const probe_i2 c0 = __builtin_nontemporal_load(reinterpret_cast<const probe_i2 *>(idx + i0));
        const probe_i2 c1 = __builtin_nontemporal_load(reinterpret_cast<const probe_i2 *>(idx + i1));
        probe_d2 v0, v1;
        v0.x = probe_gather(rx, c0.x);
        v0.y = probe_gather(rx, c0.y);
        v1.x = probe_gather(rx, c1.x);
        v1.y = probe_gather(rx, c1.y);
        __builtin_nontemporal_store(v0, reinterpret_cast<probe_d2 *>(y + i0));
        __builtin_nontemporal_store(v1, reinterpret_cast<probe_d2 *>(y + i1));
    } else {
        const int64_t e[4] = {i0, i0 + 1, i1, i1 + 1};
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (e[u] < n) y[e[u]] = probe_gather(rx, idx[e[u]]);
    }
}

hipError_t gather_probe(hipStream_t s, int64_t n, const double *x, int64_t m, const int32_t *idx,
                        double *y) {
    if (n == 0) return hipSuccess;
    const int64_t waves = (n + 255) / 256;  // 256 elements per wavefront
    const int64_t per_block = kProbeBlock / kWave;
    gather_probe_kernel<<<(unsigned)((waves + per_block - 1) / per_block), kProbeBlock, 0, s>>>(
        n, x, m, idx, y);
    return hipGetLastError();
}

// ------------------------------------------------------------------ CSR -> ELL / HYB
template <typename V>
__global__ void csr_to_ell_kernel(int64_t n, int64_t ld, const int32_t *__restrict__ rp,
                                  const int32_t *__restrict__ col, const V *__restrict__ val,
                                  int64_t K, int32_t *__restrict__ ecol, V *__restrict__ eval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ld) return;
    const int64_t b = i < n ? rp[i] : 0;
    const int64_t len = i < n ? rp[i + 1] - b : 0;
    for (int64_t j = 0; j < K; ++j) {
        if (j < len) {
            ecol[j * ld + i] = col[b + j];
            eval[j * ld + i] = val[b + j];
        } else {
            ecol[j * ld + i] = -1;
            eval[j * ld + i] = V(0);
        }
    }
}

hipError_t csr_to_ell(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                      const void *val, int64_t K, int64_t ld, int32_t *ecol, void *eval) {
    if (ld == 0 || K == 0) return hipSuccess;
    if (t == vt::f64)
        csr_to_ell_kernel<double><<<grid_for(ld, 256), 256, 0, s>>>(
            n, ld, rp, col, static_cast<const double *>(val), K, ecol, static_cast<double *>(eval));
    else
        csr_to_ell_kernel<float><<<grid_for(ld, 256), 256, 0, s>>>(
            n, ld, rp, col, static_cast<const float *>(val), K, ecol, static_cast<float *>(eval));
    return hipGetLastError();
}

__global__ void tail_len_kernel(int64_t n, const int32_t *__restrict__ rp, int64_t K,
                                int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t l = rp[i + 1] - rp[i];
    len[i] = (int32_t)(l > K ? l - K : 0);
}

hipError_t tail_lengths(hipStream_t s, int64_t n, const int32_t *rp, int64_t K, int32_t *len) {
    if (n == 0) return hipSuccess;
    tail_len_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, rp, K, len);
    return hipGetLastError();
}

template <typename V>
__global__ void csr_to_tail_kernel(int64_t n, const int32_t *__restrict__ rp,
                                   const int32_t *__restrict__ col, const V *__restrict__ val,
                                   int64_t K, const int32_t *__restrict__ tail_ptr,
                                   int32_t *__restrict__ trow, int32_t *__restrict__ tcol,
                                   V *__restrict__ tval) {
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (i >= n) return;
    const int lane = threadIdx.x % kWave;
    const int64_t b = (int64_t)rp[i] + K, e = rp[i + 1];
    const int64_t o = tail_ptr[i];
    for (int64_t k = b + lane; k < e; k += kWave) {
        trow[o + (k - b)] = (int32_t)i;
        tcol[o + (k - b)] = col[k];
        tval[o + (k - b)] = val[k];
    }
}

hipError_t csr_to_tail(hipStream_t s, vt t, int64_t n, const int32_t *rp, const int32_t *col,
                       const void *val, int64_t K, const int32_t *tail_ptr, int32_t *trow,
                       int32_t *tcol, void *tval) {
    if (n == 0) return hipSuccess;
    if (t == vt::f64)
        csr_to_tail_kernel<double><<<grid_for(n, 4), 256, 0, s>>>(
            n, rp, col, static_cast<const double *>(val), K, tail_ptr, trow, tcol,
            static_cast<double *>(tval));
    else
        csr_to_tail_kernel<float><<<grid_for(n, 4), 256, 0, s>>>(
            n, rp, col, static_cast<const float *>(val), K, tail_ptr, trow, tcol,
            static_cast<float *>(tval));
    return hipGetLastError();
}

// ------------------------------------------------------------------ ELL / HYB -> CSR
__global__ void hyb_len_kernel(int64_t n, int64_t K, int64_t ld, const int32_t *__restrict__ ecol,
                               const int32_t *__restrict__ tail_ptr, int32_t *__restrict__ len) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t l = 0;
    for (int64_t j = 0; j < K; ++j) l += ecol[j * ld + i] >= 0;
    if (tail_ptr) l += tail_ptr[i + 1] - tail_ptr[i];
    len[i] = l;
}

hipError_t hyb_lengths(hipStream_t s, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                       const int32_t *tail_ptr, int32_t *len) {
    if (n == 0) return hipSuccess;
    hyb_len_kernel<<<grid_for(n, 256), 256, 0, s>>>(n, K, ld, ecol, tail_ptr, len);
    return hipGetLastError();
}

template <typename V>
__global__ void hyb_to_csr_kernel(int64_t n, int64_t K, int64_t ld, const int32_t *__restrict__ ecol,
                                  const V *__restrict__ eval, const int32_t *__restrict__ tail_ptr,
                                  const int32_t *__restrict__ tcol, const V *__restrict__ tval,
                                  const int32_t *__restrict__ rp, int32_t *__restrict__ col,
                                  V *__restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t o = rp[i];
    for (int64_t j = 0; j < K; ++j) {
        const int32_t c = ecol[j * ld + i];
        if (c < 0) break;
        col[o] = c;
        val[o] = eval[j * ld + i];
        ++o;
    }
    if (tail_ptr)
        for (int64_t k = tail_ptr[i]; k < tail_ptr[i + 1]; ++k) {
            col[o] = tcol[k];
            val[o] = tval[k];
            ++o;
        }
}

hipError_t hyb_to_csr(hipStream_t s, vt t, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                      const void *eval, const int32_t *tail_ptr, const int32_t *tcol,
                      const void *tval, const int32_t *rp, int32_t *col, void *val) {
    if (n == 0) return hipSuccess;
    if (t == vt::f64)
        hyb_to_csr_kernel<double><<<grid_for(n, 256), 256, 0, s>>>(
            n, K, ld, ecol, static_cast<const double *>(eval), tail_ptr, tcol,
            static_cast<const double *>(tval), rp, col, static_cast<double *>(val));
    else
        hyb_to_csr_kernel<float><<<grid_for(n, 256), 256, 0, s>>>(
            n, K, ld, ecol, static_cast<const float *>(eval), tail_ptr, tcol,
            static_cast<const float *>(tval), rp, col, static_cast<float *>(val));
    return hipGetLastError();
}

// ------------------------------------------------------------------ exclusive scan
// Reduce-then-scan over tiles of 1024 lengths: tile sums, a single-block scan
// of the tile sums, then each tile scans itself from its offset.
constexpr int kScanBlock = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanBlock * kScanItems;

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

__device__ inline int32_t block_excl_scan(int32_t v, int32_t *lds, int32_t *total) {
    // inclusive wave scan, then wave offsets
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const int32_t u = __shfl_up(x, off);
        if (lane >= off) x += u;
    }
    if (lane == kWave - 1) lds[w] = x;
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int j = 0; j < kScanBlock / kWave; ++j) {
        if (j < w) woff += lds[j];
        tot += lds[j];
    }
    __syncthreads();
    *total = tot;
    return woff + x - v;
}

__global__ void scan_tile_sums(int64_t n, const int32_t *__restrict__ len, int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t v = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j)
        if (base + j < n) v += len[base + j];
    int32_t tot;
    block_excl_scan(v, lds, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void scan_sums_kernel(int64_t tiles, int32_t *__restrict__ sums) {
    __shared__ int32_t lds[kScanBlock / kWave];
    int32_t carry = 0;
    for (int64_t base = 0; base < tiles; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const int32_t v = i < tiles ? sums[i] : 0;
        int32_t tot;
        const int32_t ex = block_excl_scan(v, lds, &tot);
        if (i < tiles) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[tiles] = carry;
}

__global__ void scan_tiles_kernel(int64_t n, const int32_t *__restrict__ len,
                                  const int32_t *__restrict__ sums, int32_t *__restrict__ out) {
    __shared__ int32_t lds[kScanBlock / kWave];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    int32_t v[kScanItems], t = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        v[j] = base + j < n ? len[base + j] : 0;
        t += v[j];
    }
    int32_t tot;
    int32_t o = sums[blockIdx.x] + block_excl_scan(t, lds, &tot);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        if (base + j < n) out[base + j] = o;
        o += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = sums[gridDim.x];
}

hipError_t exclusive_scan(hipStream_t s, int64_t n, const int32_t *len, int32_t *out, int32_t *tmp) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) {
        return hipMemsetAsync(out, 0, sizeof(int32_t), s);
    }
    scan_tile_sums<<<(unsigned)tiles, kScanBlock, 0, s>>>(n, len, tmp);
    scan_sums_kernel<<<1, kScanBlock, 0, s>>>(tiles, tmp);
    scan_tiles_kernel<<<(unsigned)tiles, kScanBlock, 0, s>>>(n, len, tmp, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ casts
template <typename A, typename B>
__global__ void cast_kernel(int64_t n, const A *__restrict__ a, B *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (B)a[i];
}

hipError_t cast_values(hipStream_t s, vt from, vt to, int64_t n, const void *src, void *dst) {
    if (n == 0) return hipSuccess;
    const unsigned g = grid_for(n, 256);
    if (from == vt::f64 && to == vt::f32)
        cast_kernel<double, float><<<g, 256, 0, s>>>(n, static_cast<const double *>(src), static_cast<float *>(dst));
    else if (from == vt::f32 && to == vt::f64)
        cast_kernel<float, double><<<g, 256, 0, s>>>(n, static_cast<const float *>(src), static_cast<double *>(dst));
    else
        return hipMemcpyAsync(dst, src, n * vsize(from), hipMemcpyDeviceToDevice, s);
    return hipGetLastError();
}

}  // namespace gko
