// SpMV for COO (row-major sorted triplets) and the y <- beta y helper.
//
// Sec. 6.1 prices COO at 16 bytes per entry (value, row and column index);
// the paper's solvers use it (Sec. 6.2).  Each wavefront owns an equal chunk
// of entries, so the work split ignores row lengths.  Within a chunk the
// wave takes 64 entries at a time with coalesced loads and combines products
// of equal row by a segmented inclusive scan over the lanes, done with DPP
// lane moves (keys are sorted, so a partner lane with the same key means
// every lane between has it); the values the next batch needs from lane 63
// are read with readlane, so a batch touches no LDS.
// Rows wholly inside a chunk are written directly; a row cut by a chunk
// boundary leaves partials (head of the next chunk, tail of this one) that a
// second kernel adds in ascending chunk order.  Results are bitwise
// repeatable.
#include <climits>

#include "device.hpp"
#include "kernels.hpp"

namespace gko {

constexpr int kCooBlock = 256;
constexpr int kCooBatches = 16;                  // batches of 64 entries per wave
constexpr int kCooChunk = kWave * kCooBatches;   // entries per wave
constexpr int kCooHoist = 4;                     // batches whose loads are issued together
// DPP controls shifting the whole wavefront by one lane.  With them and the
// next group's first row loaded together with the group's own loads, the
// neighbour-row tests need neither LDS permutes nor a load of their own:
// 27-point stencil 222 -> 214 us.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;

int64_t coo_chunks(int64_t nnz) { return (nnz + kCooChunk - 1) / kCooChunk; }

template <typename V>
__device__ inline V combine(V alpha, V beta, V s, V y_old, bool accumulate) {
    if (accumulate) return y_old + alpha * s;
    return (beta == V(0)) ? alpha * s : alpha * s + beta * y_old;
}

template <typename V, bool ACC>
__global__ __launch_bounds__(kCooBlock) void spmv_coo_kernel(
    int64_t n, int64_t nnz, const int32_t *__restrict__ row, const int32_t *__restrict__ col,
    const V *__restrict__ val, const V *__restrict__ x, V alpha, V beta, V *__restrict__ y,
    V *__restrict__ head, V *__restrict__ tail) {
    // each XCD streams one contiguous share of the chunks, so x lines shared
    // by neighbouring chunks are fetched into one L2 only
    const int64_t c = xcd_block(blockIdx.x, gridDim.x) * (kCooBlock / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    const int64_t cb = c * kCooChunk;
    if (cb >= nnz) return;
    const int64_t ce = cb + kCooChunk < nnz ? cb + kCooChunk : nnz;
    const int32_t first_row = row[cb], last_row = row[ce - 1];
    const bool open_start = cb > 0 && row[cb - 1] == first_row;
    const bool open_end = ce < nnz && row[ce] == last_row;
    int32_t prev_row = cb > 0 ? row[cb - 1] : -1;
    int32_t carry_row = -1;
    V carry = V(0);

    for (int64_t base = cb; base < ce; base += kWave * kCooHoist) {
        // loads of kCooHoist batches first, then their x gathers
        int32_t rb[kCooHoist], cb_[kCooHoist];
        V vb[kCooHoist], pb[kCooHoist], yb[kCooHoist];
        // first row of the next group (wave-uniform address: a scalar load)
        const int64_t nxt = base + kWave * kCooHoist;
        const int32_t next_group_row = nxt < ce ? row[nxt] : -2;
        // A whole group (uniform) loads without bounds tests: the tested loads
        // compile to one exec-masked block each (27-point stencil 219 -> 202 us).
        if (nxt <= ce) {
#pragma unroll
            for (int j = 0; j < kCooHoist; ++j) {
                const int64_t k = base + j * kWave + lane;
                rb[j] = load_stream(row + k);
                cb_[j] = load_stream(col + k);
                vb[j] = load_stream(val + k);
            }
#pragma unroll
            for (int j = 0; j < kCooHoist; ++j) pb[j] = vb[j] * x[cb_[j]];
            // Accumulating (the COO part of HYB): the old y of every lane's
            // row, read with the group's loads.  Read where a segment ends, it
            // sat in a branch that waited for it once per batch (lognormal
            // HYB 192 -> 187 us).  Only this wave writes these rows.
            if constexpr (ACC) {
#pragma unroll
                for (int j = 0; j < kCooHoist; ++j) yb[j] = y[rb[j]];
            }
        } else {
#pragma unroll
            for (int j = 0; j < kCooHoist; ++j) {
                const int64_t k = base + j * kWave + lane;
                const bool valid = k < ce;
                rb[j] = valid ? load_stream(row + k) : INT_MAX;
                cb_[j] = valid ? load_stream(col + k) : -1;
                vb[j] = valid ? load_stream(val + k) : V(0);
            }
#pragma unroll
            for (int j = 0; j < kCooHoist; ++j) pb[j] = cb_[j] >= 0 ? vb[j] * x[cb_[j]] : V(0);
            if constexpr (ACC) {
#pragma unroll
                for (int j = 0; j < kCooHoist; ++j) yb[j] = cb_[j] >= 0 ? y[rb[j]] : V(0);
            }
        }

#pragma unroll
        for (int j = 0; j < kCooHoist; ++j) {
            const int64_t bbase = base + j * kWave;
            if (bbase >= ce) break;  // uniform across the wave
            const int64_t k = bbase + lane;
            const bool valid = k < ce;
            const int32_t r = rb[j];
            V p = pb[j];

            if (!ACC) {
                // rows without entries between the previous entry and this one
                // the previous lane's row (DPP wavefront shift right; lane 0 gets prev_row)
                int32_t rprev = __builtin_amdgcn_update_dpp(prev_row, r, kDppWaveShr1, 0xf, 0xf, false);
                if (valid)
                    for (int32_t e = rprev + 1; e < r; ++e) y[e] = combine(alpha, beta, V(0), y[e], false);
            }

            wave_segmented_scan(p, r);
            if (r == carry_row) p += carry;

            // A lane ends its row's segment when the next entry (in this batch,
            // or the first of the next batch of this chunk) has another row.
            const bool more = bbase + kWave < ce;
            const int32_t next_first = (j + 1 < kCooHoist) ? lane_value(rb[(j + 1) % kCooHoist], 0)
                                                           : next_group_row;
            // the next lane's row (DPP wavefront shift left; lane 63 gets next_first)
            int32_t rn = __builtin_amdgcn_update_dpp(more ? next_first : -2, r, kDppWaveShl1, 0xf, 0xf,
                                                     false);
            const bool seg_end = valid && rn != r;
            if (seg_end) {
                if (r == first_row && open_start) head[c] = p;
                else if (r == last_row && open_end) tail[c] = p;
                else y[r] = combine(alpha, beta, p, ACC ? yb[j] : beta != V(0) ? y[r] : V(0), ACC);
            }
            // a row still open at the batch end carries into the next batch
            carry_row = lane_value(seg_end ? -1 : r, kWave - 1);
            carry = lane_value(p, kWave - 1);
            prev_row = lane_value(r, kWave - 1);
        }
    }
    if (!ACC && ce == nnz)  // rows after the last entry
        for (int64_t e = (int64_t)last_row + 1 + lane; e < n; e += kWave)
            y[e] = combine(alpha, beta, V(0), y[e], false);
}

template <typename V, bool ACC>
__global__ void coo_fixup_kernel(int64_t nnz, const int32_t *__restrict__ row,
                                 const V *__restrict__ head, const V *__restrict__ tail, V alpha,
                                 V beta, V *__restrict__ y) {
    const int64_t chunks = (nnz + kCooChunk - 1) / kCooChunk;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= chunks) return;
    const int64_t cb = c * kCooChunk;
    const int64_t ce = cb + kCooChunk < nnz ? cb + kCooChunk : nnz;
    const int32_t r = row[ce - 1];
    const bool open_end = ce < nnz && row[ce] == r;
    if (!open_end) return;
    const bool through = cb > 0 && row[cb - 1] == r && row[cb] == r;
    if (through) return;  // the row began in an earlier chunk
    V s = tail[c];
    for (int64_t d = c + 1; d < chunks; ++d) {
        s += head[d];
        const int64_t db = d * kCooChunk;
        const int64_t de = db + kCooChunk < nnz ? db + kCooChunk : nnz;
        if (!(row[de - 1] == r && de < nnz && row[de] == r)) break;
    }
    y[r] = combine(alpha, beta, s, ACC || beta != V(0) ? y[r] : V(0), ACC);
}

template <typename V>
__global__ void scale_kernel(int64_t n, V beta, V *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (beta == V(0)) ? V(0) : beta * y[i];
}

template <typename V>
static hipError_t launch_scale(hipStream_t s, int64_t n, double beta, void *y) {
    if (n == 0) return hipSuccess;
    scale_kernel<V><<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(n, (V)beta,
                                                                          static_cast<V *>(y));
    return hipGetLastError();
}

hipError_t scale(hipStream_t s, vt t, int64_t n, double beta, void *y) {
    return t == vt::f64 ? launch_scale<double>(s, n, beta, y) : launch_scale<float>(s, n, beta, y);
}

template <typename V, bool ACC>
static hipError_t launch_coo(hipStream_t s, int64_t n, int64_t nnz, const int32_t *row,
                             const int32_t *col, const void *val, const void *x, double alpha,
                             double beta, void *y, void *head, void *tail) {
    const int64_t chunks = coo_chunks(nnz);
    const int64_t grid = (chunks + (kCooBlock / kWave) - 1) / (kCooBlock / kWave);
    spmv_coo_kernel<V, ACC><<<dim3((unsigned)grid), dim3(kCooBlock), 0, s>>>(
        n, nnz, row, col, static_cast<const V *>(val), static_cast<const V *>(x), (V)alpha,
        (V)beta, static_cast<V *>(y), static_cast<V *>(head), static_cast<V *>(tail));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    coo_fixup_kernel<V, ACC><<<dim3((unsigned)((chunks + 255) / 256)), dim3(256), 0, s>>>(
        nnz, row, static_cast<const V *>(head), static_cast<const V *>(tail), (V)alpha, (V)beta,
        static_cast<V *>(y));
    return hipGetLastError();
}

hipError_t spmv_coo(hipStream_t s, vt t, int64_t n, int64_t nnz, const int32_t *row,
                    const int32_t *col, const void *val, const void *x, double alpha, double beta,
                    void *y, bool accumulate, void *head, void *tail) {
    if (n == 0) return hipSuccess;
    if (nnz == 0) return accumulate ? hipSuccess : scale(s, t, n, beta, y);
    if (t == vt::f64)
        return accumulate ? launch_coo<double, true>(s, n, nnz, row, col, val, x, alpha, beta, y, head, tail)
                          : launch_coo<double, false>(s, n, nnz, row, col, val, x, alpha, beta, y, head, tail);
    return accumulate ? launch_coo<float, true>(s, n, nnz, row, col, val, x, alpha, beta, y, head, tail)
                      : launch_coo<float, false>(s, n, nnz, row, col, val, x, alpha, beta, y, head, tail);
}

}  // namespace gko
