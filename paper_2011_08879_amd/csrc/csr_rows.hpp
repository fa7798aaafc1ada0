// Row sums of CSR SpMV for a subwarp of W lanes owning U consecutive rows,
// shared by the plain SpMV and the CG step that fuses p.q into it.
#pragma once

#include "device.hpp"

namespace gko {

template <int W>
struct csr_shape {
    static constexpr int U = W >= 16 ? 4 : 8;  // rows per subwarp
};

// Rows longer than long_t are left out (their sum is 0 here): a separate
// kernel with a whole workgroup per row handles them.
template <typename V, int W, int U>
__device__ inline void csr_rows_sum(int64_t n, int64_t row0, int lane,
                                    const int32_t *__restrict__ rp,
                                    const int32_t *__restrict__ col, const V *__restrict__ val,
                                    const V *__restrict__ x, V (&s)[U], int32_t long_t) {
    int32_t b[U], e[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const bool ok = row0 + u < n;
        b[u] = ok ? rp[row0 + u] : 0;
        e[u] = ok ? rp[row0 + u + 1] : 0;
        if (e[u] - b[u] > long_t) e[u] = b[u];
    }
    int32_t c[U];
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t k = b[u] + lane;
        c[u] = k < e[u] ? load_stream(col + k) : -1;
        v[u] = k < e[u] ? load_stream(val + k) : V(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = c[u] >= 0 ? v[u] * x[c[u]] : V(0);
    // rows longer than W: the rest in strides of 4W, four loads in flight
#pragma unroll
    for (int u = 0; u < U; ++u)
        for (int32_t k = b[u] + W + lane; k < e[u]; k += 4 * W) {
            int32_t cc[4];
            V vv[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int32_t kj = k + j * W;
                cc[j] = kj < e[u] ? load_stream(col + kj) : -1;
                vv[j] = kj < e[u] ? load_stream(val + kj) : V(0);
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (cc[j] >= 0) s[u] += vv[j] * x[cc[j]];
        }
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = subwarp<W>::reduce_sum(s[u]);
}

// Row-per-thread CSR for matrices with short rows (see csr_kernel_width),
// generalised to G lanes per row: a workgroup of T threads owns T / G
// consecutive rows, stages their entries (one contiguous range) through LDS
// in chunks of C with coalesced loads, and the G lanes of a row walk its
// entries in the chunk, lane g taking entries g, g + G, ...; their partial
// sums are added by a xor butterfly.  The x gathers of neighbouring rows then
// hit neighbouring columns for banded and stencil patterns (as in ELL),
// unlike a subwarp reading its row from memory.  Returns the row sum in every
// lane of the row (0 for rows >= n).
// Measured on the 27-point stencil with G = 1: 235 us with a 32-lane subwarp
// per row, 171 us row-per-thread; eight gathers in flight in the walk
// instead of four 170 -> 167 us (banded rows of 24-40 entries 109 -> 105 us),
// sixteen no faster.
constexpr int kRowThreadBlock = 256;
constexpr int kRowThreadChunk = 2048;

template <typename V>
struct rowthread_lds {
    int32_t col[kRowThreadChunk];
    V val[kRowThreadChunk];
};

template <typename V, int G = 1>
__device__ inline V csr_rowthread_sum(int64_t n, int64_t r0, const int32_t *__restrict__ rp,
                                      const int32_t *__restrict__ col, const V *__restrict__ val,
                                      const V *__restrict__ x, rowthread_lds<V> &L) {
    constexpr int T = kRowThreadBlock, C = kRowThreadChunk, RT = T / G;
    const int g = threadIdx.x % G;
    const int64_t i = r0 + threadIdx.x / G;
    const int64_t rl = r0 + RT < n ? r0 + RT : n;
    const int32_t kb = rp[r0], ke = rp[rl];
    const int32_t b = i < n ? rp[i] : ke, e = i < n ? rp[i + 1] : ke;
    V s = V(0);
    for (int32_t c0 = kb; c0 < ke; c0 += C) {
        const int32_t cn = ke - c0 < C ? ke - c0 : C;
        int32_t cc[C / T];
        V vv[C / T];
#pragma unroll
        for (int j = 0; j < C / T; ++j) {
            const int t = threadIdx.x + j * T;
            cc[j] = t < cn ? load_stream(col + c0 + t) : 0;
            vv[j] = t < cn ? load_stream(val + c0 + t) : V(0);
        }
#pragma unroll
        for (int j = 0; j < C / T; ++j) {
            const int t = threadIdx.x + j * T;
            if (t < cn) {
                L.col[t] = cc[j];
                L.val[t] = vv[j];
            }
        }
        __syncthreads();
        const int32_t lo = (b > c0 ? b : c0) - c0;
        const int32_t hi = (e < c0 + cn ? e : c0 + cn) - c0;
        int32_t k = lo + g;
        for (; k + 7 * G < hi; k += 8 * G) {  // eight gathers in flight, summed in order
            V xs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) xs[u] = x[L.col[k + u * G]];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += L.val[k + u * G] * xs[u];
        }
        for (; k + 3 * G < hi; k += 4 * G) {
            const V x0 = x[L.col[k]], x1 = x[L.col[k + G]], x2 = x[L.col[k + 2 * G]],
                    x3 = x[L.col[k + 3 * G]];
            s += L.val[k] * x0;
            s += L.val[k + G] * x1;
            s += L.val[k + 2 * G] * x2;
            s += L.val[k + 3 * G] * x3;
        }
        for (; k < hi; k += G) s += L.val[k] * x[L.col[k]];
        __syncthreads();
    }
    if constexpr (G > 1) s = subwarp<G>::reduce_sum(s);
    return s;
}

}  // namespace gko
