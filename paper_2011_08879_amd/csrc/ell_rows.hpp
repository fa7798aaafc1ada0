// Row sums of ELL SpMV for a thread owning two adjacent rows, shared by the
// plain SpMV and the CG step that fuses p.q into it.
#pragma once

#include "device.hpp"
#include "kernels.hpp"

namespace gko {

// Two adjacent rows per thread: ld is a multiple of 64, so slot j of rows
// 2t and 2t+1 are adjacent and each is fetched with one 16-byte (value) and
// one 8-byte (index) load; rows in [n, ld) are all padding.  Measured on the
// 27-point stencil: 148 us with one row per thread, 140 us with two.
template <typename V> struct ell_pair;
template <> struct ell_pair<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct ell_pair<float> { typedef float type __attribute__((ext_vector_type(2))); };
typedef int32_t ell_cpair __attribute__((ext_vector_type(2)));

// s0, s1 = rows i and i+1 of A x (i even, i < ld); each row stops at its
// first padding slot, the pair when both have reached theirs.
template <typename V>
__device__ inline void ell_pair_rows(int64_t K, int64_t ld, int64_t i,
                                     const int32_t *__restrict__ ecol, const V *__restrict__ eval,
                                     const V *__restrict__ x, V &s0, V &s1) {
    using V2 = typename ell_pair<V>::type;
    const ell_cpair *c = reinterpret_cast<const ell_cpair *>(ecol + i);
    const V2 *v = reinterpret_cast<const V2 *>(eval + i);
    const int64_t ld2 = ld / 2;
    s0 = V(0);
    s1 = V(0);
    for (int64_t j = 0; j < K; j += 4) {
        ell_cpair cc[4];
        V2 vv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = j + u < K;
            cc[u] = ok ? load_stream(c + (j + u) * ld2) : ell_cpair{-1, -1};
            vv[u] = ok ? load_stream(v + (j + u) * ld2) : V2{V(0), V(0)};
        }
        // Padding slots gather x[0] (the matrix has an entry, so x has one)
        // and keep the sum: no branch per gather, so all eight are in flight
        // together instead of one at a time (27-point stencil 138.6 -> 134
        // us).  The same change in the CSR subwarp, merge-path and SELL-P
        // loops measured slower there.
        V x0[4], x1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            x0[u] = x[cc[u].x >= 0 ? cc[u].x : 0];
            x1[u] = x[cc[u].y >= 0 ? cc[u].y : 0];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const V t0 = s0 + vv[u].x * x0[u], t1 = s1 + vv[u].y * x1[u];
            s0 = cc[u].x >= 0 ? t0 : s0;
            s1 = cc[u].y >= 0 ? t1 : s1;
        }
        if (cc[3].x < 0 && cc[3].y < 0) break;
    }
}

// SELL-P: one row per thread and one slice per wavefront (kSellpSlice ==
// kWave), so the slice's offset and width are wave-uniform: read with scalar
// loads, and the slot loop runs under scalar control.  Slot j of the wave's
// 64 rows is one contiguous 256-byte (index) and 512-byte (value) run, and
// the whole slice is one contiguous block.  Measured on the 27-point stencil
// (128^3): 141 us with two rows per thread (two slices per wave), 135 us
// with one and four slot loads in flight, 133 us with eight; ELL on the same
// matrix 140 us.
struct sellp_slice_of {
    int64_t base;  // first slot of the slice
    int64_t w;     // slice width
    int64_t r;     // the row's position in the slice
};

// The caller must give a wavefront 64 consecutive rows starting at a
// multiple of 64 (rows >= n of the last slice are padding).
__device__ inline sellp_slice_of sellp_slice(int64_t i, const int64_t *__restrict__ sets) {
    static_assert(kWave == kSellpSlice, "one slice per wavefront");
    const int32_t k = __builtin_amdgcn_readfirstlane((int32_t)(i / kSellpSlice));
    const int64_t base = sets[k];
    return {base, (sets[k + 1] - base) / kSellpSlice, i - (int64_t)k * kSellpSlice};
}

// Sum over the slots j0 <= j < j1 of row r of the slice starting at base,
// eight loads in flight; a row stops at its first padding slot.
template <typename V>
__device__ inline V sellp_slots_sum(int64_t base, int64_t r, int64_t j0, int64_t j1,
                                    const int32_t *__restrict__ scol,
                                    const V *__restrict__ sval, const V *__restrict__ x) {
    const int32_t *c = scol + base + r;
    const V *v = sval + base + r;
    V s = V(0);
    for (int64_t j = j0; j < j1; j += 8) {
        int32_t cc[8];
        V vv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool ok = j + u < j1;
            cc[u] = ok ? load_stream(c + (j + u) * kSellpSlice) : -1;
            vv[u] = ok ? load_stream(v + (j + u) * kSellpSlice) : V(0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (cc[u] >= 0) s += vv[u] * x[cc[u]];
        if (cc[7] < 0) break;  // the row's padding has begun
    }
    return s;
}

// Row i of A x over its whole slice.
template <typename V>
__device__ inline V sellp_row(int64_t i, const int64_t *__restrict__ sets,
                              const int32_t *__restrict__ scol, const V *__restrict__ sval,
                              const V *__restrict__ x) {
    const sellp_slice_of sl = sellp_slice(i, sets);
    return sellp_slots_sum(sl.base, sl.r, 0, sl.w, scol, sval, x);
}

}  // namespace gko
