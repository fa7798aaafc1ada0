// Device-side building blocks shared by the kernels: subwarp primitives for
// 64-wide wavefronts, and deterministic block / grid reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gko {

constexpr int kWave = 64;

// The dispatcher deals a grid's workgroups to the 8 XCDs round-robin
// (workgroup b to XCD b mod 8), and each XCD has its own L2.  Kernels whose
// neighbouring work items share x lines renumber their workgroups so that
// each XCD takes one contiguous range: xcd_block maps the hardware index b of
// a grid of G workgroups to that order (a bijection on [0, G)).
constexpr int kXcds = 8;

__device__ inline int64_t xcd_block(int64_t b, int64_t G) {
    const int64_t x = b % kXcds, q = G / kXcds, r = G % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Workgroup order of the row-blocked kernels (row-per-thread CSR, ELL,
// SELL-P, plain and fused with the CG product): XCD-contiguous up to
// kXcdRowsMax rows, hardware order above.  Measured on the 27-point stencil
// 128^3 (2.1M rows) ELL 133.7 -> 124 us, SELL-P 133 -> 131 us, CSR 149.5 ->
// 145.3 us; on the 7-point Poisson 256^3 (16.8M rows) ELL 280 -> 303 us,
// SELL-P 288 -> 298 us and a CG iteration on ELL 0.548 -> 0.579 ms.
constexpr int64_t kXcdRowsMax = int64_t(1) << 22;

__device__ inline int64_t row_block_order(int64_t n) {
    return n <= kXcdRowsMax ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
}

// Load of a matrix stream (values, indices) that is read once per product:
// the non-temporal hint lets the caches drop these lines first, so the
// gathered vector x keeps its place in L2.
template <typename T>
__device__ __forceinline__ T load_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// ------------------------------------------------------------------ subwarps
// Contiguous subwarps of Size lanes (a power of two <= 64) inside a wavefront,
// as in Sec. 4 (cooperative groups): lane tid belongs to the subwarp of lanes
// floor((tid % 64) / Size) * Size .. + Size - 1.  The kernels need only the
// subwarp sum; __shfl_xor with width Size stays inside that lane group.
template <int Size>
struct subwarp {
    static_assert(Size >= 1 && Size <= kWave && (Size & (Size - 1)) == 0, "power of two");

    // Xor butterfly (Sec. 5 subgroup reduction): every lane of the subwarp
    // ends with the subwarp sum; the combination order is fixed.
    template <typename T>
    __device__ static T reduce_sum(T v) {
#pragma unroll
        for (int b = 1; b < Size; b <<= 1) v += __shfl_xor(v, b, Size);
        return v;
    }
};


// Value of lane l (uniform across the wave) without an LDS round trip.
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double lane_value(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float lane_value(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// ------------------------------------------------------------------ wave scans
// Inclusive segmented sum over the 64 lanes of a wavefront whose keys do not
// decrease with the lane index: afterwards each lane holds the sum of the
// values of all lanes at or below it with the same key.  Hillis-Steele steps
// over DPP lane moves (no LDS): row shifts by 1, 2, 4, 8 inside each row of
// 16 lanes, then the broadcast of lane 15 of each row into the next row and
// of lane 31 into rows 2 and 3.  A lane without a source reads key -7, which
// no row index equals, so it adds nothing.  The combination order is fixed.
namespace dpp {
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ int move(int old, int v) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(double &p, int key) {
    const int k = move<CTRL, ROWS>(-7, key);
    const int lo = move<CTRL, ROWS>(0, __double2loint(p));
    const int hi = move<CTRL, ROWS>(0, __double2hiint(p));
    if (k == key) p += __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ void seg_step(float &p, int key) {
    const int k = move<CTRL, ROWS>(-7, key);
    const int v = move<CTRL, ROWS>(0, __float_as_int(p));
    if (k == key) p += __int_as_float(v);
}

// v plus v of the DPP source lane (0 where there is none).
template <int CTRL, int ROWS>
__device__ __forceinline__ double add_moved(double v) {
    const int lo = move<CTRL, ROWS>(0, __double2loint(v));
    const int hi = move<CTRL, ROWS>(0, __double2hiint(v));
    return v + __hiloint2double(hi, lo);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float add_moved(float v) {
    return v + __int_as_float(move<CTRL, ROWS>(0, __float_as_int(v)));
}
}  // namespace dpp

// Sum over the 64 lanes of a wavefront, the same value in every lane: the
// DPP inclusive scan (row shifts, then the broadcasts of lanes 15 and 31)
// leaves the total in lane 63, which readlane broadcasts.  DPP moves are
// VALU operations, so this chain is much shorter than an LDS-crossbar
// butterfly; the summation order is fixed.
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
    v = dpp::add_moved<dpp::kRowShr1, 0xf>(v);
    v = dpp::add_moved<dpp::kRowShr2, 0xf>(v);
    v = dpp::add_moved<dpp::kRowShr4, 0xf>(v);
    v = dpp::add_moved<dpp::kRowShr8, 0xf>(v);
    v = dpp::add_moved<dpp::kRowBcast15, 0xa>(v);
    v = dpp::add_moved<dpp::kRowBcast31, 0xc>(v);
    return lane_value(v, kWave - 1);
}

template <typename T>
__device__ __forceinline__ void wave_segmented_scan(T &p, int key) {
    dpp::seg_step<dpp::kRowShr1, 0xf>(p, key);
    dpp::seg_step<dpp::kRowShr2, 0xf>(p, key);
    dpp::seg_step<dpp::kRowShr4, 0xf>(p, key);
    dpp::seg_step<dpp::kRowShr8, 0xf>(p, key);
    dpp::seg_step<dpp::kRowBcast15, 0xa>(p, key);  // rows 1 and 3
    dpp::seg_step<dpp::kRowBcast31, 0xc>(p, key);  // rows 2 and 3
}


__device__ inline int popcnt(uint32_t m) { return __popc(m); }
__device__ inline int popcnt(uint64_t m) { return __popcll(m); }

// ------------------------------------------------------------------ block reduction
// Sum over a block of BLOCK threads (multiple of 64) with a fixed tree: wave
// totals (wave_total), then the per-wave sums combined by wave 0.  Every
// thread of the block must call it.  Result valid in
// thread 0.  `lds` needs BLOCK/64 slots.
template <int BLOCK, typename T>
__device__ inline T block_sum(T v, T *lds) {
    static_assert(BLOCK % kWave == 0, "block of whole waves");
    constexpr int NW = BLOCK / kWave;
    v = wave_total(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) lds[w] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x < kWave) {
        s = (threadIdx.x < NW) ? lds[threadIdx.x] : T(0);
        s = wave_total(s);
    }
    __syncthreads();
    return s;
}

// ------------------------------------------------------------------ grid reduction
// Deterministic grid-wide sums of NV values per thread, finished once by an
// operation `op` on the totals (thread 0).  Every block first forms its NV
// block sums with a fixed tree and stores them as partials[j * grid + block].
// The partials are then summed in block order with a fixed tree, in one of
// two ways chosen by the grid size alone, so results never depend on block
// scheduling:
//  * small grids: the block that takes the last ticket sums the partials and
//    applies op in the same launch (a release fence per block, an acquire
//    fence in the last one);
//  * large grids: a one-workgroup finalize kernel launched right after sums
//    them and applies op.  On MI355X a per-block release fence writes back
//    the XCD's dirty L2 lines, which for a few thousand blocks that store
//    vectors costs more than the extra launch (measured: 2048 blocks of an
//    x+y kernel with its z.z reduction, 164 us with fences against 87 us
//    with the finalize kernel).
constexpr int kTicketMaxBlocks = 64;

struct red_args {
    double *partials;  // NV * grid doubles
    unsigned *ticket;  // zeroed; null: the partials go to a finalize kernel
};

__device__ inline double load_coherent(const double *p) {
    uint64_t bits = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    return __longlong_as_double(static_cast<long long>(bits));
}

// Sum of partials[j * g + b] over b < g in a fixed order (strided per
// thread, four loads in flight, then the block tree); valid in thread 0.
template <int BLOCK, bool COHERENT>
__device__ inline double sum_partials(const double *pj, unsigned g, double *lds) {
    double s = 0.0;
    unsigned b = threadIdx.x;
    for (; b + 3 * BLOCK < g; b += 4 * BLOCK) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = COHERENT ? load_coherent(pj + b + u * BLOCK) : pj[b + u * BLOCK];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += t[u];
    }
    for (; b < g; b += BLOCK) s += COHERENT ? load_coherent(pj + b) : pj[b];
    return block_sum<BLOCK>(s, lds);
}

template <int BLOCK, int NV, typename Op>
__device__ inline void grid_sum_apply(const double (&v)[NV], const red_args &ra, const Op &op) {
    __shared__ double lds[BLOCK / kWave];
    __shared__ bool am_last;
    double bs[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) bs[j] = block_sum<BLOCK>(v[j], lds);
    if (!ra.ticket) {
        if (threadIdx.x == 0)
#pragma unroll
            for (int j = 0; j < NV; ++j) ra.partials[(size_t)j * gridDim.x + blockIdx.x] = bs[j];
        return;
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int j = 0; j < NV; ++j) ra.partials[(size_t)j * gridDim.x + blockIdx.x] = bs[j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        am_last = atomicAdd(ra.ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!am_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double out[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j)
        out[j] = sum_partials<BLOCK, true>(ra.partials + (size_t)j * gridDim.x, gridDim.x, lds);
    if (threadIdx.x == 0) {
        __hip_atomic_store(ra.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        op(out);
    }
}

constexpr int kFinalizeBlock = 1024;

// The finalize kernel of a large grid: g blocks stored their partials.
// op.skip() repeats the early-exit test of the kernel that produced them.
// One workgroup reads all NV * g partials, 32 loads in flight per thread
// over the NV sums (the partials come from every XCD, so each round costs a
// memory latency): for g = 65536 two sums took 16 us with four loads in
// flight per sum in turn.
template <int NV, typename Op>
__global__ __launch_bounds__(kFinalizeBlock) void finalize_kernel(unsigned g, const double *partials,
                                                                  Op op) {
    constexpr int U = NV >= 32 ? 1 : 32 / NV;
    __shared__ double lds[kFinalizeBlock / kWave];
    if (op.skip()) return;
    double s[NV] = {};
    unsigned b = threadIdx.x;
    for (; b + (U - 1) * kFinalizeBlock < g; b += U * kFinalizeBlock) {
        double t[NV][U];
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) t[j][u] = partials[(size_t)j * g + b + u * kFinalizeBlock];
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int u = 0; u < U; ++u) s[j] += t[j][u];
    }
    for (; b < g; b += kFinalizeBlock)
#pragma unroll
        for (int j = 0; j < NV; ++j) s[j] += partials[(size_t)j * g + b];
    double out[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) out[j] = block_sum<kFinalizeBlock>(s[j], lds);
    if (threadIdx.x == 0) op(out);
}

// Host side: the reduction mode for a grid of g blocks, and the finalize
// launch that follows the reducing kernel when the grid is large.
inline red_args red_for(int g, double *partials, unsigned *ticket) {
    return red_args{partials, g <= kTicketMaxBlocks ? ticket : nullptr};
}

template <int NV, typename Op>
inline hipError_t red_finish(hipStream_t s, int g, const red_args &ra, const Op &op) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || ra.ticket) return e;
    finalize_kernel<NV, Op><<<1, kFinalizeBlock, 0, s>>>((unsigned)g, ra.partials, op);
    return hipGetLastError();
}

}  // namespace gko
