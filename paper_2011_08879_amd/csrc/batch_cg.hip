// Batched CG: thousands of small independent SPD systems in one persistent
// launch.  Every workgroup loops: take the next system from an atomic work
// queue (systems ordered by decreasing rows, then nonzeros, so the longest
// jobs start first), solve it to its own tolerance with the iteration
// vectors in LDS, write x, the iteration count and the true residual, and
// take the next.  In the wavefront mode, once the queue reaches systems of
// at most kWaveRows rows, each wavefront of the workgroup takes systems of
// its own (block / 64 systems per workgroup at a time).
// The matrix of a system (a few tens of KB) is read from global memory and
// stays in the L1/L2 caches across its iterations; each workgroup exits once
// the queue runs dry, so every wave reaches the end.
//
// FP64 batches run plain CG (Hestenes-Stiefel).  FP32 batches store the
// matrix in FP32 and run FP32 CG iterations inside FP64 iterative
// refinement: the residual b - A x, its norm and the update x += |r| d are
// FP64, each inner solve asks for tau_k = max(1e-5, tol |b| / (2 |r_k|)).
#include <cmath>

#include "batch_kernels.hpp"
#include "device.hpp"

namespace gko {

// Sum over the workgroup with a fixed tree; every thread gets the total.
template <int T>
__device__ inline double wg_sum(double v, double *red) {
    v = wave_total(v);
    if constexpr (T == kWave) {
        return v;
    } else {
        constexpr int NW = T / kWave;
        const int w = threadIdx.x / kWave;
        if ((threadIdx.x % kWave) == 0) red[w] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NW; ++j) s += red[j];
        __syncthreads();
        return s;
    }
}

// The same with one barrier: no thread may write `red` again before every
// thread has passed a later barrier (the CG loop alternates two buffers).
template <int T>
__device__ inline double wg_sum_once(double v, double *red) {
    v = wave_total(v);
    if constexpr (T == kWave) {
        return v;
    } else {
        constexpr int NW = T / kWave;
        const int w = threadIdx.x / kWave;
        if ((threadIdx.x % kWave) == 0) red[w] = v;
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NW; ++j) s += red[j];
        return s;
    }
}

template <int T>
__device__ inline void wg_sync() {
    __syncthreads();
}

// Orders this wavefront's LDS accesses (its lanes exchange data through
// LDS; a wavefront's LDS operations complete in order).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Who solves one system: the workgroup (T threads; sums by fixed trees
// through LDS; workgroup barriers) or one wavefront (sums by DPP; no
// barrier).
template <int T>
struct wg_team {
    static constexpr int kSize = T;
    static constexpr bool kIsWave = false;
    double (*red2)[T / kWave];  // the CG loop's two alternating reduction buffers
    double *red;
    __device__ int tid() const { return threadIdx.x; }
    __device__ double sum_once(double v, int slot) const { return wg_sum_once<T>(v, red2[slot]); }
    __device__ double sum(double v) const { return wg_sum<T>(v, red); }
    __device__ void sync() const { __syncthreads(); }
};

struct wave_team {
    static constexpr int kSize = kWave;
    static constexpr bool kIsWave = true;
    __device__ int tid() const { return threadIdx.x % kWave; }
    __device__ double sum_once(double v, int) const { return wave_total(v); }
    __device__ double sum(double v) const { return wave_total(v); }
    __device__ void sync() const { wave_sync(); }
};

struct sys_view {
    int32_t m;
    const int32_t *rp;
    const int32_t *col;
    int64_t row0;
};

// q = A p over this thread's rows (rows tid, tid+T, ...), returns sum of p_i q_i.
template <typename VA, typename VV, int T>
__device__ inline double spmv_rows(const sys_view &S, const VA *__restrict__ val, const VV *p,
                                   VV *q) {
    double pq = 0.0;
    for (int i = threadIdx.x; i < S.m; i += T) {
        VV s = VV(0);
        for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) s += (VV)val[k] * p[S.col[k]];
        q[i] = s;
        pq += (double)p[i] * (double)s;
    }
    return pq;
}

// A system's rows held in registers for its whole solve: a thread's rows
// tid + j T (j < R) with up to L entries each, unused slots with value 0 and
// the row itself as column (an in-range read that adds nothing).  Systems
// with more rows or longer rows are read from memory every iteration.
template <int T>
constexpr int batch_cache_rows() { return 1024 / T < 4 ? 1024 / T : 4; }
template <typename VA, int T>
struct sys_regs {
    static constexpr int R = batch_cache_rows<T>(), L = kBatchCacheLen;
    int32_t c[R][L];
    VA v[R][L];

    // Loads this thread's rows; true (uniform) when every row of the system fits.
    template <typename Team>
    __device__ bool load(const sys_view &S, const VA *__restrict__ val, const Team &team) {
        static_assert(Team::kSize == T, "rows of one team");
        bool fits = S.m <= R * T;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int i = team.tid() + j * T;
            const int32_t b = i < S.m ? S.rp[i] : 0, e = i < S.m ? S.rp[i + 1] : 0;
            if (e - b > L) fits = false;
#pragma unroll
            for (int q = 0; q < L; ++q) {
                const bool ok = b + q < e;
                c[j][q] = ok ? S.col[b + q] : (i < S.m ? i : 0);
                v[j][q] = ok ? val[b + q] : VA(0);
            }
        }
        return team.sum(fits ? 0.0 : 1.0) == 0.0;
    }
};

// Plain CG on A x = rhs from x = 0, vectors x, r, p, q in LDS (type VV),
// dots in FP64, q = A p from the system's rows in memory.  Returns
// iterations; *flag = 1 not SPD, 2 breakdown.
// Three barriers per iteration: p.q into red2[0], r.r into red2[1], and the
// one after the p update.  A buffer's next write comes two barriers after
// its last read; the caller passes a barrier before any other use of red2.
template <typename VA, typename VV, int T>
__device__ inline int cg_in_lds(const sys_view &S, const VA *__restrict__ val, VV *x, VV *r,
                                VV *p, VV *q, double rhs_norm2, double stop2, int maxit,
                                double (*red2)[T / kWave], int *flag) {
    double rr = rhs_norm2;
    int it = 0;
    *flag = 0;
    while (it < maxit && rr > stop2) {
        const double pq = wg_sum_once<T>(spmv_rows<VA, VV, T>(S, val, p, q), red2[0]);
        ++it;
        if (!(pq > 0.0)) {
            *flag = std::isnan(pq) ? 2 : 1;
            break;
        }
        const double alpha = rr / pq;
        double loc = 0.0;
        for (int i = threadIdx.x; i < S.m; i += T) {
            x[i] = (VV)((double)x[i] + alpha * (double)p[i]);
            const VV ri = (VV)((double)r[i] - alpha * (double)q[i]);
            r[i] = ri;
            loc += (double)ri * (double)ri;
        }
        const double rr_new = wg_sum_once<T>(loc, red2[1]);
        if (!std::isfinite(rr_new)) {
            *flag = 2;
            break;
        }
        const double beta = rr_new / rr;
        rr = rr_new;
        for (int i = threadIdx.x; i < S.m; i += T) p[i] = (VV)((double)r[i] + beta * (double)p[i]);
        wg_sync<T>();
    }
    return it;
}

// The same CG when the system's rows are held in registers: a thread's own
// entries of x, r, p and q (rows tid + j T) stay in registers too, and only p
// goes through LDS, for the neighbours' gathers.  Per row and iteration the
// LDS then serves the row's p gathers and one p store, against those plus
// eight vector reads and writes with every vector in LDS.  x comes in and
// goes out in LDS (own rows); r starts from rhs (own rows, LDS) and p = r.
// LEAN: x starts at zero in registers and rhs is read from global memory, so
// p is the only vector in LDS; on return x is left in p's place.
template <typename VA, typename VV, typename Team, bool LEAN = false>
__device__ inline int cg_cached(int32_t m, const sys_regs<VA, Team::kSize> &regs, VV *x,
                                const VV *rhs, VV *p, double rhs_norm2, double stop2, int maxit,
                                const Team &team, int *flag) {
    constexpr int T = Team::kSize;
    constexpr int R = sys_regs<VA, T>::R, L = sys_regs<VA, T>::L;
    VV xr[R], rr_[R], pr[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = team.tid() + j * T;
        xr[j] = (LEAN || i >= m) ? VV(0) : x[i];
        rr_[j] = i < m ? rhs[i] : VV(0);
        pr[j] = rr_[j];
        if (i < m) p[i] = pr[j];
    }
    team.sync();
    // FP32 iterations skip, by a scalar branch, a row block j of this
    // wavefront (rows from its first lane's thread + j T) that lies wholly
    // past the last row: its x, r, p and q stay 0.  Systems of 32..1024 rows
    // leave about half of the R T row slots of a 256-thread workgroup empty.
    // 10,000 such systems: FP32 storage 0.60 -> 0.57 ms; FP64 0.49 -> 0.54 ms,
    // so FP64 keeps the branch-free loop (its 20 LDS gathers are issued
    // together; the branches split them into four waits).
    constexpr bool kSkip = sizeof(VV) == 4;
    const int wave_row0 = __builtin_amdgcn_readfirstlane(team.tid()) & ~(kWave - 1);
    double rr = rhs_norm2;
    int it = 0;
    *flag = 0;
    while (it < maxit && rr > stop2) {
        VV qr[R];
        double pq_local = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            qr[j] = VV(0);
            if (kSkip && wave_row0 + j * T >= m) continue;
            VV s = VV(0);
#pragma unroll
            for (int k = 0; k < L; ++k) s += (VV)regs.v[j][k] * p[regs.c[j][k]];
            qr[j] = s;
            // rows >= m hold p = 0 in registers, so they add nothing
            pq_local += (double)pr[j] * (double)s;
        }
        const double pq = team.sum_once(pq_local, 0);
        ++it;
        if (!(pq > 0.0)) {
            *flag = std::isnan(pq) ? 2 : 1;
            break;
        }
        const double alpha = rr / pq;
        double loc = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (kSkip && wave_row0 + j * T >= m) continue;
            xr[j] = (VV)((double)xr[j] + alpha * (double)pr[j]);
            rr_[j] = (VV)((double)rr_[j] - alpha * (double)qr[j]);
            loc += (double)rr_[j] * (double)rr_[j];
        }
        const double rr_new = team.sum_once(loc, 1);
        if (!std::isfinite(rr_new)) {
            *flag = 2;
            break;
        }
        const double beta = rr_new / rr;
        rr = rr_new;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            if (kSkip && wave_row0 + j * T >= m) continue;
            const int i = team.tid() + j * T;
            pr[j] = (VV)((double)rr_[j] + beta * (double)pr[j]);
            if (i < m) p[i] = pr[j];
        }
        team.sync();
    }
    // every read of p ended before the last barrier the loop passed
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int i = team.tid() + j * T;
        if (i < m) (LEAN ? p : x)[i] = xr[j];
    }
    return it;
}

// FP32 storage: FP32 CG iterations inside FP64 iterative refinement, with
// x and r (FP64) and the inner d, r, p, q (FP32) in LDS from x64 on (32 bytes
// per row).  Returns the inner iterations; x is left in x64.
template <typename VA, typename Team>
__device__ inline int solve_refined(const sys_view &S, const VA *__restrict__ A,
                                    const double *__restrict__ bs, double bnorm,
                                    const sys_regs<VA, Team::kSize> &regs, bool cached, double tol,
                                    int maxit, double *x64, const Team &team, int *flag) {
    constexpr int T = Team::kSize;
    double *r64 = x64 + S.m;
    float *d = reinterpret_cast<float *>(r64 + S.m);
    float *r = d + S.m, *p = r + S.m, *q = p + S.m;
    for (int i = team.tid(); i < S.m; i += T) {
        x64[i] = 0.0;
        r64[i] = bs[i];
    }
    team.sync();
    int its = 0;
    *flag = 0;
    double rn = bnorm, prev = INFINITY;
    for (int outer = 0; outer < 20; ++outer) {
        if (!(rn > tol * bnorm) || !(rn <= 0.5 * prev)) break;
        prev = rn;
        double tau = 0.5 * (tol * bnorm / rn);
        if (tau < 1e-5) tau = 1e-5;
        double rt2 = 0.0;
        for (int i = team.tid(); i < S.m; i += T) {
            const float ri = (float)(r64[i] / rn);
            d[i] = 0.0f;
            r[i] = ri;
            p[i] = ri;
            rt2 += (double)ri * (double)ri;
        }
        rt2 = team.sum(rt2);
        if constexpr (Team::kIsWave) {
            // a wavefront only takes systems whose rows are all cached
            its += cg_cached<VA, float, Team>(S.m, regs, d, r, p, rt2, tau * tau * rt2, maxit - its,
                                              team, flag);
        } else {
            its += cached ? cg_cached<VA, float, Team>(S.m, regs, d, r, p, rt2, tau * tau * rt2,
                                                       maxit - its, team, flag)
                          : cg_in_lds<VA, float, T>(S, A, d, r, p, q, rt2, tau * tau * rt2,
                                                    maxit - its, team.red2, flag);
        }
        if (*flag) break;
        // x += |r| d, then the FP64 residual b - A x
        for (int i = team.tid(); i < S.m; i += T) x64[i] = x64[i] + rn * (double)d[i];
        team.sync();
        double loc = 0.0;
        for (int i = team.tid(); i < S.m; i += T) {
            double s = 0.0;
            for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) s += (double)A[k] * x64[S.col[k]];
            const double ri = bs[i] - s;
            r64[i] = ri;
            loc += ri * ri;
        }
        rn = sqrt(team.sum(loc));
        if (its >= maxit) break;
    }
    return its;
}

// A view of system sid of the batch.
__device__ inline sys_view system_view(int32_t sid, const int64_t *__restrict__ row_off,
                                       const int64_t *__restrict__ nnz_off,
                                       const int32_t *__restrict__ rp_local,
                                       const int32_t *__restrict__ col) {
    sys_view S;
    S.row0 = row_off[sid];
    S.m = (int32_t)(row_off[sid + 1] - S.row0);
    S.rp = rp_local + S.row0 + sid;
    S.col = col + nnz_off[sid];
    return S;
}

// True residual of the final x (in LDS, xs) in FP64 from the system's rows in
// memory, x to global memory, and the system's outputs (first thread of the
// team).
template <typename VA, typename Team>
__device__ inline void finish_system(int32_t sid, const sys_view &S, const VA *__restrict__ A,
                                     const double *__restrict__ bs, const double *xs,
                                     double *__restrict__ xout, double bnorm, double tol, int its,
                                     int flag, int32_t *__restrict__ iters,
                                     double *__restrict__ relres, int *status, const Team &team) {
    double loc = 0.0;
    for (int i = team.tid(); i < S.m; i += Team::kSize) {
        double s = 0.0;
        for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k) s += (double)A[k] * xs[S.col[k]];
        const double ri = bs[i] - s;
        loc += ri * ri;
        xout[S.row0 + i] = xs[i];
    }
    const double tr = sqrt(team.sum(loc));
    if (team.tid() == 0) {
        iters[sid] = its;
        relres[sid] = bnorm > 0.0 ? tr / bnorm : 0.0;
        const int st = flag == 1 ? kBatchNotSpd
                     : flag == 2 ? kBatchBreakdown
                     : (bnorm > 0.0 && !(tr <= tol * bnorm)) ? kBatchNotConverged : 0;
        if (st) atomicMax(status, st);
    }
}

// The next queue position for one wavefront (lane 0 takes it).
__device__ inline unsigned pop_wave(unsigned *counter) {
    unsigned q = 0;
    if (threadIdx.x % kWave == 0) q = atomicAdd(counter, 1u);
    return (unsigned)__builtin_amdgcn_readfirstlane((int)q);
}

// One system solved by one wavefront, its rows in registers.  FP64 (LEAN):
// p, then x, in this wavefront's LDS slice pw (kWaveRows doubles); FP32
// storage: the refinement's vectors in pw (4 kWaveRows doubles).
template <typename VA>
__device__ inline void solve_on_wave(int32_t sid, const int64_t *__restrict__ row_off,
                                     const int64_t *__restrict__ nnz_off,
                                     const int32_t *__restrict__ rp_local,
                                     const int32_t *__restrict__ col, const VA *__restrict__ val,
                                     const double *__restrict__ b, double *__restrict__ xout,
                                     double tol, int32_t maxit, int32_t *__restrict__ iters,
                                     double *__restrict__ relres, int *status, double *pw) {
    const wave_team team;
    const sys_view S = system_view(sid, row_off, nnz_off, rp_local, col);
    const VA *A = val + nnz_off[sid];
    const double *bs = b + S.row0;
    double bb = 0.0;
    for (int i = team.tid(); i < S.m; i += kWave) bb += bs[i] * bs[i];
    bb = team.sum(bb);
    const double bnorm = sqrt(bb);
    sys_regs<VA, kWave> regs;
    int its = 0, flag = 2;
    if (regs.load(S, A, team)) {
        if constexpr (sizeof(VA) == 8)
            its = cg_cached<VA, double, wave_team, true>(S.m, regs, nullptr, bs, pw, bb,
                                                         tol * tol * bb, maxit, team, &flag);
        else
            its = solve_refined(S, A, bs, bnorm, regs, true, tol, maxit, pw, team, &flag);
    }
    team.sync();
    finish_system(sid, S, A, bs, pw, xout, bnorm, tol, its, flag, iters, relres, status, team);
    team.sync();  // pw is rewritten by the next system
}

// LEAN (FP64 batches whose every system fits the register cache): only the
// direction p, later x, is in LDS, m doubles per workgroup instead of 4m.
// WAVES (FP64 with LEAN, or FP32 storage whose rows all fit the register
// cache): systems of at most kWaveRows rows one per wavefront.
template <typename VA, int T, bool LEAN, bool WAVES>
__global__ __launch_bounds__(T, (WAVES && T == 256) ? 4 : 1) void batch_cg_kernel(
    int64_t nsys, const int64_t *__restrict__ row_off, const int64_t *__restrict__ nnz_off,
    const int32_t *__restrict__ rp_local, const int32_t *__restrict__ col,
    const VA *__restrict__ val, const int32_t *__restrict__ order, unsigned *counter,
    const double *__restrict__ b, double *__restrict__ xout, double tol, int32_t maxit,
    int32_t *__restrict__ iters, double *__restrict__ relres, int *status) {
    extern __shared__ double lds[];
    __shared__ double red[T / kWave];
    __shared__ double red2[2][T / kWave];
    __shared__ unsigned s_next;
    constexpr bool kRefine = sizeof(VA) == 4;  // FP32 storage: FP32 CG inside FP64 refinement
    static_assert(!WAVES || LEAN != kRefine, "the wavefront mode runs LEAN FP64 or FP32 systems");
    const wg_team<T> team{red2, red};
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(counter, 1u);
        __syncthreads();
        const unsigned qi = s_next;
        __syncthreads();
        if (qi >= nsys) break;  // uniform: the queue is empty
        const int32_t sid = order[qi];
        const sys_view S = system_view(sid, row_off, nnz_off, rp_local, col);
        if constexpr (WAVES) {
            if (S.m <= kWaveRows) {  // uniform
                // The queue is ordered by decreasing rows, so every later
                // system is this small too: from here each wavefront takes
                // systems of its own (wavefront 0 this one) until the queue
                // is empty, and the workgroup passes no barrier again.
                const int wv = threadIdx.x / kWave;
                double *pw = lds + wv * kWaveRows * (kRefine ? 4 : 1);
                for (unsigned q = wv == 0 ? qi : pop_wave(counter); q < nsys; q = pop_wave(counter))
                    solve_on_wave(order[q], row_off, nnz_off, rp_local, col, val, b, xout, tol,
                                  maxit, iters, relres, status, pw);
                return;
            }
        }
        const VA *A = val + nnz_off[sid];
        const double *bs = b + S.row0;
        double bb = 0.0;
        for (int i = threadIdx.x; i < S.m; i += T) bb += bs[i] * bs[i];
        bb = wg_sum<T>(bb, red);
        const double bnorm = sqrt(bb);
        sys_regs<VA, T> regs;
        const bool cached = regs.load(S, A, team);
        int its = 0, flag = 0;
        double *x64 = lds;            // m doubles
        if constexpr (LEAN) {
            // the host chooses LEAN only when every system is cached
            if (cached)
                its = cg_cached<VA, double, wg_team<T>, true>(S.m, regs, nullptr, bs, x64, bb,
                                                              tol * tol * bb, maxit, team, &flag);
            else
                flag = 2;
        } else if constexpr (!kRefine) {
            double *r = x64 + S.m, *p = r + S.m, *q = p + S.m;
            for (int i = threadIdx.x; i < S.m; i += T) {
                x64[i] = 0.0;
                r[i] = bs[i];
                p[i] = bs[i];
            }
            wg_sync<T>();
            its = cached ? cg_cached<VA, double, wg_team<T>>(S.m, regs, x64, r, p, bb,
                                                             tol * tol * bb, maxit, team, &flag)
                         : cg_in_lds<VA, double, T>(S, A, x64, r, p, q, bb, tol * tol * bb, maxit,
                                                    red2, &flag);
        } else {
            its = solve_refined(S, A, bs, bnorm, regs, cached, tol, maxit, x64, team, &flag);
        }
        // true residual of the final x (FP64), x to global memory
        wg_sync<T>();
        finish_system(sid, S, A, bs, x64, xout, bnorm, tol, its, flag, iters, relres, status, team);
        __syncthreads();
    }
}

// Structure check, one workgroup per system: local offsets start at 0, do
// not decrease, end at the system's nonzero count; columns in [0, m).
__global__ void batch_validate_kernel(int64_t nsys, const int64_t *__restrict__ row_off,
                                      const int64_t *__restrict__ nnz_off,
                                      const int32_t *__restrict__ rp_local,
                                      const int32_t *__restrict__ col, int *err) {
    int longest = 0;
    const int64_t sid = blockIdx.x;
    if (sid >= nsys) return;
    const int64_t m = row_off[sid + 1] - row_off[sid];
    const int64_t nz = nnz_off[sid + 1] - nnz_off[sid];
    const int32_t *rp = rp_local + row_off[sid] + sid;
    const int32_t *c = col + nnz_off[sid];
    int bad = 0;
    if (threadIdx.x == 0 && (rp[0] != 0 || (int64_t)rp[m] != nz)) bad = 1;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        if (rp[i + 1] < rp[i]) bad = 1;
        else {
            if (rp[i + 1] - rp[i] > longest) longest = rp[i + 1] - rp[i];
            for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
                if (c[k] < 0 || c[k] >= m) bad = 1;
        }
    }
    if (bad) atomicOr(err, 1);
    if (longest) atomicMax(err + 1, longest);  // err[1]: the longest row of any system
}

hipError_t batch_validate(hipStream_t s, int64_t nsys, const int64_t *row_off,
                          const int64_t *nnz_off, const int32_t *rp_local, const int32_t *col,
                          int *err) {
    if (nsys == 0) return hipSuccess;
    batch_validate_kernel<<<(unsigned)nsys, 256, 0, s>>>(nsys, row_off, nnz_off, rp_local, col, err);
    return hipGetLastError();
}

__global__ void batch_reset_kernel(unsigned *counter, int *status) {
    *counter = 0u;
    *status = 0;
}

size_t batch_lds_bytes(vt t, int64_t max_m, bool lean, bool waves, int block) {
    // bytes per row: p (LEAN), x r p q (FP64), x r in FP64 and d r p q in FP32
    const int64_t per_row = lean ? 8 : t == vt::f64 ? 4 * 8 : 2 * 8 + 4 * 4;
    const int64_t rows = waves ? (int64_t)(block / kWave) * kWaveRows : 0;
    return (size_t)((max_m > rows ? max_m : rows) * per_row);
}

bool batch_waves_fit(vt t, bool lean, int64_t max_row_len) {
    return t == vt::f64 ? lean : max_row_len <= kBatchCacheLen;
}

bool batch_lean_fits(vt t, int block, int64_t max_m, int64_t max_row_len) {
    if (t != vt::f64 || block <= 0) return false;
    const int64_t rows = (1024 / block < 4 ? 1024 / block : 4) * (int64_t)block;
    return max_m <= rows && max_row_len <= kBatchCacheLen;
}

// Workgroups of batch_cg_kernel<VA, T, LEAN, WAVES> resident on the device at once.
template <typename VA, int T, bool LEAN, bool WAVES>
static hipError_t resident_t(int64_t max_m, int *out) {
    const size_t lds = batch_lds_bytes(sizeof(VA) == 8 ? vt::f64 : vt::f32, max_m, LEAN, WAVES, T);
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_cg_kernel<VA, T, LEAN, WAVES>,
                                                         T, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    *out = cus * per_cu;
    return hipSuccess;
}

template <typename VA, bool LEAN, bool WAVES>
static hipError_t resident_v(int block, int64_t max_m, int *out) {
    switch (block) {
        case 64: return resident_t<VA, 64, LEAN, WAVES>(max_m, out);
        case 128: return resident_t<VA, 128, LEAN, WAVES>(max_m, out);
        case 256: return resident_t<VA, 256, LEAN, WAVES>(max_m, out);
        case 512: return resident_t<VA, 512, LEAN, WAVES>(max_m, out);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_resident(vt t, int block, int64_t max_m, bool lean, bool waves, int *workgroups) {
    if ((lean && t != vt::f64) || (waves && t == vt::f64 && !lean)) return hipErrorInvalidValue;
    if (t == vt::f32)
        return waves ? resident_v<float, false, true>(block, max_m, workgroups)
                     : resident_v<float, false, false>(block, max_m, workgroups);
    if (!lean) return resident_v<double, false, false>(block, max_m, workgroups);
    return waves ? resident_v<double, true, true>(block, max_m, workgroups)
                 : resident_v<double, true, false>(block, max_m, workgroups);
}

template <typename VA, int T, bool LEAN, bool WAVES>
static hipError_t launch_batch_t(hipStream_t s, const batch_args &a) {
    const size_t lds =
        batch_lds_bytes(sizeof(VA) == 8 ? vt::f64 : vt::f32, a.max_m, LEAN, WAVES, T);
    int resident = 0;
    hipError_t e = resident_t<VA, T, LEAN, WAVES>(a.max_m, &resident);
    if (e != hipSuccess) return e;
    int64_t grid = resident;
    if (grid > a.nsys) grid = a.nsys;
    if (grid < 1) grid = 1;
    batch_reset_kernel<<<1, 1, 0, s>>>(a.counter, a.status);
    batch_cg_kernel<VA, T, LEAN, WAVES><<<(unsigned)grid, T, lds, s>>>(
        a.nsys, a.row_off, a.nnz_off, a.rp_local, a.col, static_cast<const VA *>(a.val), a.order,
        a.counter, a.b, a.x, a.tol, a.maxit, a.iters, a.relres, a.status);
    return hipGetLastError();
}

template <typename VA, bool LEAN, bool WAVES>
static hipError_t launch_batch_v(hipStream_t s, const batch_args &a) {
    switch (a.block) {
        case 64: return launch_batch_t<VA, 64, LEAN, WAVES>(s, a);
        case 128: return launch_batch_t<VA, 128, LEAN, WAVES>(s, a);
        case 256: return launch_batch_t<VA, 256, LEAN, WAVES>(s, a);
        case 512: return launch_batch_t<VA, 512, LEAN, WAVES>(s, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_cg(hipStream_t s, vt t, const batch_args &a) {
    if (a.nsys == 0) return hipSuccess;
    if (a.lean && !batch_lean_fits(t, a.block, a.max_m, a.max_row_len)) return hipErrorInvalidValue;
    if (a.waves && !batch_waves_fit(t, a.lean, a.max_row_len)) return hipErrorInvalidValue;
    if (t == vt::f32)
        return a.waves ? launch_batch_v<float, false, true>(s, a)
                       : launch_batch_v<float, false, false>(s, a);
    if (!a.lean) return launch_batch_v<double, false, false>(s, a);
    return a.waves ? launch_batch_v<double, true, true>(s, a)
                   : launch_batch_v<double, true, false>(s, a);
}

}  // namespace gko
