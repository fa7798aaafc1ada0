// The C ABI (include/gko.h): handles, argument checks, format dispatch,
// conversions, and the host drivers of the Krylov solvers.  All arithmetic
// runs in the HIP kernels; this file only orders launches and moves a few
// scalars to the host for convergence checks.
#include <hip/hip_runtime.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <iterator>
#include <chrono>
#include <numeric>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "batch_kernels.hpp"
#include "gko.h"
#include "selector_kernels.hpp"
#include "kernels.hpp"
#include "solver_kernels.hpp"

using namespace gko;

namespace {

thread_local std::string g_last_error;

struct api_error : std::runtime_error {
    gko_status status;
    api_error(gko_status s, const std::string &m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] void fail(gko_status s, const std::string &m) { throw api_error(s, m); }

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(GKO_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}
#define HIPC(expr) hip_check((expr), #expr)

template <typename F>
gko_status guarded(F &&f) {
    try {
        f();
        g_last_error.clear();
        return GKO_OK;
    } catch (const api_error &e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return GKO_ERR_ALLOC;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return GKO_ERR_INVALID_ARG;
    } catch (...) {
        g_last_error = "unknown error";
        return GKO_ERR_INVALID_ARG;
    }
}

double now_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

gko_solver_opts default_opts() {
    gko_solver_opts o;
    o.precision = GKO_PREC_FP64;
    o.precond = GKO_PRECOND_NONE;
    o.block_size = 8;
    o.check_every = 16;
    o.inner_tol = 1e-5;
    o.max_inner = 1000;
    o.max_outer = 20;
    o.single_workgroup = 1;
    o.krylov_dim = 30;
    o.graphs = 1;
    return o;
}

}  // namespace

// ====================================================================== handles
struct gko_context_s {
    hipStream_t stream = nullptr;
    int device = 0;
    gko_alloc_fn alloc = nullptr;
    gko_dealloc_fn dealloc = nullptr;
    void *user = nullptr;
    gko_solver_opts opts = default_opts();
    gko_solve_info info{};
    double *red_partials = nullptr;  // scratch of gko_dot / gko_norm2
    unsigned *red_ticket = nullptr;
    struct gko_mlp_s *selector = nullptr;  // used by gko_convert(AUTO) when set
    int64_t small_cg_rows = -1;            // single-workgroup CG limit, queried once
    unsigned char *scratch = nullptr;      // this device's copy of the no-allocation scratch

    void *alloc_bytes(size_t bytes) {
        if (bytes == 0) bytes = 8;
        void *p = nullptr;
        if (alloc) {
            p = alloc(bytes, (void *)stream, user);
            if (!p) fail(GKO_ERR_ALLOC, "allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMallocAsync(&p, bytes, stream);
            if (e != hipSuccess || !p)
                fail(GKO_ERR_ALLOC, "hipMallocAsync(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
        }
        return p;
    }
    void free_bytes(void *p) {
        if (!p) return;
        if (dealloc) dealloc(p, (void *)stream, user);
        else (void)hipFreeAsync(p, stream);
    }
    void sync() { HIPC(hipStreamSynchronize(stream)); }
};

namespace {

// Device buffer owned by a context, released on scope exit.
struct dbuf {
    gko_context ctx = nullptr;
    void *p = nullptr;
    dbuf() = default;
    dbuf(gko_context c, size_t bytes) : ctx(c), p(c->alloc_bytes(bytes)) {}
    dbuf(const dbuf &) = delete;
    dbuf &operator=(const dbuf &) = delete;
    dbuf(dbuf &&o) noexcept : ctx(o.ctx), p(o.p) { o.p = nullptr; }
    dbuf &operator=(dbuf &&o) noexcept {
        if (this != &o) {
            if (p) ctx->free_bytes(p);
            ctx = o.ctx;
            p = o.p;
            o.p = nullptr;
        }
        return *this;
    }
    ~dbuf() {
        if (p) ctx->free_bytes(p);
    }
    template <typename T>
    T *as() const { return static_cast<T *>(p); }
    void *release() {
        void *q = p;
        p = nullptr;
        return q;
    }
};

}  // namespace

struct gko_matrix_s {
    gko_context ctx = nullptr;
    gko_format fmt = GKO_FMT_CSR;
    gko_dtype dt = GKO_F64;
    int64_t n = 0, m = 0, nnz = 0;
    int32_t *rp = nullptr;    // CSR, CSR_MERGE
    int32_t *row = nullptr;   // COO
    int32_t *col = nullptr;   // CSR, CSR_MERGE, COO
    void *val = nullptr;      // CSR, CSR_MERGE, COO
    int32_t *part = nullptr;  // CSR_MERGE partition, 2 * (tiles + 1)
    int64_t tiles = 0;
    int64_t K = 0, ld = 0;    // ELL, HYBRID
    int32_t *ecol = nullptr;  // ELL / HYBRID slots; SELLP: the slice slots
    void *eval = nullptr;
    int64_t slots = 0;        // SELLP: slots of all slices (sets[slices])
    int64_t *sset = nullptr;  // SELLP: slices + 1 slot offsets
    int32_t *swidth = nullptr;  // SELLP: width of each slice
    // SELLP slices wider than kSellpWide, split into column chunks
    int64_t n_wide = 0, n_wide_items = 0;
    int32_t *wide_slices = nullptr, *wide_first = nullptr, *wide_items = nullptr;
    void *wide_partial = nullptr;  // n_wide_items * kSellpSlice doubles
    int64_t tnnz = 0;         // HYBRID tail
    int32_t *trow = nullptr, *tcol = nullptr;
    void *tval = nullptr;
    int subwarp = 1;
    int row_lanes = 1;              // CSR row-per-thread kernel: lanes per row
    bool merge_rows = false;        // CSR_MERGE: tiles sum their rows in parallel
    int64_t max_len = -1;           // longest row (a property of the matrix), -1 until needed
    int64_t n_long = 0;             // CSR rows handled by a workgroup each
    int32_t *long_rows = nullptr;
    void *carry_a = nullptr, *carry_b = nullptr;  // merge / COO carries
    int64_t carry_elems = 0;
    // FP32 copies of the value arrays, made on demand for mixed precision
    void *val32 = nullptr, *eval32 = nullptr, *tval32 = nullptr;
    // block-Jacobi inverse cache
    int bj_bs = 0;
    double *bj64 = nullptr;
    float *bj32 = nullptr;

    vt type() const { return dt == GKO_F64 ? vt::f64 : vt::f32; }
    size_t vs() const { return vsize(type()); }
    int64_t slices() const { return (n + kSellpSlice - 1) / kSellpSlice; }
    // elements of ecol / eval
    int64_t ell_elems() const { return fmt == GKO_FMT_SELLP ? slots : K * ld; }
    sellp_wide wide() const {
        sellp_wide w;
        w.n_wide = n_wide;
        w.n_items = n_wide_items;
        w.slices = wide_slices;
        w.first = wide_first;
        w.items = wide_items;
        w.partial = wide_partial;
        return w;
    }

    void drop(void *&p) {
        ctx->free_bytes(p);
        p = nullptr;
    }
    template <typename T>
    void drop(T *&p) {
        ctx->free_bytes((void *)p);
        p = nullptr;
    }
    void drop_caches() {
        drop(val32);
        drop(eval32);
        drop(tval32);
        drop(bj64);
        drop(bj32);
        bj_bs = 0;
    }
    void drop_storage() {
        drop(rp); drop(row); drop(col); drop(val); drop(part); drop(ecol); drop(eval);
        drop(trow); drop(tcol); drop(tval); drop(carry_a); drop(carry_b); drop(long_rows);
        drop(sset); drop(swidth); drop(wide_slices); drop(wide_first); drop(wide_items);
        drop(wide_partial);
        tiles = K = ld = tnnz = carry_elems = n_long = slots = n_wide = n_wide_items = 0;
        drop_caches();
    }
    int64_t stored_bytes() const {
        const int64_t s = (int64_t)vs();
        switch (fmt) {
            case GKO_FMT_CSR: return (n + 1) * 4 + nnz * (4 + s);
            case GKO_FMT_CSR_MERGE: return (n + 1) * 4 + nnz * (4 + s) + 8 * (tiles + 1);
            case GKO_FMT_COO: return nnz * (8 + s);
            case GKO_FMT_ELL: return K * ld * (4 + s);
            case GKO_FMT_HYBRID: return K * ld * (4 + s) + tnnz * (8 + s);
            case GKO_FMT_SELLP:
                return slots * (4 + s) + (slices() + 1) * 8 + slices() * 4 + n_wide * 4 +
                       (n_wide > 0 ? (n_wide + 1) * 4 : 0) + n_wide_items * (8 + kSellpSlice * 8);
            default: return 0;
        }
    }
};

namespace {

void require(bool ok, gko_status s, const std::string &m) {
    if (!ok) fail(s, m);
}

int64_t round_up64(int64_t v) { return (v + 63) / 64 * 64; }

// Scratch of the grid reductions: up to 3 values per block of the vector
// kernels' grids, or up to kFusedMaxSums per block of a fused product's
// larger grid.
constexpr size_t kPartialBytes =
    (size_t)std::max(3 * kMaxReductionBlocks, kFusedMaxSums * kFusedMaxBlocks) * sizeof(double);

// ---------------------------------------------------------------- no-allocation scratch
// The device memory of gko_cg_solve_noalloc: one static array per device,
// held until the process ends.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol): each device's
// address comes from hipGetSymbolAddress, resolved once per device when the
// first context on it is created, and kept in a per-device table.
constexpr size_t kScratchBytes = size_t(64) << 20;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_addr;  // indexed by device

// Address of this device's scratch array; the device must be current.
unsigned char *resolve_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_addr.size() <= device) g_scratch_addr.resize(device + 1, nullptr);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(GKO_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[device] = static_cast<unsigned char *>(p);
    }
    return g_scratch_addr[device];
}

void ensure_carries(gko_matrix A, int64_t elems) {
    if (A->carry_elems >= elems && A->carry_a) return;
    A->drop(A->carry_a);
    A->drop(A->carry_b);
    A->carry_a = A->ctx->alloc_bytes((size_t)std::max<int64_t>(elems, 1) * 8);
    A->carry_b = A->ctx->alloc_bytes((size_t)std::max<int64_t>(elems, 1) * 8);
    A->carry_elems = elems;
}

// Value arrays of one precision: the stored ones, or the FP32 copies.
struct values {
    vt t;
    const void *val, *eval, *tval;
};

values own_values(gko_matrix A) { return {A->type(), A->val, A->eval, A->tval}; }

void spmv_dispatch(gko_matrix A, const values &v, double alpha, const void *x, double beta, void *y) {
    hipStream_t s = A->ctx->stream;
    // No entries: y <- beta y.  The ELL kernels read x[0] for padding slots,
    // so the kernels below run only when x has an element.
    if (A->nnz == 0) {
        HIPC(scale(s, v.t, A->n, beta, y));
        return;
    }
    switch (A->fmt) {
        case GKO_FMT_CSR:
            HIPC(spmv_csr(s, v.t, A->n, A->rp, A->col, v.val, x, alpha, beta, y, A->subwarp,
                          A->row_lanes, A->n_long, A->long_rows));
            break;
        case GKO_FMT_CSR_MERGE:
            HIPC(spmv_merge(s, v.t, A->n, A->nnz, A->rp, A->col, v.val, A->part, x, alpha, beta, y,
                            static_cast<int32_t *>(A->carry_a), A->carry_b, A->merge_rows));
            break;
        case GKO_FMT_COO:
            HIPC(spmv_coo(s, v.t, A->n, A->nnz, A->row, A->col, v.val, x, alpha, beta, y, false,
                          A->carry_a, A->carry_b));
            break;
        case GKO_FMT_ELL:
            HIPC(spmv_ell(s, v.t, A->n, A->K, A->ld, A->ecol, v.eval, x, alpha, beta, y));
            break;
        case GKO_FMT_HYBRID:
            HIPC(spmv_ell(s, v.t, A->n, A->K, A->ld, A->ecol, v.eval, x, alpha, beta, y));
            if (A->tnnz > 0)
                HIPC(spmv_coo(s, v.t, A->n, A->tnnz, A->trow, A->tcol, v.tval, x, alpha, 1.0, y,
                              true, A->carry_a, A->carry_b));
            break;
        case GKO_FMT_SELLP:
            HIPC(spmv_sellp(s, v.t, A->n, A->sset, A->ecol, v.eval, x, alpha, beta, y, A->wide()));
            break;
        default:
            fail(GKO_ERR_INVALID_ARG, "matrix has no storage format");
    }
}

// ---------------------------------------------------------------- conversions
// Writes the logical matrix as CSR (n+1 offsets, nnz columns, nnz values of
// the given value arrays) into device buffers, whatever the stored format.
void export_csr_into(gko_matrix A, const values &v, int32_t *rp, int32_t *col, void *val) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    const size_t vb = vsize(v.t);
    switch (A->fmt) {
        case GKO_FMT_CSR:
        case GKO_FMT_CSR_MERGE:
            HIPC(hipMemcpyAsync(rp, A->rp, (A->n + 1) * 4, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(col, A->col, A->nnz * 4, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(val, v.val, A->nnz * vb, hipMemcpyDeviceToDevice, s));
            break;
        case GKO_FMT_COO:
            HIPC(rows_to_ptr(s, A->n, A->nnz, A->row, rp));
            HIPC(hipMemcpyAsync(col, A->col, A->nnz * 4, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(val, v.val, A->nnz * vb, hipMemcpyDeviceToDevice, s));
            break;
        case GKO_FMT_ELL:
        case GKO_FMT_HYBRID: {
            dbuf tptr;
            if (A->fmt == GKO_FMT_HYBRID) {
                tptr = dbuf(c, (A->n + 1) * 4);
                HIPC(rows_to_ptr(s, A->n, A->tnnz, A->trow, tptr.as<int32_t>()));
            }
            dbuf len(c, std::max<int64_t>(A->n, 1) * 4);
            dbuf tmp(c, scan_tmp_elems(A->n) * 4);
            HIPC(hyb_lengths(s, A->n, A->K, A->ld, A->ecol, tptr.as<int32_t>(), len.as<int32_t>()));
            HIPC(exclusive_scan(s, A->n, len.as<int32_t>(), rp, tmp.as<int32_t>()));
            HIPC(hyb_to_csr(s, v.t, A->n, A->K, A->ld, A->ecol, v.eval, tptr.as<int32_t>(), A->tcol,
                            v.tval, rp, col, val));
            c->sync();
            break;
        }
        case GKO_FMT_SELLP: {
            dbuf len(c, std::max<int64_t>(A->n, 1) * 4);
            dbuf tmp(c, scan_tmp_elems(A->n) * 4);
            HIPC(sellp_lengths(s, A->n, A->sset, A->ecol, len.as<int32_t>()));
            HIPC(exclusive_scan(s, A->n, len.as<int32_t>(), rp, tmp.as<int32_t>()));
            HIPC(sellp_to_csr(s, v.t, A->n, A->sset, A->ecol, v.eval, rp, col, val));
            c->sync();
            break;
        }
        default:
            fail(GKO_ERR_INVALID_ARG, "matrix has no storage format");
    }
}

int64_t read_int(gko_context c, const int *d);

int64_t max_len_of_csr(gko_matrix A);

// Rows too long for a subwarp get a workgroup each (see spmv_csr).
void refresh_long_rows(gko_matrix A) {
    A->drop(A->long_rows);
    A->n_long = 0;
    if (A->n == 0) return;
    if (A->max_len < 0) A->max_len = max_len_of_csr(A);
    if (!csr_has_long_rows(A->n, A->nnz, A->max_len, A->subwarp)) return;
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    dbuf flag(c, A->n * 4), pos(c, (A->n + 1) * 4), tmp(c, scan_tmp_elems(A->n) * 4);
    HIPC(csr_long_flags(s, A->n, A->rp, csr_long_threshold(A->subwarp), flag.as<int32_t>()));
    HIPC(exclusive_scan(s, A->n, flag.as<int32_t>(), pos.as<int32_t>(), tmp.as<int32_t>()));
    const int64_t nl = read_int(c, pos.as<int>() + A->n);
    if (nl > 0) {
        dbuf rows(c, nl * 4);
        HIPC(csr_long_scatter(s, A->n, flag.as<int32_t>(), pos.as<int32_t>(), rows.as<int32_t>()));
        c->sync();
        A->long_rows = static_cast<int32_t *>(rows.release());
        A->n_long = nl;
    }
}

// The CSR kernel for this matrix (csr_kernel_width: a thread per row for
// short rows, else a subwarp per row), then the list of rows too long for
// that subwarp width.
void analyse_csr(gko_matrix A) {
    if (A->max_len < 0) A->max_len = A->n > 0 ? max_len_of_csr(A) : 0;
    A->subwarp = csr_kernel_width(A->n, A->nnz, A->max_len);
    A->row_lanes = csr_row_lanes(A->n, A->nnz);
    refresh_long_rows(A);
}

void to_csr(gko_matrix A) {
    if (A->fmt == GKO_FMT_CSR) return;
    if (A->fmt == GKO_FMT_CSR_MERGE) {
        A->drop(A->part);
        A->tiles = 0;
        A->fmt = GKO_FMT_CSR;
        refresh_long_rows(A);
        return;
    }
    gko_context c = A->ctx;
    dbuf rp(c, (A->n + 1) * 4), col(c, A->nnz * 4), val(c, A->nnz * A->vs());
    export_csr_into(A, own_values(A), rp.as<int32_t>(), col.as<int32_t>(), val.p);
    c->sync();
    A->drop_storage();
    A->rp = static_cast<int32_t *>(rp.release());
    A->col = static_cast<int32_t *>(col.release());
    A->val = val.release();
    A->fmt = GKO_FMT_CSR;
    analyse_csr(A);
}

int64_t read_int(gko_context c, const int *d) {
    int h = 0;
    HIPC(hipMemcpyAsync(&h, d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    return h;
}

int64_t max_len_of_csr(gko_matrix A) {
    dbuf ml(A->ctx, 4);
    HIPC(hipMemsetAsync(ml.p, 0, 4, A->ctx->stream));
    HIPC(max_row_len(A->ctx->stream, A->n, A->rp, ml.as<int>()));
    return read_int(A->ctx, ml.as<int>());
}

// K* = argmin_K n*K*(s+4) + (s+8)*sum_i max(0, len_i - K), ties to the smaller K,
// from the row-length histogram (integer arithmetic, exact).
int64_t hyb_width_of_csr(gko_matrix A, int64_t maxlen) {
    gko_context c = A->ctx;
    dbuf hist(c, (maxlen + 1) * 4);
    HIPC(hipMemsetAsync(hist.p, 0, (maxlen + 1) * 4, c->stream));
    HIPC(row_len_hist(c->stream, A->n, A->rp, hist.as<int>(), maxlen));
    std::vector<int> h(maxlen + 1);
    HIPC(hipMemcpyAsync(h.data(), hist.p, (maxlen + 1) * 4, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    const int64_t s = (int64_t)A->vs();
    // rows_gt[K] = #rows with len > K, ent_gt[K] = sum of len over those rows
    int64_t rows_gt = 0, ent_gt = 0;
    std::vector<int64_t> tail(maxlen + 1);
    for (int64_t K = maxlen; K >= 0; --K) {
        tail[K] = ent_gt - K * rows_gt;
        rows_gt += h[K];
        ent_gt += (int64_t)h[K] * K;
    }
    int64_t best = 0, best_cost = -1;
    for (int64_t K = 0; K <= maxlen; ++K) {
        const int64_t cost = A->n * K * (s + 4) + (s + 8) * tail[K];
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = K;
        }
    }
    return best;
}

// SELL-P layout of the rows given by the offsets rp (device): slice widths
// from the device, slot offsets summed on the host in int64.
struct sellp_layout {
    std::vector<int32_t> widths;
    std::vector<int64_t> sets;
};

sellp_layout sellp_layout_of(gko_matrix A, const int32_t *rp) {
    gko_context c = A->ctx;
    const int64_t ns = A->slices();
    sellp_layout L;
    L.widths.assign(ns, 0);
    L.sets.assign(ns + 1, 0);
    if (ns == 0) return L;
    dbuf w(c, ns * 4);
    HIPC(sellp_widths(c->stream, A->n, rp, w.as<int32_t>()));
    HIPC(hipMemcpyAsync(L.widths.data(), w.p, ns * 4, hipMemcpyDeviceToHost, c->stream));
    c->sync();
    for (int64_t k = 0; k < ns; ++k) L.sets[k + 1] = L.sets[k] + (int64_t)L.widths[k] * kSellpSlice;
    return L;
}

void csr_to_format(gko_matrix A, gko_format fmt) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    switch (fmt) {
        case GKO_FMT_CSR:
            return;
        case GKO_FMT_CSR_MERGE: {
            A->drop(A->long_rows);
            A->n_long = 0;
            const int64_t tiles = merge_tiles(A->n, A->nnz);
            dbuf part(c, 2 * (tiles + 1) * 4);
            HIPC(merge_partition(s, A->n, A->nnz, A->rp, part.as<int32_t>()));
            ensure_carries(A, tiles);
            if (A->max_len < 0) A->max_len = A->n > 0 ? max_len_of_csr(A) : 0;
            c->sync();
            A->part = static_cast<int32_t *>(part.release());
            A->tiles = tiles;
            A->merge_rows = merge_rows_parallel(A->n, A->nnz, A->max_len);
            A->fmt = GKO_FMT_CSR_MERGE;
            return;
        }
        case GKO_FMT_COO: {
            dbuf row(c, A->nnz * 4);
            HIPC(csr_rows(s, A->n, A->rp, row.as<int32_t>()));
            ensure_carries(A, coo_chunks(A->nnz));
            c->sync();
            A->drop(A->rp);
            A->drop(A->long_rows);
            A->n_long = 0;
            A->row = static_cast<int32_t *>(row.release());
            A->fmt = GKO_FMT_COO;
            return;
        }
        case GKO_FMT_ELL:
        case GKO_FMT_HYBRID: {
            const int64_t maxlen = max_len_of_csr(A);
            const int64_t K = fmt == GKO_FMT_ELL ? maxlen : hyb_width_of_csr(A, maxlen);
            const int64_t ld = round_up64(A->n);
            const int64_t vsz = (int64_t)A->vs();
            dbuf tptr, trow, tcol, tval;
            int64_t tnnz = 0;
            if (fmt == GKO_FMT_HYBRID) {
                dbuf len(c, std::max<int64_t>(A->n, 1) * 4), tmp(c, scan_tmp_elems(A->n) * 4);
                tptr = dbuf(c, (A->n + 1) * 4);
                HIPC(tail_lengths(s, A->n, A->rp, K, len.as<int32_t>()));
                HIPC(exclusive_scan(s, A->n, len.as<int32_t>(), tptr.as<int32_t>(), tmp.as<int32_t>()));
                tnnz = read_int(c, tptr.as<int>() + A->n);
                trow = dbuf(c, tnnz * 4);
                tcol = dbuf(c, tnnz * 4);
                tval = dbuf(c, tnnz * vsz);
                HIPC(csr_to_tail(s, A->type(), A->n, A->rp, A->col, A->val, K, tptr.as<int32_t>(),
                                 trow.as<int32_t>(), tcol.as<int32_t>(), tval.p));
            }
            dbuf ecol(c, K * ld * 4), eval(c, K * ld * vsz);
            HIPC(csr_to_ell(s, A->type(), A->n, A->rp, A->col, A->val, K, ld, ecol.as<int32_t>(), eval.p));
            if (tnnz > 0) ensure_carries(A, coo_chunks(tnnz));
            c->sync();
            void *ca = A->carry_a, *cb = A->carry_b;
            const int64_t ce = A->carry_elems;
            A->carry_a = A->carry_b = nullptr;
            A->drop_storage();
            A->carry_a = ca;
            A->carry_b = cb;
            A->carry_elems = ce;
            A->K = K;
            A->ld = ld;
            A->ecol = static_cast<int32_t *>(ecol.release());
            A->eval = eval.release();
            A->tnnz = tnnz;
            A->trow = static_cast<int32_t *>(trow.release());
            A->tcol = static_cast<int32_t *>(tcol.release());
            A->tval = tval.release();
            A->fmt = fmt;
            return;
        }
        case GKO_FMT_SELLP: {
            const sellp_layout L = sellp_layout_of(A, A->rp);
            const int64_t ns = A->slices();
            dbuf sets(c, (ns + 1) * 8), widths(c, std::max<int64_t>(ns, 1) * 4);
            dbuf scol(c, L.sets[ns] * 4), sval(c, L.sets[ns] * A->vs());
            HIPC(hipMemcpyAsync(sets.p, L.sets.data(), (ns + 1) * 8, hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(widths.p, L.widths.data(), ns * 4, hipMemcpyHostToDevice, s));
            HIPC(csr_to_sellp(s, A->type(), A->n, A->rp, A->col, A->val, sets.as<int64_t>(),
                              scol.as<int32_t>(), sval.p));
            // wide slices: (slice, first column) work items of kSellpWideChunk columns
            std::vector<int32_t> wsl, wfirst, witems;
            for (int64_t k = 0; k < ns; ++k) {
                if (L.widths[k] <= kSellpWide) continue;
                wsl.push_back((int32_t)k);
                wfirst.push_back((int32_t)(witems.size() / 2));
                for (int64_t j = 0; j < L.widths[k]; j += kSellpWideChunk) {
                    witems.push_back((int32_t)k);
                    witems.push_back((int32_t)j);
                }
            }
            wfirst.push_back((int32_t)(witems.size() / 2));
            const int64_t nw = (int64_t)wsl.size(), nitems = (int64_t)witems.size() / 2;
            dbuf dws, dwf, dwi, dwp;
            if (nw > 0) {
                dws = dbuf(c, nw * 4);
                dwf = dbuf(c, (nw + 1) * 4);
                dwi = dbuf(c, nitems * 8);
                dwp = dbuf(c, nitems * kSellpSlice * 8);
                HIPC(hipMemcpyAsync(dws.p, wsl.data(), nw * 4, hipMemcpyHostToDevice, s));
                HIPC(hipMemcpyAsync(dwf.p, wfirst.data(), (nw + 1) * 4, hipMemcpyHostToDevice, s));
                HIPC(hipMemcpyAsync(dwi.p, witems.data(), nitems * 8, hipMemcpyHostToDevice, s));
            }
            c->sync();
            A->drop_storage();
            A->slots = L.sets[ns];
            A->sset = static_cast<int64_t *>(sets.release());
            A->swidth = static_cast<int32_t *>(widths.release());
            A->n_wide = nw;
            A->n_wide_items = nitems;
            A->wide_slices = static_cast<int32_t *>(dws.release());
            A->wide_first = static_cast<int32_t *>(dwf.release());
            A->wide_items = static_cast<int32_t *>(dwi.release());
            A->wide_partial = dwp.release();
            A->ecol = static_cast<int32_t *>(scol.release());
            A->eval = sval.release();
            A->fmt = GKO_FMT_SELLP;
            return;
        }
        default:
            fail(GKO_ERR_INVALID_ARG, "unknown format");
    }
}

bool ell_feasible(gko_matrix A, int64_t maxlen) {
    const int64_t s = (int64_t)A->vs();
    const double ell = (double)maxlen * (double)round_up64(A->n) * (double)(s + 4);
    const double csr = (double)A->nnz * (double)(s + 4) + (double)(A->n + 1) * 4.0;
    return ell <= 4.0 * csr;
}

// Maximum row length of the logical matrix, whatever the format.
int64_t max_len_any(gko_matrix A) {
    if (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE) return max_len_of_csr(A);
    gko_context c = A->ctx;
    dbuf rp(c, (A->n + 1) * 4), col(c, A->nnz * 4), val(c, A->nnz * A->vs());
    export_csr_into(A, own_values(A), rp.as<int32_t>(), col.as<int32_t>(), val.p);
    dbuf ml(c, 4);
    HIPC(hipMemsetAsync(ml.p, 0, 4, c->stream));
    HIPC(max_row_len(c->stream, A->n, rp.as<int32_t>(), ml.as<int>()));
    return read_int(c, ml.as<int>());
}

// SELL-P is refused, like ELL, when its padded slots would take more than
// 4x the CSR storage.
bool sellp_feasible(gko_matrix A, int64_t slots) {
    const int64_t s = (int64_t)A->vs();
    const double sellp = (double)slots * (double)(s + 4);
    const double csr = (double)A->nnz * (double)(s + 4) + (double)(A->n + 1) * 4.0;
    return sellp <= 4.0 * csr;
}

void check_sellp_feasible(gko_matrix A) {
    int64_t slots = 0;
    if (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE) {
        slots = sellp_layout_of(A, A->rp).sets.back();
    } else {
        gko_context c = A->ctx;
        dbuf rp(c, (A->n + 1) * 4), col(c, A->nnz * 4), val(c, A->nnz * A->vs());
        export_csr_into(A, own_values(A), rp.as<int32_t>(), col.as<int32_t>(), val.p);
        slots = sellp_layout_of(A, rp.as<int32_t>()).sets.back();
    }
    if (!sellp_feasible(A, slots))
        fail(GKO_ERR_UNSUPPORTED, "SELL-P storage would exceed 4x the CSR storage (" +
                                      std::to_string(slots) + " slots for " +
                                      std::to_string(A->nnz) + " nonzeros)");
}

void convert_to(gko_matrix A, gko_format fmt) {
    if (fmt == A->fmt) return;
    if (fmt == GKO_FMT_ELL) {
        const int64_t maxlen = max_len_any(A);
        if (!ell_feasible(A, maxlen))
            fail(GKO_ERR_UNSUPPORTED, "ELL storage would exceed 4x the CSR storage (max row length " +
                                          std::to_string(maxlen) + ")");
    }
    if (fmt == GKO_FMT_SELLP) check_sellp_feasible(A);
    A->drop_caches();
    to_csr(A);
    csr_to_format(A, fmt);
}

// ---------------------------------------------------------------- FP32 copies
values f32_values(gko_matrix A) {
    if (A->dt == GKO_F32) return own_values(A);
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    if (A->val && !A->val32) {
        A->val32 = c->alloc_bytes(A->nnz * 4);
        HIPC(cast_values(s, vt::f64, vt::f32, A->nnz, A->val, A->val32));
    }
    if (A->eval && !A->eval32) {
        A->eval32 = c->alloc_bytes(A->ell_elems() * 4);
        HIPC(cast_values(s, vt::f64, vt::f32, A->ell_elems(), A->eval, A->eval32));
    }
    if (A->tval && !A->tval32) {
        A->tval32 = c->alloc_bytes(A->tnnz * 4);
        HIPC(cast_values(s, vt::f64, vt::f32, A->tnnz, A->tval, A->tval32));
    }
    return {vt::f32, A->val32, A->eval32, A->tval32};
}

// ---------------------------------------------------------------- block-Jacobi
void ensure_block_jacobi(gko_matrix A, int bs, bool need32) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    if (A->bj_bs != bs) {
        A->drop(A->bj64);
        A->drop(A->bj32);
        A->bj_bs = 0;
        const int64_t nb = (A->n + bs - 1) / bs;
        dbuf inv(c, nb * bs * bs * 8), err(c, 4);
        HIPC(hipMemsetAsync(err.p, 0, 4, s));
        if (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE) {
            HIPC(bj_invert(s, A->n, A->rp, A->col, static_cast<const double *>(A->val), bs,
                           inv.as<double>(), err.as<int>()));
        } else {
            dbuf rp(c, (A->n + 1) * 4), col(c, A->nnz * 4), val(c, A->nnz * 8);
            export_csr_into(A, own_values(A), rp.as<int32_t>(), col.as<int32_t>(), val.p);
            HIPC(bj_invert(s, A->n, rp.as<int32_t>(), col.as<int32_t>(), val.as<double>(), bs,
                           inv.as<double>(), err.as<int>()));
            c->sync();
        }
        if (read_int(c, err.as<int>()))
            fail(GKO_ERR_BREAKDOWN, "block-Jacobi: a diagonal block is singular");
        const int64_t packed = nb * (bs * (bs + 1) / 2);
        dbuf up(c, packed * 8);
        HIPC(bj_pack_upper(s, nb, bs, inv.as<double>(), up.as<double>()));
        c->sync();  // the full inverse is freed on return
        A->bj64 = up.as<double>();
        up.release();
        A->bj_bs = bs;
    }
    if (need32 && !A->bj32) {
        const int64_t packed = (A->n + bs - 1) / bs * (bs * (bs + 1) / 2);
        A->bj32 = static_cast<float *>(c->alloc_bytes(packed * 4));
        HIPC(cast_values(s, vt::f64, vt::f32, packed, A->bj64, A->bj32));
    }
}

// ---------------------------------------------------------------- solver drivers
template <typename T>
T read_back(gko_context c, const T *d) {
    T h;
    HIPC(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    return h;
}

double device_norm(gko_context c, vt t, int64_t n, const void *x, double *out, double *partials,
                   unsigned *ticket) {
    HIPC(dot(c->stream, t, n, x, x, out, partials, ticket, true));
    return read_back(c, out);
}

struct solve_result {
    int32_t flag = kRunning;
    int32_t iters = 0;
    int32_t restarts = 0;
    double relres = 0.0;
    double true_relres = 0.0;
};

gko_status flag_status(int32_t f) {
    switch (f) {
        case kConverged: return GKO_OK;
        case kNotSpd: return GKO_ERR_NOT_SPD;
        case kBreakdown: return GKO_ERR_BREAKDOWN;
        default: return GKO_ERR_NOT_CONVERGED;
    }
}

// The fused-product view of A with the value arrays v; false when its
// storage has no fused kernel (COO, CSR merge, CSR with long rows, HYB with
// a tail, SELL-P with wide slices): the solvers then run the format's SpMV
// and a separate reduction.
bool fused_view(gko_matrix A, const values &v, fused_matrix &f) {
    f = fused_matrix{};
    f.t = v.t;
    f.n = A->n;
    if (A->fmt == GKO_FMT_CSR && A->n_long == 0) {
        f.format = fused_matrix::csr;
        f.rp = A->rp;
        f.col = A->col;
        f.val = v.val;
        f.w = A->subwarp;
        f.lanes = A->row_lanes;
        return true;
    }
    if (A->fmt == GKO_FMT_ELL || (A->fmt == GKO_FMT_HYBRID && A->tnnz == 0)) {
        f.format = fused_matrix::ell;
        f.K = A->K;
        f.ld = A->ld;
        f.ecol = A->ecol;
        f.eval = v.eval;
        return true;
    }
    if (A->fmt == GKO_FMT_SELLP && A->n_wide == 0) {
        f.format = fused_matrix::sellp;
        f.sets = A->sset;
        f.scol = A->ecol;
        f.sval = v.eval;
        return true;
    }
    return false;
}

// One polling interval of a solver loop (check_every iterations of kernel
// launches) as a HIP graph: the first run() captures the body's launches on a
// stream of its own, which the body sees as the context stream, and every
// run() replays them on the context stream with one call instead of one
// enqueue per kernel.  The body must only launch kernels: no allocation, copy,
// memset or synchronization.  Disabled, run() calls the body directly.
// Used for matrices of at most kGraphMaxRows rows: Poisson 3D, per iteration,
// 32^3 rows CG 21.1 -> 17.9 us and BiCGSTAB 34.5 -> 27.4 us; 128^3 and 256^3
// rows 0.5% slower from a graph, where the kernels hide the enqueue cost.
constexpr int64_t kGraphMaxRows = int64_t(1) << 20;

class interval_graph {
  public:
    interval_graph(gko_context c, int64_t n)
        : c_(c), enabled_(c->opts.graphs != 0 && n <= kGraphMaxRows) {}
    interval_graph(const interval_graph &) = delete;
    interval_graph &operator=(const interval_graph &) = delete;
    ~interval_graph() {
        if (exec_) (void)hipGraphExecDestroy(exec_);
        if (cap_) (void)hipStreamDestroy(cap_);
    }

    template <typename F>
    void run(F &&body) {
        if (!enabled_) {
            body();
            return;
        }
        if (!exec_) capture(body);
        HIPC(hipGraphLaunch(exec_, c_->stream));
    }

  private:
    template <typename F>
    void capture(F &body) {
        HIPC(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
        HIPC(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
        const hipStream_t saved = c_->stream;
        hipGraph_t g = nullptr;
        c_->stream = cap_;
        try {
            body();
        } catch (...) {
            c_->stream = saved;
            if (hipStreamEndCapture(cap_, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
            throw;
        }
        c_->stream = saved;
        HIPC(hipStreamEndCapture(cap_, &g));
        const hipError_t e = hipGraphInstantiate(&exec_, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        HIPC(e);
    }

    gko_context c_;
    bool enabled_;
    hipStream_t cap_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
};

// (P)CG on A with the value arrays `v` (FP64 or FP32), b and x of that type.
// inv: block-Jacobi inverse of type v.t (bs > 0) or null.
// Device buffers of one (P)CG solve: vectors r, p, q (and z with a
// preconditioner) of n values, the grid reductions' partials and ticket, the
// iteration scalars and a norm slot.  The solvers allocate them per call
// (cg_buffers); gko_cg_solve_noalloc carves them from the library's static
// scratch array instead.  graphs = false keeps the iteration kernel by
// kernel (no graph is instantiated).
struct cg_workspace {
    void *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
    double *partials = nullptr, *nrm = nullptr;
    unsigned *ticket = nullptr;
    krylov_scalars *S = nullptr;
    bool graphs = true;
};

struct cg_buffers {
    dbuf r, p, q, z, partials, ticket, sc, nrm;
    cg_buffers(gko_context c, int64_t n, size_t vb, int bs)
        : r(c, n * vb), p(c, n * vb), q(c, n * vb), z(c, bs > 0 ? n * vb : 8),
          partials(c, kPartialBytes), ticket(c, 8), sc(c, sizeof(krylov_scalars)), nrm(c, 8) {}
    cg_workspace view() {
        cg_workspace w;
        w.r = r.p;
        w.p = p.p;
        w.q = q.p;
        w.z = z.p;
        w.partials = partials.as<double>();
        w.nrm = nrm.as<double>();
        w.ticket = ticket.as<unsigned>();
        w.S = sc.as<krylov_scalars>();
        return w;
    }
};

solve_result cg_core(gko_matrix A, const values &v, const void *b, void *x, double tol, int32_t maxit,
                     const void *inv, int bs, int check_every, bool true_check, bool flexible,
                     const cg_workspace &w) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    const int64_t n = A->n;
    const size_t vb = vsize(v.t);
    // a fill kernel, not a memset, so that no memset node is ever captured
    HIPC(fill_zero(s, vt::f64, 1, w.ticket));
    krylov_scalars *S = w.S;
    HIPC(scalars_reset(s, S, maxit));
    void *zz = bs > 0 ? w.z : w.r;
    fused_matrix fm;
    const bool fused = fused_view(A, v, fm);
    interval_graph graph(c, w.graphs ? n : kGraphMaxRows + 1);
    solve_result res;
    krylov_scalars h{};
    for (;;) {
        HIPC(hipMemcpyAsync(w.r, b, n * vb, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, w.r);
        HIPC(cg_init(s, v.t, n, b, w.r, zz, w.p, inv, bs, tol, S, w.partials, w.ticket));
        h = read_back(c, S);
        while (h.done == kRunning) {
            graph.run([&] {
                const hipStream_t st = c->stream;
                for (int j = 0; j < check_every; ++j) {
                    if (fused) {
                        HIPC(cg_spmv(st, fm, w.p, w.q, S, w.partials, w.ticket));
                    } else {
                        spmv_dispatch(A, v, 1.0, w.p, 0.0, w.q);
                        HIPC(cg_pq(st, v.t, n, w.p, w.q, S, w.partials, w.ticket));
                    }
                    HIPC(cg_update(st, v.t, n, x, w.r, zz, w.p, w.q, inv, bs, S, w.partials,
                                   w.ticket, flexible));
                    HIPC(cg_direction(st, v.t, n, zz, w.p, S));
                }
            });
            h = read_back(c, S);
        }
        res.flag = h.done;
        res.iters = h.iter;
        res.relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        if (!true_check) break;
        // true residual b - A x (q is free now)
        HIPC(hipMemcpyAsync(w.q, b, n * vb, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, w.q);
        const double tn = device_norm(c, v.t, n, w.q, w.nrm, w.partials, w.ticket);
        res.true_relres = h.bb > 0 ? tn / std::sqrt(h.bb) : 0.0;
        if (h.done != kConverged) break;
        if (tn <= tol * std::sqrt(h.bb)) break;
        if (res.restarts == 2 || h.iter >= maxit) {
            res.flag = kMaxIter;
            break;
        }
        res.restarts += 1;  // restart from the current x
    }
    return res;
}

// Pipelined (P)CG (Ghysels and Vanroose) with the same stopping test,
// true-residual check and restarts as cg_core; one product and one fused
// vector kernel (one reduction) per iteration.
solve_result pipecg_core(gko_matrix A, const values &v, const void *b, void *x, double tol,
                         int32_t maxit, const void *inv, int bs, int check_every, bool true_check) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    const int64_t n = A->n;
    const size_t vb = vsize(v.t);
    const size_t pre = bs > 0 ? n * vb : 8;
    dbuf r(c, n * vb), w(c, n * vb), nn(c, n * vb), z(c, n * vb), sv(c, n * vb), p(c, n * vb);
    dbuf u(c, pre), m(c, pre), q(c, pre);
    dbuf partials(c, kPartialBytes), ticket(c, 8), sc(c, sizeof(krylov_scalars)), nrm(c, 8);
    HIPC(hipMemsetAsync(ticket.p, 0, 8, s));
    auto *S = sc.as<krylov_scalars>();
    HIPC(scalars_reset(s, S, maxit));
    pipe_vectors pv;
    pv.n = nn.p;
    pv.z = z.p;
    pv.s = sv.p;
    pv.p = p.p;
    pv.x = x;
    pv.r = r.p;
    pv.w = w.p;
    pv.u = bs > 0 ? u.p : r.p;
    pv.m = bs > 0 ? m.p : w.p;
    pv.q = bs > 0 ? q.p : sv.p;
    interval_graph graph(c, n);
    solve_result res;
    krylov_scalars h{};
    for (;;) {
        HIPC(hipMemcpyAsync(r.p, b, n * vb, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, r.p);
        // the first step multiplies z, q, s, p by beta = 0: they start at zero
        for (void *vec : {pv.z, pv.q, pv.s, pv.p}) HIPC(fill_zero(s, v.t, n, vec));
        if (bs > 0) HIPC(pipe_precond(s, v.t, n, r.p, pv.u, inv, bs));
        spmv_dispatch(A, v, 1.0, pv.u, 0.0, w.p);
        HIPC(pipe_init(s, v.t, n, b, r.p, pv.u, w.p, pv.m, inv, bs, tol, S, partials.as<double>(),
                       ticket.as<unsigned>()));
        h = read_back(c, S);
        while (h.done == kRunning) {
            graph.run([&] {
                for (int j = 0; j < check_every; ++j) {
                    spmv_dispatch(A, v, 1.0, pv.m, 0.0, nn.p);
                    HIPC(pipe_update(c->stream, v.t, n, pv, inv, bs, S, partials.as<double>(),
                                     ticket.as<unsigned>()));
                }
            });
            h = read_back(c, S);
        }
        res.flag = h.done;
        res.iters = h.iter;
        res.relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
        if (!true_check) break;
        HIPC(hipMemcpyAsync(nn.p, b, n * vb, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, nn.p);
        const double tn = device_norm(c, v.t, n, nn.p, nrm.as<double>(), partials.as<double>(),
                                      ticket.as<unsigned>());
        res.true_relres = h.bb > 0 ? tn / std::sqrt(h.bb) : 0.0;
        if (h.done != kConverged) break;
        if (tn <= tol * std::sqrt(h.bb)) break;
        if (res.restarts == 2 || h.iter >= maxit) {
            res.flag = kMaxIter;
            break;
        }
        res.restarts += 1;   // pipe_init restarts the recurrences; the count goes on
    }
    return res;
}

enum class cg_variant { plain, flexible, pipelined };

solve_result cg_variant_core(cg_variant var, gko_matrix A, const values &v, const void *b, void *x,
                             double tol, int32_t maxit, const void *inv, int bs, int check_every,
                             bool true_check) {
    if (var == cg_variant::pipelined)
        return pipecg_core(A, v, b, x, tol, maxit, inv, bs, check_every, true_check);
    cg_buffers buf(A->ctx, A->n, vsize(v.t), bs);
    return cg_core(A, v, b, x, tol, maxit, inv, bs, check_every, true_check,
                   var == cg_variant::flexible, buf.view());
}

struct mixed_result {
    gko_status status = GKO_OK;
    int32_t inner = 0, outer = 0;
    double true_relres = 0.0;
};

// maxit caps the inner iterations summed over the outer steps, as in the
// FP64 solvers (Sec. 6.2 solvers; mixed-precision reading of the cap)
mixed_result mixed_ir(gko_matrix A, const void *b, void *x, double tol, int32_t maxit,
                      const gko_solver_opts &o, int bs, double bnorm, cg_variant var) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    const int64_t n = A->n;
    const values v64 = own_values(A), v32 = f32_values(A);
    dbuf r(c, n * 8), rt(c, n * 4), d(c, n * 4), nrm(c, 8), partials(c, kPartialBytes), ticket(c, 8);
    HIPC(hipMemsetAsync(ticket.p, 0, 8, s));
    mixed_result res;
    double prev = std::numeric_limits<double>::infinity();
    for (;;) {
        HIPC(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v64, -1.0, x, 1.0, r.p);
        const double rn = device_norm(c, vt::f64, n, r.p, nrm.as<double>(), partials.as<double>(),
                                      ticket.as<unsigned>());
        res.true_relres = rn / bnorm;
        if (std::isnan(rn)) { res.status = GKO_ERR_BREAKDOWN; break; }
        if (rn <= tol * bnorm) { res.status = GKO_OK; break; }
        if (res.outer >= o.max_outer || !(rn <= 0.5 * prev) || res.inner >= maxit) {
            res.status = GKO_ERR_NOT_CONVERGED;
            break;
        }
        prev = rn;
        HIPC(scaled_cast(s, n, r.as<double>(), nrm.as<double>(), rt.as<float>()));
        HIPC(fill_zero(s, vt::f32, n, d.p));
        // ask the inner solve only for the reduction still missing (factor 2
        // of margin), never for less than inner_tol
        const double tau = std::max(o.inner_tol, 0.5 * (tol * bnorm / rn));
        const int32_t cap = std::min(o.max_inner, maxit - res.inner);
        solve_result in = cg_variant_core(var, A, v32, rt.p, d.p, tau, cap,
                                          bs > 0 ? (const void *)A->bj32 : nullptr, bs,
                                          o.check_every, false);
        res.inner += in.iters;
        if (in.flag == kNotSpd || in.flag == kBreakdown) {
            res.status = flag_status(in.flag);
            break;
        }
        HIPC(refine_update(s, n, static_cast<double *>(x), nrm.as<double>(), d.as<float>()));
        res.outer += 1;
    }
    return res;
}

void check_square_f64(gko_matrix A) {
    require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
    require(A->n == A->m, GKO_ERR_DIM_MISMATCH, "matrix must be square");
    require(A->dt == GKO_F64, GKO_ERR_UNSUPPORTED, "solvers take FP64 matrices (mixed precision makes its own FP32 copy)");
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + nb && pb < pa + na;
}

// b is re-read after x has changed (true residual, restarts, refinement
// steps), so the two must not share memory.
void check_solve_args(const void *b, void *x, int64_t n, double tol, int32_t maxit) {
    require(b && x, GKO_ERR_INVALID_ARG, "null b or x");
    require(!overlap(b, size_t(n) * 8, x, size_t(n) * 8), GKO_ERR_INVALID_ARG,
            "b and x overlap");
    require(tol > 0.0 && std::isfinite(tol), GKO_ERR_INVALID_ARG, "tol must be positive and finite");
    require(maxit >= 0, GKO_ERR_INVALID_ARG, "maxit must be >= 0");
}

}  // namespace

// ====================================================================== batches
struct gko_batch_s {
    gko_context ctx = nullptr;
    gko_dtype dt = GKO_F64;
    int64_t nsys = 0, rows = 0, nnz = 0, max_m = 0, max_row_len = 0;
    bool want_lean = true;  // direction-only LDS requested (used where it fits)
    bool lean = false;      // in effect: only the direction in LDS (FP64, rows in registers)
    bool want_waves = false;  // small systems one per wavefront requested (with lean)
    bool waves = false;       // in effect
    int64_t *row_off = nullptr, *nnz_off = nullptr;
    int32_t *rp_local = nullptr, *col = nullptr, *order = nullptr;
    void *val = nullptr;
    unsigned *counter = nullptr;
    int *status = nullptr;
    int block = 128;

    void free_all() {
        void *ps[] = {row_off, nnz_off, rp_local, col, order, val, counter, status};
        for (void *p : ps) ctx->free_bytes(p);
        row_off = nnz_off = nullptr;
        rp_local = col = order = nullptr;
        val = nullptr;
        counter = nullptr;
        status = nullptr;
    }
};

namespace {

bool batch_lean_ok(const gko_batch_s *B, int block) {
    return batch_lean_fits(B->dt == GKO_F64 ? vt::f64 : vt::f32, block, B->max_m, B->max_row_len);
}

bool batch_waves_ok(const gko_batch_s *B, bool lean) {
    return batch_waves_fit(B->dt == GKO_F64 ? vt::f64 : vt::f32, lean, B->max_row_len);
}

// Whether mode (gko_batch_lds) can run at this workgroup size.
bool batch_mode_ok(const gko_batch_s *B, int mode, int block) {
    if (mode == GKO_BATCH_LDS_ALL) return true;
    if (mode == GKO_BATCH_LDS_DIRECTION) return batch_lean_ok(B, block);
    return batch_waves_ok(B, batch_lean_ok(B, block));
}

// The workgroup size and the LDS mode (direction only where requested and
// where every system fits the register cache at that size).
void batch_use_block(gko_batch B, int block) {
    B->block = block;
    B->lean = B->want_lean && batch_lean_ok(B, block);
    B->waves = B->want_waves && batch_waves_ok(B, B->lean);
}

// The mode of gko_batch_set_lds_mode in effect.
int batch_mode(const gko_batch_s *B) {
    return B->waves ? GKO_BATCH_WAVE_SYSTEMS : B->lean ? GKO_BATCH_LDS_DIRECTION : GKO_BATCH_LDS_ALL;
}

void batch_want_mode(gko_batch B, int mode) {
    B->want_lean = mode != GKO_BATCH_LDS_ALL;
    B->want_waves = mode == GKO_BATCH_WAVE_SYSTEMS;
}

gko_status batch_run(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                     int32_t *iters, double *relres, float *ms) {
    gko_context c = B->ctx;
    hipStream_t s = c->stream;
    batch_args a;
    a.nsys = B->nsys;
    a.row_off = B->row_off;
    a.nnz_off = B->nnz_off;
    a.rp_local = B->rp_local;
    a.col = B->col;
    a.val = B->val;
    a.order = B->order;
    a.counter = B->counter;
    a.b = b;
    a.x = x;
    a.tol = tol;
    a.maxit = maxit;
    a.iters = iters;
    a.relres = relres;
    a.status = B->status;
    a.max_m = B->max_m;
    a.max_row_len = B->max_row_len;
    a.block = B->block;
    a.lean = B->lean;
    a.waves = B->waves;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        HIPC(hipEventCreate(&e0));
        HIPC(hipEventCreate(&e1));
        HIPC(hipEventRecord(e0, s));
    }
    HIPC(batch_cg(s, B->dt == GKO_F64 ? vt::f64 : vt::f32, a));
    if (ms) {
        HIPC(hipEventRecord(e1, s));
        HIPC(hipEventSynchronize(e1));
        HIPC(hipEventElapsedTime(ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    const int st = read_int(c, B->status);
    switch (st) {
        case 0: return GKO_OK;
        case kBatchNotSpd: return GKO_ERR_NOT_SPD;
        case kBatchBreakdown: return GKO_ERR_BREAKDOWN;
        default: return GKO_ERR_NOT_CONVERGED;
    }
}

void check_batch_solve_args(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                            int32_t *iters, double *relres) {
    require(B != nullptr, GKO_ERR_INVALID_ARG, "null batch");
    require(B->nsys == 0 || (b && x && iters && relres), GKO_ERR_INVALID_ARG, "null array");
    require(B->nsys == 0 || !overlap(b, size_t(B->rows) * 8, x, size_t(B->rows) * 8),
            GKO_ERR_INVALID_ARG, "b and x overlap");
    require(tol > 0.0 && std::isfinite(tol), GKO_ERR_INVALID_ARG, "tol must be positive and finite");
    require(maxit >= 0, GKO_ERR_INVALID_ARG, "maxit must be >= 0");
}

}  // namespace

// ====================================================================== selector
struct gko_mlp_s {
    gko_context ctx = nullptr;
    float *params = nullptr;  // kMlpParams
    float *norm = nullptr;    // mean[32], std[32]
    float *adam_m = nullptr, *adam_v = nullptr;
    int *step = nullptr;
    float *grads = nullptr;
    double *lossp = nullptr, *msum = nullptr;
    unsigned *ticket = nullptr;

    void free_all() {
        void *ps[] = {params, norm, adam_m, adam_v, step, grads, lossp, msum, ticket};
        for (void *p : ps) ctx->free_bytes(p);
    }
    mlp_work work() const { return {msum, grads, lossp, ticket, adam_m, adam_v, step}; }
};

namespace {

constexpr char kMlpMagic[8] = {'G', 'K', 'O', 'M', 'L', 'P', '1', '\0'};

gko_mlp new_mlp(gko_context ctx, const float *params_host, const float *norm_host) {
    auto M = new gko_mlp_s();
    M->ctx = ctx;
    try {
        hipStream_t s = ctx->stream;
        M->params = static_cast<float *>(ctx->alloc_bytes(kMlpParams * 4));
        M->norm = static_cast<float *>(ctx->alloc_bytes(2 * kMlpIn * 4));
        M->adam_m = static_cast<float *>(ctx->alloc_bytes(kMlpParams * 4));
        M->adam_v = static_cast<float *>(ctx->alloc_bytes(kMlpParams * 4));
        M->step = static_cast<int *>(ctx->alloc_bytes(8));
        M->grads = static_cast<float *>(ctx->alloc_bytes((size_t)kMlpMaxBlocks * kMlpParams * 4));
        M->lossp = static_cast<double *>(ctx->alloc_bytes(kMlpMaxBlocks * 8));
        M->msum = static_cast<double *>(ctx->alloc_bytes(8));
        M->ticket = static_cast<unsigned *>(ctx->alloc_bytes(8));
        std::vector<float> norm(2 * kMlpIn, 0.0f);
        if (norm_host) std::copy(norm_host, norm_host + 2 * kMlpIn, norm.begin());
        else std::fill(norm.begin() + kMlpIn, norm.end(), 1.0f);
        HIPC(hipMemcpyAsync(M->params, params_host, kMlpParams * 4, hipMemcpyHostToDevice, s));
        HIPC(hipMemcpyAsync(M->norm, norm.data(), 2 * kMlpIn * 4, hipMemcpyHostToDevice, s));
        HIPC(hipMemsetAsync(M->adam_m, 0, kMlpParams * 4, s));
        HIPC(hipMemsetAsync(M->adam_v, 0, kMlpParams * 4, s));
        HIPC(hipMemsetAsync(M->step, 0, 8, s));
        HIPC(hipMemsetAsync(M->ticket, 0, 8, s));
        ctx->sync();
    } catch (...) {
        M->free_all();
        delete M;
        throw;
    }
    return M;
}

// The 32 features from the row-length histogram and the entry counters; the
// same definitions as listed in the header (row-length statistics exact from
// integer counts, ratios and logarithms in FP64, rounded to FP32 at the end).
void finish_features(int64_t n, int64_t m, int64_t nnz, const std::vector<int> &h,
                     const unsigned long long *c, int64_t sellp_slots, float *out) {
    const int64_t maxl = (int64_t)h.size() - 1;
    const double dn = (double)n, dnz = nnz > 0 ? (double)nnz : 1.0, dm = m > 0 ? (double)m : 1.0;
    const double mean = n > 0 ? (double)nnz / dn : 0.0;
    int64_t minl = 0;
    while (minl < maxl && h[minl] == 0) ++minl;
    double var = 0.0;
    for (int64_t L = 0; L <= maxl; ++L) var += (double)h[L] * ((double)L - mean) * ((double)L - mean);
    const double sd = n > 0 ? std::sqrt(var / dn) : 0.0;
    auto pct = [&](int64_t P) {  // smallest L with #rows(len <= L) >= ceil(P n / 100)
        const int64_t need = (n * P + 99) / 100;
        int64_t cum = 0;
        for (int64_t L = 0; L <= maxl; ++L) {
            cum += h[L];
            if (cum >= need && need > 0) return (double)L;
        }
        return (double)(need > 0 ? maxl : 0);
    };
    __int128 wsum = 0;
    int64_t rank = 0;
    for (int64_t L = 0; L <= maxl; ++L) {
        const int64_t cnt = h[L];
        wsum += (__int128)L * ((__int128)cnt * rank + (__int128)cnt * (cnt + 1) / 2);
        rank += cnt;
    }
    const double gini = (n > 0 && nnz > 0) ? 2.0 * (double)wsum / (dn * (double)nnz) -
                                                 (double)(n + 1) / dn : 0.0;
    double ent = 0.0;
    for (int64_t L = 0; L <= maxl; ++L)
        if (h[L] > 0) {
            const double p = (double)h[L] / dn;
            ent -= p * std::log(p);
        }
    int64_t left = (n + 99) / 100, topnnz = 0;
    for (int64_t L = maxl; L >= 0 && left > 0; --L) {
        const int64_t take = std::min<int64_t>(left, h[L]);
        topnnz += take * L;
        left -= take;
    }
    // HYB width (FP64 values) and its tail, from the same histogram
    int64_t rows_gt = 0, ent_gt = 0, best = 0, best_cost = -1, tail_best = 0;
    std::vector<int64_t> tail(maxl + 1);
    for (int64_t K = maxl; K >= 0; --K) {
        tail[K] = ent_gt - K * rows_gt;
        rows_gt += h[K];
        ent_gt += (int64_t)h[K] * K;
    }
    for (int64_t K = 0; K <= maxl; ++K) {
        const int64_t cost = n * K * 12 + 16 * tail[K];
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            best = K;
            tail_best = tail[K];
        }
    }
    const double ws = 12.0 * (double)nnz + 4.0 * (double)(n + 1) + 8.0 * (double)m + 8.0 * dn;
    const double pairs = (double)c[6];
    double f[kNumFeatures];
    f[0] = n > 0 ? std::log10(dn) : 0.0;
    f[1] = std::log10(nnz > 0 ? (double)nnz : 1.0);
    f[2] = mean;
    f[3] = sd;
    f[4] = mean > 0 ? sd / mean : 0.0;
    f[5] = (double)minl;
    f[6] = (double)maxl;
    f[7] = pct(50);
    f[8] = pct(90);
    f[9] = pct(99);
    f[10] = mean > 0 ? (double)maxl / mean : 0.0;
    f[11] = n > 0 ? (double)h[0] / dn : 0.0;
    int64_t le4 = 0;
    for (int64_t L = 0; L <= std::min<int64_t>(4, maxl); ++L) le4 += h[L];
    f[12] = n > 0 ? (double)le4 / dn : 0.0;
    f[13] = nnz > 0 ? dn * (double)maxl / (double)nnz : 1.0;
    f[14] = mean > 0 ? (double)best / mean : 0.0;
    f[15] = (double)tail_best / dnz;
    f[16] = gini;
    f[17] = ent;
    f[18] = (double)topnnz / dnz;
    f[19] = std::log10(ws);
    f[20] = nnz > 0 ? (double)sellp_slots / (double)nnz : 1.0;
    f[21] = n > 0 ? (double)m / dn : 0.0;
    f[22] = (double)c[0] / dnz / dm;
    f[23] = (double)c[1] / dm;
    f[24] = (double)c[2] / dnz;
    f[25] = (double)c[3] / dnz;
    f[26] = (double)c[4] / dnz;
    f[27] = std::log10(1.0 + (pairs > 0 ? (double)c[5] / pairs : 0.0));
    f[28] = pairs > 0 ? (double)c[7] / pairs : 0.0;
    f[29] = (double)c[8] / dnz;
    f[30] = n == m ? (double)c[9] / dnz : 0.0;
    f[31] = std::log10(1.0 + (c[11] > 0 ? (double)c[10] / (double)c[11] : 0.0));
    for (int j = 0; j < kNumFeatures; ++j) out[j] = (float)f[j];
}

// Features of A into host memory (32 floats); returns the SELL-P slot count.
int64_t matrix_features(gko_matrix A, float *out) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    dbuf rpb, colb, valb;
    const int32_t *rp = A->rp, *col = A->col;
    if (!(A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE)) {
        rpb = dbuf(c, (A->n + 1) * 4);
        colb = dbuf(c, A->nnz * 4);
        valb = dbuf(c, A->nnz * A->vs());
        export_csr_into(A, own_values(A), rpb.as<int32_t>(), colb.as<int32_t>(), valb.p);
        rp = rpb.as<int32_t>();
        col = colb.as<int32_t>();
    }
    dbuf ml(c, 4);
    HIPC(hipMemsetAsync(ml.p, 0, 4, s));
    HIPC(max_row_len(s, A->n, rp, ml.as<int>()));
    const int64_t maxl = read_int(c, ml.as<int>());
    dbuf hist(c, (maxl + 1) * 4), cnt(c, kFeatCounters * 8);
    HIPC(hipMemsetAsync(hist.p, 0, (maxl + 1) * 4, s));
    HIPC(hipMemsetAsync(cnt.p, 0, kFeatCounters * 8, s));
    HIPC(row_len_hist(s, A->n, rp, hist.as<int>(), maxl));
    HIPC(feature_counts(s, A->n, A->m, rp, col, cnt.as<unsigned long long>()));
    std::vector<int> h(maxl + 1);
    unsigned long long cc[kFeatCounters];
    HIPC(hipMemcpyAsync(h.data(), hist.p, (maxl + 1) * 4, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(cc, cnt.p, kFeatCounters * 8, hipMemcpyDeviceToHost, s));
    c->sync();
    if (A->n == 0) h.assign(1, 0);
    const int64_t slots = sellp_layout_of(A, rp).sets.back();
    finish_features(A->n, A->m, A->nnz, h, cc, slots, out);
    return slots;
}

// The formats the autotuner times and the selector scores, in output order.
const gko_format kAllFormats[kMlpOut] = {GKO_FMT_CSR, GKO_FMT_CSR_MERGE, GKO_FMT_COO,
                                         GKO_FMT_ELL, GKO_FMT_HYBRID, GKO_FMT_SELLP};

// Mean SpMV time of a clone of A in every format (infinity when infeasible);
// A itself is not changed.
void time_formats(gko_matrix A, float *ms_out, int reps) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    const size_t vb = A->vs();
    dbuf x(c, std::max<int64_t>(A->m, 1) * vb), y(c, std::max<int64_t>(A->n, 1) * vb);
    HIPC(fill_zero(s, A->type(), A->m, x.p));
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    HIPC(hipEventCreate(&e1));
    try {
        for (int f = 0; f < kMlpOut; ++f) {
            gko_matrix B = nullptr;
            if (gko_matrix_clone(A, &B) != GKO_OK) fail(GKO_ERR_ALLOC, g_last_error);
            try {
                convert_to(B, kAllFormats[f]);
            } catch (const api_error &e) {
                gko_matrix_destroy(B);
                if (e.status != GKO_ERR_UNSUPPORTED) throw;
                ms_out[f] = std::numeric_limits<float>::infinity();
                continue;
            }
            spmv_dispatch(B, own_values(B), 1.0, x.p, 0.0, y.p);
            spmv_dispatch(B, own_values(B), 1.0, x.p, 0.0, y.p);
            HIPC(hipEventRecord(e0, s));
            for (int r = 0; r < reps; ++r) spmv_dispatch(B, own_values(B), 1.0, x.p, 0.0, y.p);
            HIPC(hipEventRecord(e1, s));
            HIPC(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPC(hipEventElapsedTime(&ms, e0, e1));
            ms_out[f] = ms / reps;
            gko_matrix_destroy(B);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

gko_format select_with(gko_matrix A, gko_mlp model, float *scores) {
    gko_context c = A->ctx;
    hipStream_t s = c->stream;
    float feat[kNumFeatures], sc[kMlpOut];
    const int64_t slots = matrix_features(A, feat);
    dbuf fd(c, kNumFeatures * 4), od(c, kMlpOut * 4);
    HIPC(hipMemcpyAsync(fd.p, feat, kNumFeatures * 4, hipMemcpyHostToDevice, s));
    HIPC(mlp_forward(s, 1, fd.as<float>(), model->params, model->norm, od.as<float>()));
    HIPC(hipMemcpyAsync(sc, od.p, kMlpOut * 4, hipMemcpyDeviceToHost, s));
    c->sync();
    const bool ell_ok = ell_feasible(A, (int64_t)feat[6]);
    const bool sellp_ok = sellp_feasible(A, slots);
    int best = -1;
    for (int f = 0; f < kMlpOut; ++f) {
        if (scores) scores[f] = sc[f];
        if (kAllFormats[f] == GKO_FMT_ELL && !ell_ok) continue;
        if (kAllFormats[f] == GKO_FMT_SELLP && !sellp_ok) continue;
        if (best < 0 || sc[f] < sc[best]) best = f;
    }
    return kAllFormats[best];
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char *gko_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------- autotune cache
// Choices of gko_batch_autotune persist in a text file, one "key value" line
// per entry, keyed by the device architecture and the batch's shape; a batch
// created later with the same key starts from the stored choice.  The file
// is GKO_AUTOTUNE_CACHE when that is set (empty: no cache), else
// $XDG_CACHE_HOME/gko_mi355x/autotune, else ~/.cache/gko_mi355x/autotune.
namespace {

std::mutex g_cache_mu;

std::string autotune_cache_path() {
    if (const char *p = std::getenv("GKO_AUTOTUNE_CACHE")) return p;
    std::string dir;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) dir = x;
    else if (const char *h = std::getenv("HOME"); h && *h) dir = std::string(h) + "/.cache";
    else return "";
    return dir + "/gko_mi355x/autotune";
}

std::string device_arch(int device) {
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    for (char &ch : a)
        if (ch == ' ') ch = '_';
    return a.empty() ? "unknown" : a;
}

std::string batch_cache_key(const gko_batch_s *B) {
    return "batch_cg " + device_arch(B->ctx->device) + " " + (B->dt == GKO_F64 ? "f64" : "f32") +
           " nsys=" + std::to_string(B->nsys) + " rows=" + std::to_string(B->rows) +
           " nnz=" + std::to_string(B->nnz) + " max_m=" + std::to_string(B->max_m);
}

// Lines are "<key> = <value>"; the key never contains " = ".
constexpr const char *kCacheSep = " = ";

// The stored value of key (the last line for it), or "".
std::string cache_lookup(const std::string &key) {
    const std::string path = autotune_cache_path();
    if (path.empty()) return "";
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::ifstream in(path);
    std::string line, found;
    const std::string head = key + kCacheSep;
    while (std::getline(in, line))
        if (line.compare(0, head.size(), head) == 0) found = line.substr(head.size());
    return found;
}

// Replaces (or adds) key's line; the file is rewritten through a temporary
// file and a rename, so readers never see a partial file.  Failures to
// write leave the cache as it was (the choice still applies to this batch).
void cache_store(const std::string &key, const std::string &value) {
    const std::string path = autotune_cache_path();
    if (path.empty()) return;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    std::vector<std::string> lines;
    const std::string head = key + kCacheSep;
    {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line))
            if (line.compare(0, head.size(), head) != 0) lines.push_back(line);
    }
    lines.push_back(head + value);
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string(getpid());
    {
        std::ofstream out(tmp);
        if (!out) return;
        for (const auto &l : lines) out << l << "\n";
        if (!out) {
            std::remove(tmp.c_str());
            return;
        }
    }
    if (std::rename(tmp.c_str(), path.c_str()) != 0) std::remove(tmp.c_str());
}

}  // namespace

gko_status gko_batch_create_csr(gko_context ctx, int64_t nsys, const int64_t *row_off,
                                const int64_t *nnz_off, const int32_t *row_ptr_local,
                                const int32_t *col_idx, const void *values, gko_dtype dt,
                                gko_batch *out) {
    return guarded([&] {
        require(ctx && out, GKO_ERR_INVALID_ARG, "null context or output handle");
        *out = nullptr;
        require(nsys >= 0 && nsys < std::numeric_limits<int32_t>::max(), GKO_ERR_INVALID_ARG,
                "bad system count");
        require(dt == GKO_F64 || dt == GKO_F32, GKO_ERR_INVALID_ARG, "bad dtype");
        require(nsys == 0 || (row_off && nnz_off && row_ptr_local), GKO_ERR_INVALID_ARG,
                "null offsets");
        hipStream_t s = ctx->stream;
        std::vector<int64_t> ro(nsys + 1, 0), no(nsys + 1, 0);
        if (nsys > 0) {
            HIPC(hipMemcpyAsync(ro.data(), row_off, (nsys + 1) * 8, hipMemcpyDeviceToHost, s));
            HIPC(hipMemcpyAsync(no.data(), nnz_off, (nsys + 1) * 8, hipMemcpyDeviceToHost, s));
            ctx->sync();
        }
        require(ro[0] == 0 && no[0] == 0, GKO_ERR_INVALID_ARG, "offsets must start at 0");
        int64_t max_m = 0;
        std::vector<int64_t> nz(nsys);
        for (int64_t i = 0; i < nsys; ++i) {
            const int64_t m = ro[i + 1] - ro[i];
            nz[i] = no[i + 1] - no[i];
            require(m >= 1 && m <= kBatchMaxRows, GKO_ERR_INVALID_ARG,
                    "system " + std::to_string(i) + " has " + std::to_string(m) +
                        " rows (1.." + std::to_string(kBatchMaxRows) + " supported)");
            require(nz[i] >= 0, GKO_ERR_INVALID_ARG, "nonzero offsets must not decrease");
            max_m = std::max(max_m, m);
        }
        const int64_t rows = ro[nsys], nnz = no[nsys];
        require(nnz < std::numeric_limits<int32_t>::max(), GKO_ERR_UNSUPPORTED, "nnz must be below 2^31");
        require(nnz == 0 || (col_idx && values), GKO_ERR_INVALID_ARG, "null columns or values");
        // queue order: most rows first, then most nonzeros (ties by index); the
        // wavefront mode relies on the rows never increasing along the queue
        std::vector<int32_t> order(nsys);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            const int64_t ma = ro[a + 1] - ro[a], mb = ro[b + 1] - ro[b];
            return ma != mb ? ma > mb : nz[a] > nz[b];
        });
        auto B = new gko_batch_s();
        B->ctx = ctx;
        try {
            const size_t vb = dt == GKO_F64 ? 8 : 4;
            B->dt = dt;
            B->nsys = nsys;
            B->rows = rows;
            B->nnz = nnz;
            B->max_m = max_m;
            B->row_off = static_cast<int64_t *>(ctx->alloc_bytes((nsys + 1) * 8));
            B->nnz_off = static_cast<int64_t *>(ctx->alloc_bytes((nsys + 1) * 8));
            B->rp_local = static_cast<int32_t *>(ctx->alloc_bytes((rows + nsys) * 4));
            B->col = static_cast<int32_t *>(ctx->alloc_bytes(nnz * 4));
            B->val = ctx->alloc_bytes(nnz * vb);
            B->order = static_cast<int32_t *>(ctx->alloc_bytes(nsys * 4));
            B->counter = static_cast<unsigned *>(ctx->alloc_bytes(8));
            B->status = static_cast<int *>(ctx->alloc_bytes(8));
            HIPC(hipMemcpyAsync(B->row_off, ro.data(), (nsys + 1) * 8, hipMemcpyHostToDevice, s));
            HIPC(hipMemcpyAsync(B->nnz_off, no.data(), (nsys + 1) * 8, hipMemcpyHostToDevice, s));
            if (nsys > 0) {
                HIPC(hipMemcpyAsync(B->rp_local, row_ptr_local, (rows + nsys) * 4,
                                    hipMemcpyDeviceToDevice, s));
                HIPC(hipMemcpyAsync(B->order, order.data(), nsys * 4, hipMemcpyHostToDevice, s));
            }
            if (nnz > 0) {
                HIPC(hipMemcpyAsync(B->col, col_idx, nnz * 4, hipMemcpyDeviceToDevice, s));
                HIPC(hipMemcpyAsync(B->val, values, nnz * vb, hipMemcpyDeviceToDevice, s));
            }
            HIPC(hipMemsetAsync(B->status, 0, 8, s));
            HIPC(batch_validate(s, nsys, B->row_off, B->nnz_off, B->rp_local, B->col, B->status));
            if (read_int(ctx, B->status))
                fail(GKO_ERR_INVALID_ARG, "malformed system (offsets or column indices)");
            B->max_row_len = read_int(ctx, B->status + 1);
            B->block = max_m <= 256 ? 64 : 128;
            // a stored "block lds_mode" choice for this architecture and shape
            int cb = 0, cm = 0;
            const std::string cv = cache_lookup(batch_cache_key(B));
            if (std::sscanf(cv.c_str(), "%d %d", &cb, &cm) == 2 &&
                (cb == 64 || cb == 128 || cb == 256 || cb == 512) && cm >= 0 && cm <= 2) {
                batch_want_mode(B, cm);
                B->block = cb;
            }
            batch_use_block(B, B->block);
        } catch (...) {
            B->free_all();
            delete B;
            throw;
        }
        *out = B;
    });
}

gko_status gko_batch_destroy(gko_batch B) {
    return guarded([&] {
        if (!B) return;
        B->free_all();
        delete B;
    });
}

gko_status gko_batch_set_block(gko_batch B, int32_t block) {
    return guarded([&] {
        require(B != nullptr, GKO_ERR_INVALID_ARG, "null batch");
        require(block == 64 || block == 128 || block == 256 || block == 512, GKO_ERR_INVALID_ARG,
                "block must be 64, 128, 256 or 512");
        batch_use_block(B, block);
    });
}

gko_status gko_batch_launch_info(gko_batch B, int32_t *resident_workgroups,
                                 int64_t *lds_bytes_per_workgroup) {
    return guarded([&] {
        require(B && resident_workgroups && lds_bytes_per_workgroup, GKO_ERR_INVALID_ARG,
                "null batch or output");
        const vt t = B->dt == GKO_F64 ? vt::f64 : vt::f32;
        int r = 0;
        HIPC(batch_resident(t, B->block, B->max_m, B->lean, B->waves, &r));
        *resident_workgroups = r;
        *lds_bytes_per_workgroup =
            (int64_t)batch_lds_bytes(t, B->max_m, B->lean, B->waves, B->block);
    });
}

gko_status gko_batch_set_lds_mode(gko_batch B, int32_t mode) {
    return guarded([&] {
        require(B != nullptr, GKO_ERR_INVALID_ARG, "null batch");
        require(mode == GKO_BATCH_LDS_ALL || mode == GKO_BATCH_LDS_DIRECTION ||
                    mode == GKO_BATCH_WAVE_SYSTEMS,
                GKO_ERR_INVALID_ARG, "unknown LDS mode");
        require(batch_mode_ok(B, mode, B->block), GKO_ERR_UNSUPPORTED,
                "direction-only LDS needs FP64 values and every system in the register cache at "
                "this workgroup size; wavefront systems need that (FP64) or every row in the "
                "register cache (FP32)");
        batch_want_mode(B, mode);
        batch_use_block(B, B->block);
    });
}

gko_status gko_batch_get_lds_mode(gko_batch B, int32_t *mode) {
    return guarded([&] {
        require(B && mode, GKO_ERR_INVALID_ARG, "null batch or output");
        *mode = batch_mode(B);
    });
}

gko_status gko_batch_get_block(gko_batch B, int32_t *block) {
    return guarded([&] {
        require(B && block, GKO_ERR_INVALID_ARG, "null batch or output");
        *block = B->block;
    });
}

gko_status gko_batch_cg_solve(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                              int32_t *iters_out, double *relres_out) {
    gko_status st = GKO_OK;
    gko_status call = guarded([&] {
        check_batch_solve_args(B, b, x, tol, maxit, iters_out, relres_out);
        if (B->nsys == 0) return;
        st = batch_run(B, b, x, tol, maxit, iters_out, relres_out, nullptr);
    });
    if (call != GKO_OK) return call;
    if (st != GKO_OK) g_last_error = std::string("batch cg: ") + gko_status_string(st);
    return st;
}

gko_status gko_batch_autotune(gko_batch B, const double *b, double *x, double tol, int32_t maxit,
                              int32_t *iters_out, double *relres_out, int32_t *block_out,
                              float *times_ms) {
    return guarded([&] {
        check_batch_solve_args(B, b, x, tol, maxit, iters_out, relres_out);
        const int cand[4] = {64, 128, 256, 512};
        constexpr int kModes = 3;  // gko_batch_lds
        int best = B->block, best_mode = batch_mode(B);
        float best_ms = std::numeric_limits<float>::infinity();
        for (int j = 0; j < 4; ++j)
            for (int mode = 0; mode < kModes; ++mode) {
                float ms = std::numeric_limits<float>::infinity();
                if (batch_mode_ok(B, mode, cand[j])) {
                    batch_want_mode(B, mode);
                    batch_use_block(B, cand[j]);
                    (void)batch_run(B, b, x, tol, maxit, iters_out, relres_out, nullptr);  // warm-up
                    (void)batch_run(B, b, x, tol, maxit, iters_out, relres_out, &ms);
                }
                if (times_ms) times_ms[kModes * j + mode] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand[j];
                    best_mode = mode;
                }
            }
        batch_want_mode(B, best_mode);
        batch_use_block(B, best);
        if (block_out) *block_out = best;
        cache_store(batch_cache_key(B), std::to_string(best) + " " + std::to_string(best_mode));
    });
}

const char *gko_status_string(gko_status s) {
    switch (s) {
        case GKO_OK: return "ok";
        case GKO_ERR_INVALID_ARG: return "invalid argument";
        case GKO_ERR_DIM_MISMATCH: return "dimension mismatch";
        case GKO_ERR_UNSUPPORTED: return "unsupported";
        case GKO_ERR_ALLOC: return "allocation failed";
        case GKO_ERR_HIP: return "HIP runtime error";
        case GKO_ERR_NOT_CONVERGED: return "not converged";
        case GKO_ERR_BREAKDOWN: return "breakdown";
        case GKO_ERR_NOT_SPD: return "matrix not SPD";
        default: return "unknown status";
    }
}

gko_status gko_context_create(void *hip_stream, gko_context *out) {
    return guarded([&] {
        require(out != nullptr, GKO_ERR_INVALID_ARG, "null output handle");
        *out = nullptr;
        auto c = new gko_context_s();
        try {
            HIPC(hipGetDevice(&c->device));
            c->scratch = resolve_scratch(c->device);
            c->stream = static_cast<hipStream_t>(hip_stream);
            HIPC(hipMalloc(&c->red_partials, kPartialBytes));
            HIPC(hipMalloc(&c->red_ticket, 8));
            HIPC(hipMemsetAsync(c->red_ticket, 0, 8, c->stream));
            HIPC(hipStreamSynchronize(c->stream));
        } catch (...) {
            if (c->red_partials) (void)hipFree(c->red_partials);
            if (c->red_ticket) (void)hipFree(c->red_ticket);
            delete c;
            throw;
        }
        *out = c;
    });
}

gko_status gko_context_destroy(gko_context ctx) {
    return guarded([&] {
        if (!ctx) return;
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->red_partials);
        (void)hipFree(ctx->red_ticket);
        delete ctx;
    });
}

gko_status gko_context_set_stream(gko_context ctx, void *hip_stream) {
    return guarded([&] {
        require(ctx != nullptr, GKO_ERR_INVALID_ARG, "null context");
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    });
}

gko_status gko_context_set_allocator(gko_context ctx, gko_alloc_fn alloc, gko_dealloc_fn dealloc,
                                     void *user) {
    return guarded([&] {
        require(ctx != nullptr, GKO_ERR_INVALID_ARG, "null context");
        require((alloc == nullptr) == (dealloc == nullptr), GKO_ERR_INVALID_ARG,
                "alloc and dealloc must both be set or both be NULL");
        ctx->alloc = alloc;
        ctx->dealloc = dealloc;
        ctx->user = user;
    });
}

gko_status gko_matrix_create_csr(gko_context ctx, int64_t n_rows, int64_t n_cols, int64_t nnz,
                                 gko_dtype dt, const void *row_ptr, gko_itype row_ptr_type,
                                 const int32_t *col_idx, const void *values, gko_matrix *out) {
    return guarded([&] {
        require(ctx && out, GKO_ERR_INVALID_ARG, "null context or output handle");
        *out = nullptr;
        require(n_rows >= 0 && n_cols >= 0 && nnz >= 0, GKO_ERR_INVALID_ARG, "negative size");
        require(n_rows < std::numeric_limits<int32_t>::max() &&
                    n_cols <= std::numeric_limits<int32_t>::max(),
                GKO_ERR_UNSUPPORTED, "dimensions must fit int32 indices");
        require(nnz < std::numeric_limits<int32_t>::max(), GKO_ERR_UNSUPPORTED,
                "nnz must be below 2^31");
        require(dt == GKO_F64 || dt == GKO_F32, GKO_ERR_INVALID_ARG, "bad dtype");
        require(row_ptr_type == GKO_I32 || row_ptr_type == GKO_I64, GKO_ERR_INVALID_ARG, "bad itype");
        require(row_ptr != nullptr, GKO_ERR_INVALID_ARG, "null row_ptr");
        require(nnz == 0 || (col_idx && values), GKO_ERR_INVALID_ARG, "null col_idx or values");
        hipStream_t s = ctx->stream;
        const size_t vb = dt == GKO_F64 ? 8 : 4;
        dbuf rp(ctx, (n_rows + 1) * 4), col(ctx, nnz * 4), val(ctx, nnz * vb), err(ctx, 4);
        HIPC(hipMemsetAsync(err.p, 0, 4, s));
        if (row_ptr_type == GKO_I64)
            HIPC(narrow_row_ptr(s, n_rows, static_cast<const int64_t *>(row_ptr), rp.as<int32_t>(),
                                err.as<int>()));
        else
            HIPC(hipMemcpyAsync(rp.p, row_ptr, (n_rows + 1) * 4, hipMemcpyDeviceToDevice, s));
        if (nnz > 0) {
            HIPC(hipMemcpyAsync(col.p, col_idx, nnz * 4, hipMemcpyDeviceToDevice, s));
            HIPC(hipMemcpyAsync(val.p, values, nnz * vb, hipMemcpyDeviceToDevice, s));
        }
        HIPC(validate_csr(s, n_rows, n_cols, nnz, rp.as<int32_t>(), col.as<int32_t>(), err.as<int>()));
        const int64_t e = read_int(ctx, err.as<int>());
        if (e & 1) fail(GKO_ERR_INVALID_ARG, "row_ptr must start at 0, be non-decreasing and end at nnz");
        if (e & 2) fail(GKO_ERR_INVALID_ARG, "column index out of range");
        if (e & 4) fail(GKO_ERR_INVALID_ARG, "column indices must be strictly increasing within a row");
        auto A = new gko_matrix_s();
        A->ctx = ctx;
        A->fmt = GKO_FMT_CSR;
        A->dt = dt;
        A->n = n_rows;
        A->m = n_cols;
        A->nnz = nnz;
        A->rp = static_cast<int32_t *>(rp.release());
        A->col = static_cast<int32_t *>(col.release());
        A->val = val.release();
        try {
            analyse_csr(A);
        } catch (...) {
            A->drop_storage();
            delete A;
            throw;
        }
        *out = A;
    });
}

gko_status gko_matrix_destroy(gko_matrix A) {
    return guarded([&] {
        if (!A) return;
        A->drop_storage();
        delete A;
    });
}

gko_status gko_matrix_clone(gko_matrix A, gko_matrix *out) {
    return guarded([&] {
        require(A && out, GKO_ERR_INVALID_ARG, "null matrix or output handle");
        *out = nullptr;
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        auto B = new gko_matrix_s();
        try {
            B->ctx = c; B->fmt = A->fmt; B->dt = A->dt; B->n = A->n; B->m = A->m; B->nnz = A->nnz;
            B->tiles = A->tiles; B->K = A->K; B->ld = A->ld; B->tnnz = A->tnnz; B->subwarp = A->subwarp;
            B->row_lanes = A->row_lanes;
            B->merge_rows = A->merge_rows;
            B->max_len = A->max_len;
            B->slots = A->slots;
            auto copy = [&](const void *src, size_t bytes) -> void * {
                if (!src) return nullptr;
                void *d = c->alloc_bytes(bytes);
                HIPC(hipMemcpyAsync(d, src, bytes, hipMemcpyDeviceToDevice, s));
                return d;
            };
            const size_t vb = A->vs();
            B->rp = (int32_t *)copy(A->rp, (A->n + 1) * 4);
            B->row = (int32_t *)copy(A->row, A->nnz * 4);
            B->col = (int32_t *)copy(A->col, A->nnz * 4);
            B->val = copy(A->val, A->nnz * vb);
            B->part = (int32_t *)copy(A->part, 2 * (A->tiles + 1) * 4);
            B->ecol = (int32_t *)copy(A->ecol, A->ell_elems() * 4);
            B->eval = copy(A->eval, A->ell_elems() * vb);
            B->sset = (int64_t *)copy(A->sset, (A->slices() + 1) * 8);
            B->swidth = (int32_t *)copy(A->swidth, A->slices() * 4);
            B->n_wide = A->n_wide;
            B->n_wide_items = A->n_wide_items;
            B->wide_slices = (int32_t *)copy(A->wide_slices, A->n_wide * 4);
            B->wide_first = (int32_t *)copy(A->wide_first, (A->n_wide + 1) * 4);
            B->wide_items = (int32_t *)copy(A->wide_items, A->n_wide_items * 8);
            if (A->wide_partial) B->wide_partial = c->alloc_bytes(A->n_wide_items * kSellpSlice * 8);
            B->trow = (int32_t *)copy(A->trow, A->tnnz * 4);
            B->tcol = (int32_t *)copy(A->tcol, A->tnnz * 4);
            B->tval = copy(A->tval, A->tnnz * vb);
            B->n_long = A->n_long;
            B->long_rows = (int32_t *)copy(A->long_rows, A->n_long * 4);
            if (A->carry_a) ensure_carries(B, A->carry_elems);
            c->sync();
        } catch (...) {
            B->drop_storage();
            delete B;
            throw;
        }
        *out = B;
    });
}

gko_status gko_matrix_describe(gko_matrix A, gko_matrix_desc *out) {
    return guarded([&] {
        require(A && out, GKO_ERR_INVALID_ARG, "null matrix or output");
        out->format = A->fmt;
        out->dtype = A->dt;
        out->n_rows = A->n;
        out->n_cols = A->m;
        out->nnz = A->nnz;
        out->ell_width = (A->fmt == GKO_FMT_ELL || A->fmt == GKO_FMT_HYBRID) ? A->K : 0;
        out->ell_ld = (A->fmt == GKO_FMT_ELL || A->fmt == GKO_FMT_HYBRID) ? A->ld : 0;
        out->coo_nnz = A->fmt == GKO_FMT_COO ? A->nnz : (A->fmt == GKO_FMT_HYBRID ? A->tnnz : 0);
        out->stored_bytes = A->stored_bytes();
        out->csr_kernel = A->fmt == GKO_FMT_CSR ? A->subwarp : -1;
        out->csr_row_lanes = (A->fmt == GKO_FMT_CSR && A->subwarp == kCsrRowThread) ? A->row_lanes : 0;
        out->max_row_len = (int32_t)A->max_len;
        out->csr_long_rows = A->fmt == GKO_FMT_CSR ? A->n_long : 0;
        const bool sellp = A->fmt == GKO_FMT_SELLP;
        out->sellp_slice = sellp ? kSellpSlice : 0;
        out->sellp_slices = sellp ? A->slices() : 0;
        out->sellp_slots = sellp ? A->slots : 0;
        out->sellp_wide_slices = sellp ? A->n_wide : 0;
    });
}

gko_status gko_matrix_export_csr(gko_matrix A, int32_t *row_ptr, int32_t *col_idx, void *values) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        require(row_ptr && (A->nnz == 0 || (col_idx && values)), GKO_ERR_INVALID_ARG, "null output");
        export_csr_into(A, own_values(A), row_ptr, col_idx, values);
        A->ctx->sync();
    });
}

gko_status gko_matrix_export_storage(gko_matrix A, int32_t *ell_col, void *ell_val, int32_t *coo_row,
                                     int32_t *coo_col, void *coo_val) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const size_t vb = A->vs();
        const bool has_ell = A->fmt == GKO_FMT_ELL || A->fmt == GKO_FMT_HYBRID;
        const bool has_coo = A->fmt == GKO_FMT_COO || A->fmt == GKO_FMT_HYBRID;
        require(has_ell || (!ell_col && !ell_val), GKO_ERR_INVALID_ARG, "format stores no ELL arrays");
        require(has_coo || (!coo_row && !coo_col && !coo_val), GKO_ERR_INVALID_ARG,
                "format stores no COO arrays");
        const int64_t slots = A->K * A->ld;
        if (ell_col) HIPC(hipMemcpyAsync(ell_col, A->ecol, slots * 4, hipMemcpyDeviceToDevice, s));
        if (ell_val) HIPC(hipMemcpyAsync(ell_val, A->eval, slots * vb, hipMemcpyDeviceToDevice, s));
        const bool hyb = A->fmt == GKO_FMT_HYBRID;
        const int64_t cn = hyb ? A->tnnz : A->nnz;
        if (coo_row) HIPC(hipMemcpyAsync(coo_row, hyb ? A->trow : A->row, cn * 4, hipMemcpyDeviceToDevice, s));
        if (coo_col) HIPC(hipMemcpyAsync(coo_col, hyb ? A->tcol : A->col, cn * 4, hipMemcpyDeviceToDevice, s));
        if (coo_val) HIPC(hipMemcpyAsync(coo_val, hyb ? A->tval : A->val, cn * vb, hipMemcpyDeviceToDevice, s));
        c->sync();
    });
}

gko_status gko_matrix_export_sellp(gko_matrix A, int64_t *slice_sets, int32_t *slice_widths,
                                   int32_t *col, void *val) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        require(A->fmt == GKO_FMT_SELLP, GKO_ERR_INVALID_ARG, "matrix is not stored as SELL-P");
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const int64_t ns = A->slices();
        if (slice_sets)
            HIPC(hipMemcpyAsync(slice_sets, A->sset, (ns + 1) * 8, hipMemcpyDeviceToDevice, s));
        if (slice_widths)
            HIPC(hipMemcpyAsync(slice_widths, A->swidth, ns * 4, hipMemcpyDeviceToDevice, s));
        if (col) HIPC(hipMemcpyAsync(col, A->ecol, A->slots * 4, hipMemcpyDeviceToDevice, s));
        if (val) HIPC(hipMemcpyAsync(val, A->eval, A->slots * A->vs(), hipMemcpyDeviceToDevice, s));
        c->sync();
    });
}

gko_status gko_spmv(gko_matrix A, double alpha, const void *x, double beta, void *y) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        require((x || A->m == 0) && (y || A->n == 0), GKO_ERR_INVALID_ARG, "null x or y");
        const size_t vb = A->vs();
        require(!(x && y && overlap(x, A->m * vb, y, A->n * vb)), GKO_ERR_INVALID_ARG,
                "x and y must not overlap");
        spmv_dispatch(A, own_values(A), alpha, x, beta, y);
    });
}

gko_status gko_convert(gko_matrix A, gko_format fmt) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        require(fmt >= GKO_FMT_CSR && fmt <= GKO_FMT_SELLP, GKO_ERR_INVALID_ARG, "unknown format");
        if (fmt == GKO_FMT_AUTO) {
            if (A->ctx->selector) {
                convert_to(A, select_with(A, A->ctx->selector, nullptr));
            } else {
                float ms[kMlpOut];
                time_formats(A, ms, 5);
                int best = 0;
                for (int f = 1; f < kMlpOut; ++f)
                    if (ms[f] < ms[best]) best = f;
                convert_to(A, kAllFormats[best]);
            }
            return;
        }
        convert_to(A, fmt);
    });
}

gko_status gko_dot(gko_context ctx, gko_dtype dt, int64_t n, const void *x, const void *y,
                   double *result) {
    return guarded([&] {
        require(ctx && result, GKO_ERR_INVALID_ARG, "null context or result");
        require(n >= 0 && (n == 0 || (x && y)), GKO_ERR_INVALID_ARG, "bad vectors");
        require(dt == GKO_F64 || dt == GKO_F32, GKO_ERR_INVALID_ARG, "bad dtype");
        HIPC(dot(ctx->stream, dt == GKO_F64 ? vt::f64 : vt::f32, n, x, y, result, ctx->red_partials,
                 ctx->red_ticket, false));
    });
}

gko_status gko_norm2(gko_context ctx, gko_dtype dt, int64_t n, const void *x, double *result) {
    return guarded([&] {
        require(ctx && result, GKO_ERR_INVALID_ARG, "null context or result");
        require(n >= 0 && (n == 0 || x), GKO_ERR_INVALID_ARG, "bad vector");
        require(dt == GKO_F64 || dt == GKO_F32, GKO_ERR_INVALID_ARG, "bad dtype");
        HIPC(dot(ctx->stream, dt == GKO_F64 ? vt::f64 : vt::f32, n, x, x, result, ctx->red_partials,
                 ctx->red_ticket, true));
    });
}

gko_status gko_stream(gko_context ctx, gko_stream_op op, int64_t n, const double *a,
                      const double *b, double s, double *c) {
    return guarded([&] {
        require(ctx != nullptr, GKO_ERR_INVALID_ARG, "null context");
        require(op == GKO_STREAM_COPY || op == GKO_STREAM_TRIAD, GKO_ERR_INVALID_ARG, "bad op");
        require(n >= 0 && (n == 0 || (a && c && (op == GKO_STREAM_COPY || b))), GKO_ERR_INVALID_ARG,
                "bad arrays");
        HIPC(stream_op(ctx->stream, (int)op, n, a, b, s, c));
    });
}

gko_status gko_gather_probe(gko_context ctx, int64_t n, const double *x, int64_t m,
                            const int32_t *idx, double *y) {
    return guarded([&] {
        require(ctx != nullptr, GKO_ERR_INVALID_ARG, "null context");
        require(n >= 0 && m >= 1 && m < (int64_t(1) << 28), GKO_ERR_INVALID_ARG,
                "n >= 0 and 1 <= m < 2^28 required");
        require(n == 0 || (x && idx && y), GKO_ERR_INVALID_ARG, "null array");
        require((((uintptr_t)idx | (uintptr_t)y) & 15) == 0, GKO_ERR_INVALID_ARG,
                "idx and y must be 16-byte aligned");
        require(!overlap(x, size_t(m) * 8, y, size_t(n) * 8), GKO_ERR_INVALID_ARG,
                "x and y must not overlap");
        HIPC(gather_probe(ctx->stream, n, x, m, idx, y));
    });
}

gko_status gko_matrix_features(gko_matrix A, float *features) {
    return guarded([&] {
        require(A && features, GKO_ERR_INVALID_ARG, "null matrix or output");
        matrix_features(A, features);
    });
}

gko_status gko_autotune_format(gko_matrix A, gko_format *best, float *times_ms) {
    return guarded([&] {
        require(A != nullptr, GKO_ERR_INVALID_ARG, "null matrix");
        float ms[kMlpOut];
        time_formats(A, ms, 5);
        int b = 0;
        for (int f = 0; f < kMlpOut; ++f) {
            if (times_ms) times_ms[f] = ms[f];
            if (ms[f] < ms[b]) b = f;
        }
        if (best) *best = kAllFormats[b];
    });
}

gko_status gko_select_format(gko_matrix A, gko_mlp model, gko_format *out, float *scores) {
    return guarded([&] {
        require(A && model && out, GKO_ERR_INVALID_ARG, "null matrix, model or output");
        require(model->ctx == A->ctx, GKO_ERR_INVALID_ARG, "model and matrix belong to different contexts");
        *out = select_with(A, model, scores);
    });
}

gko_status gko_context_set_selector(gko_context ctx, gko_mlp model) {
    return guarded([&] {
        require(ctx != nullptr, GKO_ERR_INVALID_ARG, "null context");
        require(!model || model->ctx == ctx, GKO_ERR_INVALID_ARG, "model from another context");
        ctx->selector = model;
    });
}

gko_status gko_mlp_create(gko_context ctx, const float *params, gko_mlp *out) {
    return guarded([&] {
        require(ctx && params && out, GKO_ERR_INVALID_ARG, "null context, params or output");
        *out = new_mlp(ctx, params, nullptr);
    });
}

gko_status gko_mlp_destroy(gko_mlp M) {
    return guarded([&] {
        if (!M) return;
        if (M->ctx->selector == M) M->ctx->selector = nullptr;
        M->free_all();
        delete M;
    });
}

gko_status gko_mlp_get_params(gko_mlp M, float *params, float *norm) {
    return guarded([&] {
        require(M != nullptr, GKO_ERR_INVALID_ARG, "null model");
        hipStream_t s = M->ctx->stream;
        if (params) HIPC(hipMemcpyAsync(params, M->params, kMlpParams * 4, hipMemcpyDeviceToHost, s));
        if (norm) HIPC(hipMemcpyAsync(norm, M->norm, 2 * kMlpIn * 4, hipMemcpyDeviceToHost, s));
        M->ctx->sync();
    });
}

gko_status gko_mlp_fit_normalization(gko_mlp M, int64_t n, const float *X) {
    return guarded([&] {
        require(M && (n == 0 || X) && n >= 0, GKO_ERR_INVALID_ARG, "bad arguments");
        HIPC(mlp_norm_fit(M->ctx->stream, n, X, M->norm));
    });
}

gko_status gko_mlp_forward(gko_mlp M, int64_t n, const float *X, float *out) {
    return guarded([&] {
        require(M && n >= 0 && (n == 0 || (X && out)), GKO_ERR_INVALID_ARG, "bad arguments");
        HIPC(mlp_forward(M->ctx->stream, n, X, M->params, M->norm, out));
    });
}

gko_status gko_mlp_loss_grad(gko_mlp M, int64_t n, const float *X, const float *Y, const float *mask,
                             float *grad, double *loss) {
    return guarded([&] {
        require(M && n > 0 && X && Y && mask && grad && loss, GKO_ERR_INVALID_ARG, "bad arguments");
        hipStream_t s = M->ctx->stream;
        HIPC(mlp_mask_sum(s, n * kMlpOut, mask, M->msum));
        HIPC(mlp_grad(s, M->work(), n, X, Y, mask, M->params, M->norm, grad, loss, false, 0.f, nullptr));
    });
}

gko_status gko_mlp_train(gko_mlp M, int64_t n, const float *X, const float *Y, const float *mask,
                         int32_t steps, float lr, float *loss_history) {
    return guarded([&] {
        require(M && n > 0 && X && Y && mask && steps >= 0 && lr > 0.f, GKO_ERR_INVALID_ARG,
                "bad arguments");
        hipStream_t s = M->ctx->stream;
        HIPC(mlp_mask_sum(s, n * kMlpOut, mask, M->msum));
        int step0 = read_int(M->ctx, M->step);
        float *hist = loss_history;
        for (int32_t k = 0; k < steps; ++k)
            HIPC(mlp_grad(s, M->work(), n, X, Y, mask, M->params, M->norm, nullptr, nullptr, true, lr,
                          hist ? hist - step0 : nullptr));
        M->ctx->sync();
    });
}

gko_status gko_mlp_save(gko_mlp M, const char *path) {
    return guarded([&] {
        require(M && path, GKO_ERR_INVALID_ARG, "null model or path");
        std::vector<float> p(kMlpParams), nrm(2 * kMlpIn);
        HIPC(hipMemcpyAsync(p.data(), M->params, kMlpParams * 4, hipMemcpyDeviceToHost, M->ctx->stream));
        HIPC(hipMemcpyAsync(nrm.data(), M->norm, 2 * kMlpIn * 4, hipMemcpyDeviceToHost, M->ctx->stream));
        M->ctx->sync();
        std::ofstream f(path, std::ios::binary);
        require((bool)f, GKO_ERR_INVALID_ARG, std::string("cannot write ") + path);
        const int32_t version = 1, np = kMlpParams;
        char arch[16] = "gfx950";
        f.write(kMlpMagic, 8);
        f.write(reinterpret_cast<const char *>(&version), 4);
        f.write(reinterpret_cast<const char *>(&np), 4);
        f.write(arch, 16);
        f.write(reinterpret_cast<const char *>(nrm.data()), nrm.size() * 4);
        f.write(reinterpret_cast<const char *>(p.data()), p.size() * 4);
        require((bool)f, GKO_ERR_INVALID_ARG, std::string("write failed: ") + path);
    });
}

gko_status gko_mlp_load(gko_context ctx, const char *path, gko_mlp *out) {
    return guarded([&] {
        require(ctx && path && out, GKO_ERR_INVALID_ARG, "null context, path or output");
        *out = nullptr;
        std::ifstream f(path, std::ios::binary);
        require((bool)f, GKO_ERR_INVALID_ARG, std::string("cannot read ") + path);
        char magic[8], arch[16];
        int32_t version = 0, np = 0;
        f.read(magic, 8);
        f.read(reinterpret_cast<char *>(&version), 4);
        f.read(reinterpret_cast<char *>(&np), 4);
        f.read(arch, 16);
        require((bool)f && std::memcmp(magic, kMlpMagic, 8) == 0 && version == 1 && np == kMlpParams,
                GKO_ERR_INVALID_ARG, "not a model file of this library");
        std::vector<float> nrm(2 * kMlpIn), p(kMlpParams);
        f.read(reinterpret_cast<char *>(nrm.data()), nrm.size() * 4);
        f.read(reinterpret_cast<char *>(p.data()), p.size() * 4);
        require((bool)f, GKO_ERR_INVALID_ARG, "truncated model file");
        *out = new_mlp(ctx, p.data(), nrm.data());
    });
}

gko_status gko_context_set_solver_opts(gko_context ctx, const gko_solver_opts *o) {
    return guarded([&] {
        require(ctx && o, GKO_ERR_INVALID_ARG, "null context or options");
        require(o->precision == GKO_PREC_FP64 || o->precision == GKO_PREC_MIXED_IR,
                GKO_ERR_INVALID_ARG, "bad precision");
        require(o->precond == GKO_PRECOND_NONE || o->precond == GKO_PRECOND_BLOCK_JACOBI,
                GKO_ERR_INVALID_ARG, "bad preconditioner");
        const int bs = o->block_size;
        require(bs == 1 || bs == 2 || bs == 4 || bs == 8 || bs == 16, GKO_ERR_UNSUPPORTED,
                "block size must be 1, 2, 4, 8 or 16");
        require(o->check_every >= 1, GKO_ERR_INVALID_ARG, "check_every must be >= 1");
        require(o->inner_tol > 0.0 && o->inner_tol < 1.0, GKO_ERR_INVALID_ARG, "inner_tol in (0,1)");
        require(o->max_inner >= 1 && o->max_outer >= 1, GKO_ERR_INVALID_ARG, "iteration caps >= 1");
        require(o->krylov_dim >= 1 && o->krylov_dim <= kGmresMaxKrylov, GKO_ERR_INVALID_ARG,
                "krylov_dim must be in 1.." + std::to_string(kGmresMaxKrylov));
        require(o->single_workgroup == 0 || o->single_workgroup == 1, GKO_ERR_INVALID_ARG,
                "single_workgroup must be 0 or 1");
        require(o->graphs == 0 || o->graphs == 1, GKO_ERR_INVALID_ARG, "graphs must be 0 or 1");
        ctx->opts = *o;
    });
}

gko_status gko_context_get_solver_opts(gko_context ctx, gko_solver_opts *out) {
    return guarded([&] {
        require(ctx && out, GKO_ERR_INVALID_ARG, "null context or output");
        *out = ctx->opts;
    });
}

gko_status gko_context_get_solve_info(gko_context ctx, gko_solve_info *out) {
    return guarded([&] {
        require(ctx && out, GKO_ERR_INVALID_ARG, "null context or output");
        *out = ctx->info;
    });
}

// FP64 CG on one workgroup in one launch (the matrix's longest row known);
// the kernel leaves its counts and residuals in *res.  Fills the solve info.
static gko_status run_small_cg(gko_matrix A, const void *b, void *x, double tol, int32_t maxit,
                               small_cg_result *res, double t0) {
    gko_context c = A->ctx;
    HIPC(small_cg(c->stream, A->n, A->max_len, A->rp, A->col, static_cast<const double *>(A->val),
                  static_cast<const double *>(b), static_cast<double *>(x), tol, maxit, res));
    small_cg_result h{};
    HIPC(hipMemcpyAsync(&h, res, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    c->sync();
    const gko_status st = h.bb == 0.0 ? GKO_OK : flag_status(h.flag);
    c->info.iterations = h.iters;
    c->info.restarts = h.restarts;
    c->info.rel_residual = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    c->info.true_rel_residual = h.bb > 0 ? std::sqrt(h.tr2 / h.bb) : 0.0;
    c->info.status = st;
    c->info.seconds = now_seconds() - t0;
    return st;
}

// CG, flexible CG or pipelined CG: the same options; only CG has the
// single-workgroup path for small systems.
static gko_status cg_family_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit,
                                  cg_variant var) {
    gko_status st = GKO_OK;
    gko_status call = guarded([&] {
        check_square_f64(A);
        check_solve_args(b, x, A->n, tol, maxit);
        gko_context c = A->ctx;
        const double t0 = now_seconds();
        c->info = gko_solve_info{};
        const gko_solver_opts o = c->opts;
        const int64_t n = A->n;
        if (c->small_cg_rows < 0) c->small_cg_rows = small_cg_max_rows();
        const bool single = var == cg_variant::plain && o.single_workgroup &&
                            o.precision == GKO_PREC_FP64 &&
                            o.precond == GKO_PRECOND_NONE && n > 0 && n <= c->small_cg_rows &&
                            (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE);
        if (single) {
            if (A->max_len < 0) A->max_len = max_len_of_csr(A);
            dbuf res(c, sizeof(small_cg_result));
            st = run_small_cg(A, b, x, tol, maxit, res.as<small_cg_result>(), t0);
            return;
        }
        // ||b|| decides the trivial cases before any iteration
        dbuf partials(c, kPartialBytes), ticket(c, 8), nrm(c, 8);
        HIPC(hipMemsetAsync(ticket.p, 0, 8, c->stream));
        const double bnorm = device_norm(c, vt::f64, n, b, nrm.as<double>(), partials.as<double>(),
                                         ticket.as<unsigned>());
        if (!std::isfinite(bnorm)) {
            st = GKO_ERR_BREAKDOWN;
        } else if (bnorm == 0.0) {
            HIPC(fill_zero(c->stream, vt::f64, n, x));
            c->sync();
            st = GKO_OK;
        } else {
            const int bs = o.precond == GKO_PRECOND_BLOCK_JACOBI ? o.block_size : 0;
            if (bs > 0) {
                const double ts = now_seconds();
                ensure_block_jacobi(A, bs, o.precision == GKO_PREC_MIXED_IR);
                c->sync();
                c->info.setup_seconds = now_seconds() - ts;
            }
            if (o.precision == GKO_PREC_MIXED_IR) {
                mixed_result r = mixed_ir(A, b, x, tol, maxit, o, bs, bnorm, var);
                st = r.status;
                c->info.iterations = r.inner;
                c->info.outer_iterations = r.outer;
                c->info.rel_residual = r.true_relres;
                c->info.true_rel_residual = r.true_relres;
            } else {
                solve_result r = cg_variant_core(var, A, own_values(A), b, x, tol, maxit,
                                                 bs > 0 ? (const void *)A->bj64 : nullptr, bs,
                                                 o.check_every, true);
                st = flag_status(r.flag);
                c->info.iterations = r.iters;
                c->info.restarts = r.restarts;
                c->info.rel_residual = r.relres;
                c->info.true_rel_residual = r.true_relres;
            }
        }
        c->sync();
        c->info.status = st;
        c->info.seconds = now_seconds() - t0;
    });
    if (call != GKO_OK) {
        if (A) A->ctx->info.status = call;
        return call;
    }
    if (st != GKO_OK)
        g_last_error = std::string(var == cg_variant::plain      ? "cg: "
                                   : var == cg_variant::flexible ? "fcg: "
                                                                 : "pipecg: ") +
                       gko_status_string(st);
    return st;
}

gko_status gko_cg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return cg_family_solve(A, b, x, tol, maxit, cg_variant::plain);
}

// ---------------------------------------------------------------- CG without allocation
// Byte offsets of gko_cg_solve_noalloc's buffers in the scratch array: the
// single-workgroup result and the longest-row slot, the reduction ticket, the
// iteration scalars, a norm slot, the reduction partials, then r, p and q.
namespace {
constexpr size_t round256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaSmall = 0, kNaMaxLen = 128, kNaTicket = 256, kNaScalars = 512;
constexpr size_t kNaNorm = kNaScalars + round256(sizeof(krylov_scalars));
constexpr size_t kNaPartials = kNaNorm + 256;
constexpr size_t kNaVectors = kNaPartials + round256(kPartialBytes);
static_assert(sizeof(small_cg_result) <= kNaMaxLen, "small-CG result overlaps the max-length slot");
// each of r, p, q takes round256(8 n) bytes
constexpr int64_t kNaMaxRows = int64_t((kScratchBytes - kNaVectors) / 3 / 256 * 256 / 8);
static_assert(kNaMaxRows == GKO_CG_NOALLOC_MAX_ROWS, "header limit out of date");
static_assert(kScratchBytes == GKO_NOALLOC_SCRATCH_BYTES, "header scratch size out of date");
}  // namespace

gko_status gko_cg_solve_noalloc(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    gko_status st = GKO_OK;
    gko_status call = guarded([&] {
        check_square_f64(A);
        check_solve_args(b, x, A->n, tol, maxit);
        gko_context c = A->ctx;
        const gko_solver_opts o = c->opts;
        require(o.precision == GKO_PREC_FP64 && o.precond == GKO_PRECOND_NONE,
                GKO_ERR_UNSUPPORTED, "only FP64 CG without a preconditioner runs without allocation");
        const int64_t n = A->n;
        require(n <= kNaMaxRows, GKO_ERR_INVALID_ARG,
                "n_rows " + std::to_string(n) + " above the no-allocation limit of " +
                    std::to_string(kNaMaxRows) + " rows");
        require(c->scratch != nullptr, GKO_ERR_HIP, "scratch address not resolved");
        unsigned char *base = c->scratch;
        hipStream_t s = c->stream;
        const double t0 = now_seconds();
        c->info = gko_solve_info{};
        if (c->small_cg_rows < 0) c->small_cg_rows = small_cg_max_rows();
        if (o.single_workgroup && n > 0 && n <= c->small_cg_rows &&
            (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE)) {
            if (A->max_len < 0) {
                int *ml = reinterpret_cast<int *>(base + kNaMaxLen);
                HIPC(fill_zero(s, vt::f32, 1, ml));
                HIPC(max_row_len(s, n, A->rp, ml));
                A->max_len = read_int(c, ml);
            }
            st = run_small_cg(A, b, x, tol, maxit,
                              reinterpret_cast<small_cg_result *>(base + kNaSmall), t0);
            return;
        }
        cg_workspace w;
        w.ticket = reinterpret_cast<unsigned *>(base + kNaTicket);
        w.S = reinterpret_cast<krylov_scalars *>(base + kNaScalars);
        w.nrm = reinterpret_cast<double *>(base + kNaNorm);
        w.partials = reinterpret_cast<double *>(base + kNaPartials);
        const size_t vb = round256(size_t(n) * 8);
        w.r = base + kNaVectors;
        w.p = base + kNaVectors + vb;
        w.q = base + kNaVectors + 2 * vb;
        w.graphs = false;
        HIPC(fill_zero(s, vt::f64, 1, w.ticket));
        const double bnorm = device_norm(c, vt::f64, n, b, w.nrm, w.partials, w.ticket);
        if (!std::isfinite(bnorm)) {
            st = GKO_ERR_BREAKDOWN;
        } else if (bnorm == 0.0) {
            HIPC(fill_zero(s, vt::f64, n, x));
            st = GKO_OK;
        } else {
            solve_result r = cg_core(A, own_values(A), b, x, tol, maxit, nullptr, 0, o.check_every,
                                     true, false, w);
            st = flag_status(r.flag);
            c->info.iterations = r.iters;
            c->info.restarts = r.restarts;
            c->info.rel_residual = r.relres;
            c->info.true_rel_residual = r.true_relres;
        }
        c->sync();
        c->info.status = st;
        c->info.seconds = now_seconds() - t0;
    });
    if (call != GKO_OK) {
        if (A) A->ctx->info.status = call;
        return call;
    }
    if (st != GKO_OK) g_last_error = std::string("cg_noalloc: ") + gko_status_string(st);
    return st;
}

gko_status gko_fcg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return cg_family_solve(A, b, x, tol, maxit, cg_variant::flexible);
}

gko_status gko_pipecg_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return cg_family_solve(A, b, x, tol, maxit, cg_variant::pipelined);
}

// The frame shared by the unpreconditioned FP64 solvers without a
// single-workgroup path (BiCGSTAB, CGS, GMRES): argument checks, ||b||
// (NaN/Inf: breakdown; 0: x = 0 at zero iterations), the true relative
// residual at exit, timing and the error message.  body(bnorm, partials,
// ticket) runs the iteration, fills the solve info and returns a solver_flag.
extern "C++" {
template <typename Body>
static gko_status nonsym_solve(const char *name, gko_matrix A, const void *b, void *x, double tol,
                               int32_t maxit, Body body) {
    gko_status st = GKO_OK;
    gko_status call = guarded([&] {
        check_square_f64(A);
        check_solve_args(b, x, A->n, tol, maxit);
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const double t0 = now_seconds();
        c->info = gko_solve_info{};
        const int64_t n = A->n;
        dbuf partials(c, kPartialBytes), ticket(c, 8), nrm(c, 8);
        HIPC(hipMemsetAsync(ticket.p, 0, 8, s));
        double *P = partials.as<double>();
        unsigned *T = ticket.as<unsigned>();
        const double bnorm = device_norm(c, vt::f64, n, b, nrm.as<double>(), P, T);
        if (!std::isfinite(bnorm)) {
            st = GKO_ERR_BREAKDOWN;
        } else if (bnorm == 0.0) {
            HIPC(fill_zero(s, vt::f64, n, x));
            st = GKO_OK;
        } else {
            st = flag_status(body(bnorm, P, T));
            dbuf r(c, n * 8);
            HIPC(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
            spmv_dispatch(A, own_values(A), -1.0, x, 1.0, r.p);
            c->info.true_rel_residual = device_norm(c, vt::f64, n, r.p, nrm.as<double>(), P, T) / bnorm;
        }
        c->sync();
        c->info.status = st;
        c->info.seconds = now_seconds() - t0;
    });
    if (call != GKO_OK) {
        if (A) A->ctx->info.status = call;
        return call;
    }
    if (st != GKO_OK) g_last_error = std::string(name) + ": " + gko_status_string(st);
    return st;
}
}  // extern "C++"

gko_status gko_bicgstab_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return nonsym_solve("bicgstab", A, b, x, tol, maxit, [&](double, double *P, unsigned *T) {
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const int64_t n = A->n;
        const values v = own_values(A);
        dbuf r(c, n * 8), rh(c, n * 8), p(c, n * 8), vv(c, n * 8), sv(c, n * 8), t(c, n * 8);
        dbuf sc(c, sizeof(krylov_scalars));
        auto *S = sc.as<krylov_scalars>();
        HIPC(scalars_reset(s, S, maxit));
        HIPC(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, r.p);
        HIPC(bicg_init(s, n, b, r.p, rh.p, p.p, vv.p, tol, S, P, T));
        fused_matrix fm;
        const bool fused = fused_view(A, v, fm);
        krylov_scalars h = read_back(c, S);
        interval_graph graph(c, n);
        while (h.done == kRunning) {
            graph.run([&] {
                const hipStream_t st = c->stream;
                for (int j = 0; j < c->opts.check_every; ++j) {
                    HIPC(bicg_p(st, n, r.p, vv.p, p.p, S));
                    if (fused) {
                        HIPC(bicg_spmv_alpha(st, fm, p.p, vv.p, rh.p, S, P, T));
                    } else {
                        spmv_dispatch(A, v, 1.0, p.p, 0.0, vv.p);
                        HIPC(bicg_alpha(st, n, rh.p, vv.p, S, P, T));
                    }
                    HIPC(bicg_s(st, n, r.p, vv.p, sv.p, S, P, T));
                    if (fused) {
                        HIPC(bicg_spmv_omega(st, fm, sv.p, t.p, S, P, T));
                    } else {
                        spmv_dispatch(A, v, 1.0, sv.p, 0.0, t.p);
                        HIPC(bicg_omega(st, n, t.p, sv.p, S, P, T));
                    }
                    HIPC(bicg_update(st, n, x, r.p, rh.p, p.p, sv.p, t.p, S, P, T));
                }
            });
            h = read_back(c, S);
        }
        c->info.iterations = h.iter;
        c->info.rel_residual = std::sqrt(h.rr / h.bb);
        return h.done;
    });
}

gko_status gko_cgs_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return nonsym_solve("cgs", A, b, x, tol, maxit, [&](double, double *P, unsigned *T) {
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const int64_t n = A->n;
        const values v = own_values(A);
        dbuf r(c, n * 8), rh(c, n * 8), p(c, n * 8), u(c, n * 8), q(c, n * 8), w(c, n * 8),
            t(c, n * 8);
        dbuf sc(c, sizeof(krylov_scalars));
        auto *S = sc.as<krylov_scalars>();
        HIPC(scalars_reset(s, S, maxit));
        HIPC(hipMemcpyAsync(r.p, b, n * 8, hipMemcpyDeviceToDevice, s));
        spmv_dispatch(A, v, -1.0, x, 1.0, r.p);
        HIPC(cgs_init(s, n, b, r.p, rh.p, p.p, u.p, tol, S, P, T));
        fused_matrix fm;
        const bool fused = fused_view(A, v, fm);
        krylov_scalars h = read_back(c, S);
        interval_graph graph(c, n);
        while (h.done == kRunning) {
            graph.run([&] {
                const hipStream_t st = c->stream;
                for (int j = 0; j < c->opts.check_every; ++j) {
                    if (fused) {
                        HIPC(cgs_spmv_alpha(st, fm, p.p, t.p, rh.p, S, P, T));
                    } else {
                        spmv_dispatch(A, v, 1.0, p.p, 0.0, t.p);
                        HIPC(cgs_alpha(st, n, t.p, rh.p, S, P, T));
                    }
                    HIPC(cgs_qwx(st, n, u.p, t.p, q.p, w.p, x, S));
                    spmv_dispatch(A, v, 1.0, w.p, 0.0, t.p);
                    HIPC(cgs_update(st, n, r.p, t.p, rh.p, S, P, T));
                    HIPC(cgs_direction(st, n, r.p, q.p, u.p, p.p, S));
                }
            });
            h = read_back(c, S);
        }
        c->info.iterations = h.iter;
        c->info.rel_residual = std::sqrt(h.rr / h.bb);
        return h.done;
    });
}

gko_status gko_gmres_solve(gko_matrix A, const void *b, void *x, double tol, int32_t maxit) {
    return nonsym_solve("gmres", A, b, x, tol, maxit, [&](double bnorm, double *, unsigned *) {
        gko_context c = A->ctx;
        hipStream_t s = c->stream;
        const int64_t n = A->n;
        const int m = c->opts.krylov_dim;
        const int check_every = c->opts.check_every;
        const values v = own_values(A);
        const int64_t ldv = gmres_ld(n);
        dbuf V(c, (size_t)(m + 1) * ldv * 8);
        if (c->opts.single_workgroup && n <= gmres_small_max_rows() && m <= kGmresSmallKrylov &&
            (A->fmt == GKO_FMT_CSR || A->fmt == GKO_FMT_CSR_MERGE)) {
            // the whole solve on one workgroup, one launch
            dbuf state(c, sizeof(gmres_state));
            auto *S = state.as<gmres_state>();
            HIPC(gmres_small(s, n, m, A->rp, A->col, static_cast<const double *>(v.val),
                             static_cast<const double *>(b), static_cast<double *>(x), V.as<double>(),
                             ldv, tol * bnorm, maxit, S));
            gmres_state h{};
            HIPC(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, s));
            c->sync();
            c->info.iterations = h.iter;
            c->info.outer_iterations = h.cycles;
            c->info.reorthogonalized = h.reorths;
            c->info.rel_residual = h.est / bnorm;
            return h.done;
        }
        // work arrays carved from one buffer
        const int64_t np = gmres_partial_elems(n, m);
        const int64_t sizes[] = {np, m + 2, m + 2, 1, 1, m + 1, (int64_t)(m + 1) * m, m, m,
                                 m + 1, m};
        int64_t total = 0;
        for (int64_t z : sizes) total += z;
        dbuf work(c, total * 8), state(c, sizeof(gmres_state));
        double *q = work.as<double>();
        gmres_work wk;
        double **slots[] = {&wk.partials, &wk.dot1, &wk.dot2, &wk.upd1, &wk.upd2, &wk.hcol,
                            &wk.H,        &wk.cs,   &wk.sn,   &wk.g,    &wk.y};
        static_assert(std::size(sizes) == std::size(slots), "one size per work array");
        for (size_t i = 0; i < std::size(slots); ++i) {
            *slots[i] = q;
            q += sizes[i];
        }
        HIPC(fill_zero(s, vt::f64, total, work.p));
        gmres_state h{};
        h.stop = tol * bnorm;
        h.maxit = maxit;
        h.done = kRunning;
        h.cycle_done = 1;
        auto *S = state.as<gmres_state>();
        HIPC(hipMemcpyAsync(S, &h, sizeof(h), hipMemcpyHostToDevice, s));
        c->sync();   // h is reused as the read-back buffer below
        double *V0 = V.as<double>();
        for (;;) {
            HIPC(hipMemcpyAsync(V0, b, n * 8, hipMemcpyDeviceToDevice, s));
            spmv_dispatch(A, v, -1.0, x, 1.0, V0);
            HIPC(gmres_cycle_start(s, n, V0, S, wk));
            HIPC(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, s));
            c->sync();
            if (h.done != kRunning) break;
            for (int j = 0; j < m; ++j) {
                spmv_dispatch(A, v, 1.0, V0 + (int64_t)j * ldv, 0.0, V0 + (int64_t)(j + 1) * ldv);
                HIPC(gmres_arnoldi_step(s, n, m, j, V0, ldv, S, wk));
                if ((j + 1) % check_every == 0 && j + 1 < m) {
                    HIPC(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, s));
                    c->sync();
                    if (h.cycle_done) break;
                }
            }
            HIPC(gmres_cycle_end(s, n, m, V0, ldv, static_cast<double *>(x), S, wk));
            HIPC(hipMemcpyAsync(&h, S, sizeof(h), hipMemcpyDeviceToHost, s));
            c->sync();
            if (h.done != kRunning) break;   // breakdown inside the cycle
        }
        c->info.iterations = h.iter;
        c->info.outer_iterations = h.cycles;
        c->info.reorthogonalized = h.reorths;
        c->info.rel_residual = h.est / bnorm;
        return h.done;
    });
}

}  // extern "C"
