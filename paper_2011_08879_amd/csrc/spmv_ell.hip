// SpMV for ELL (and the ELL part of HYB): slots stored column-major, so
// thread i reading slot j of row i and thread i+1 reading slot j of row i+1
// touch consecutive addresses -- every load of the kernel is coalesced and
// there is no cross-lane reduction.  Padding slots (col = -1) come last in a
// row, so a thread stops at its row's first padding slot.
#include "device.hpp"
#include "kernels.hpp"

namespace gko {

constexpr int kEllBlock = 256;

template <typename V>
__global__ __launch_bounds__(kEllBlock) void spmv_ell_kernel(int64_t n, int64_t K, int64_t ld,
                                                             const int32_t *__restrict__ ecol,
                                                             const V *__restrict__ eval,
                                                             const V *__restrict__ x, V alpha,
                                                             V beta, V *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * kEllBlock + threadIdx.x;
    if (i >= n) return;
    V s = V(0);
    const int32_t *c = ecol + i;
    const V *v = eval + i;
    int64_t j = 0;
    // four slots per step, loads issued before use
    for (; j + 4 <= K; j += 4) {
        const int32_t c0 = load_stream(c + (j + 0) * ld), c1 = load_stream(c + (j + 1) * ld);
        const int32_t c2 = load_stream(c + (j + 2) * ld), c3 = load_stream(c + (j + 3) * ld);
        const V v0 = load_stream(v + (j + 0) * ld), v1 = load_stream(v + (j + 1) * ld);
        const V v2 = load_stream(v + (j + 2) * ld), v3 = load_stream(v + (j + 3) * ld);
        if (c0 >= 0) s += v0 * x[c0];
        if (c1 >= 0) s += v1 * x[c1];
        if (c2 >= 0) s += v2 * x[c2];
        if (c3 >= 0) s += v3 * x[c3];
        if (c3 < 0) break;
    }
    if (j + 4 > K)
        for (; j < K; ++j) {
            const int32_t cj = c[j * ld];
            if (cj < 0) break;
            s += v[j * ld] * x[cj];
        }
    y[i] = (beta == V(0)) ? alpha * s : alpha * s + beta * y[i];
}

template <typename V>
static hipError_t launch_ell(hipStream_t s, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                             const void *eval, const void *x, double alpha, double beta, void *y) {
    spmv_ell_kernel<V><<<dim3((unsigned)((n + kEllBlock - 1) / kEllBlock)), dim3(kEllBlock), 0, s>>>(
        n, K, ld, ecol, static_cast<const V *>(eval), static_cast<const V *>(x), (V)alpha, (V)beta,
        static_cast<V *>(y));
    return hipGetLastError();
}

hipError_t spmv_ell(hipStream_t s, vt t, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                    const void *eval, const void *x, double alpha, double beta, void *y) {
    if (n == 0) return hipSuccess;
    return t == vt::f64 ? launch_ell<double>(s, n, K, ld, ecol, eval, x, alpha, beta, y)
                        : launch_ell<float>(s, n, K, ld, ecol, eval, x, alpha, beta, y);
}

}  // namespace gko
