// SpMV for ELL (and the ELL part of HYB): slots stored column-major, so
// neighbouring threads reading slot j of neighbouring rows touch consecutive
// addresses -- every load of the kernel is coalesced and there is no
// cross-lane reduction.  Padding slots (col = -1) come last in a row, so a
// row stops at its first padding slot.
#include "device.hpp"
#include "ell_rows.hpp"
#include "kernels.hpp"

namespace gko {

constexpr int kEllBlock = 256;

template <typename V>
__global__ __launch_bounds__(kEllBlock) void spmv_ell_kernel(int64_t n, int64_t K, int64_t ld,
                                                             const int32_t *__restrict__ ecol,
                                                             const V *__restrict__ eval,
                                                             const V *__restrict__ x, V alpha,
                                                             V beta, V *__restrict__ y) {
    // Up to kXcdRowsMax rows each XCD takes one contiguous range of rows, so
    // the x lines that neighbouring rows share are fetched into one L2.
    const int64_t i = 2 * (row_block_order(n) * kEllBlock + threadIdx.x);
    if (i >= n) return;
    V s0, s1;
    ell_pair_rows(K, ld, i, ecol, eval, x, s0, s1);
    y[i] = (beta == V(0)) ? alpha * s0 : alpha * s0 + beta * y[i];
    if (i + 1 < n) y[i + 1] = (beta == V(0)) ? alpha * s1 : alpha * s1 + beta * y[i + 1];
}

template <typename V>
static hipError_t launch_ell(hipStream_t s, int64_t n, int64_t K, int64_t ld, const int32_t *ecol,
                             const void *eval, const void *x, double alpha, double beta, void *y) {
    const int64_t pairs = (n + 1) / 2;
    spmv_ell_kernel<V><<<dim3((unsigned)((pairs + kEllBlock - 1) / kEllBlock)), dim3(kEllBlock), 0, s>>>(
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
