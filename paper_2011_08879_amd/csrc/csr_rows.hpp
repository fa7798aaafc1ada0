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

}  // namespace gko
