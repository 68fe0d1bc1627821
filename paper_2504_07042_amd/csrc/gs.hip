// Gather-scatter: the binary matrix Q of Sec. 2.1 and its transpose, which assemble the global
// operator A = Q^T blockdiag(A_e) Q of Eq. (1).  Q^T is a segmented sum over the CSR inverse of
// the local-to-global map, taken in ascending local id by one thread per global node: no atomics,
// so the result is deterministic and independent of the launch shape.
#include <vector>

#include "ax_internal.h"
#include "gs_impl.h"

namespace ax {

// Column c = blockIdx.y; each thread takes kUnroll nodes per tile (stride 256) so that their
// loads are in flight together.

template <typename T, typename IP>
__global__ void __launch_bounds__(256)
gs_qt_kernel(int64_t n_local, int64_t n_global, const IP* __restrict__ gptr,
             const int32_t* __restrict__ gidx, const uint8_t* __restrict__ mask,
             const T* __restrict__ in, T* __restrict__ out)
{
    const int c = blockIdx.y;
    const T* x = in + (int64_t)c * n_local;
    T* o = out + (int64_t)c * n_global;
    for (int64_t g0 = xcd_tile(blockIdx.x, gridDim.x) * 256 * kUnroll + threadIdx.x; g0 < n_global;
         g0 += (int64_t)gridDim.x * 256 * kUnroll) {
        T s[kUnroll];
        int64_t g[kUnroll];
        bool ok[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            g[u] = g0 + u * 256;
            ok[u] = g[u] < n_global;
        }
        gather_sums<kUnroll>(gptr, gidx, x, g, ok, s);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (ok[u]) o[g[u]] = (mask && mask[g[u]]) ? T(0) : s[u];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
gs_q_kernel(int64_t n_local, int64_t n_global, const int32_t* __restrict__ l2g,
            const T* __restrict__ in, T* __restrict__ out)
{
    const int c = blockIdx.y;
    const T* x = in + (int64_t)c * n_global;
    T* o = out + (int64_t)c * n_local;
    for (int64_t l0 = xcd_tile(blockIdx.x, gridDim.x) * 256 * kUnroll + threadIdx.x; l0 < n_local;
         l0 += (int64_t)gridDim.x * 256 * kUnroll) {
        int32_t id[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) id[u] = l0 + u * 256 < n_local ? l2g[l0 + u * 256] : 0;
        T v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[u] = x[id[u]];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (l0 + u * 256 < n_local) o[l0 + u * 256] = v[u];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
gs_qqt_kernel(int64_t n_local, const int32_t* __restrict__ l2g, const int64_t* __restrict__ gptr,
              const int32_t* __restrict__ gidx, const uint8_t* __restrict__ mask, const T* __restrict__ in,
              T* __restrict__ out)
{
    const int c = blockIdx.y;
    const T* x = in + (int64_t)c * n_local;
    T* o = out + (int64_t)c * n_local;
    for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < n_local; l += (int64_t)gridDim.x * 256) {
        const int64_t g = l2g[l];
        const bool ok = true;
        T s;
        gather_sums<1>(gptr, gidx, x, &g, &ok, &s);
        o[l] = (mask && mask[g]) ? T(0) : s;
    }
}

static unsigned gs_grid(int64_t n, int per_thread)
{
    const int64_t b = (n + 256LL * per_thread - 1) / (256LL * per_thread);
    return (unsigned)(b < 65535 ? (b > 0 ? b : 1) : 65535);
}

template <typename T>
static int gs_launch(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
                     const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, const void* in,
                     void* out, hipStream_t st)
{
    switch (mode) {
    case GS_QT:
        hipLaunchKernelGGL((gs_qt_kernel<T, int64_t>), dim3(gs_grid(n_global, kUnroll), nrhs), dim3(256), 0, st,
                           n_local, n_global, gptr, gidx, mask, (const T*)in, (T*)out);
        break;
    case GS_Q:
        hipLaunchKernelGGL(gs_q_kernel<T>, dim3(gs_grid(n_local, kUnroll), nrhs), dim3(256), 0, st, n_local,
                           n_global, l2g, (const T*)in, (T*)out);
        break;
    default:
        hipLaunchKernelGGL(gs_qqt_kernel<T>, dim3(gs_grid(n_local, 1), nrhs), dim3(256), 0, st, n_local, l2g, gptr,
                           gidx, mask, (const T*)in, (T*)out);
        break;
    }
    return hip_check(hipGetLastError(), "gs_assemble launch");
}

// Entry used by the solver (no re-validation).
int gs_apply(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
             const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, int dtype, const void* in,
             void* out, hipStream_t st)
{
    if (dtype == AX_FP64) return gs_launch<double>(n_local, n_global, l2g, gptr, gidx, mask, mode, nrhs, in, out, st);
    return gs_launch<float>(n_local, n_global, l2g, gptr, gidx, mask, mode, nrhs, in, out, st);
}

}  // namespace ax

using namespace ax;

extern "C" int gs_build_csr(int64_t n_local, int64_t n_global, const int32_t* l2g, int64_t* gptr,
                            int32_t* gidx)
{
    clear_error();
    if (n_local < 0 || n_global < 0) return fail(AX_ERR_ARG, "negative size");
    if (n_local > 0x7fffffffLL) return fail(AX_ERR_UNSUPPORTED, "n_local exceeds int32 local ids");
    if (!gptr || (n_local > 0 && (!l2g || !gidx))) return fail(AX_ERR_ARG, "NULL pointer");
    for (int64_t g = 0; g <= n_global; ++g) gptr[g] = 0;
    for (int64_t l = 0; l < n_local; ++l) {
        const int32_t g = l2g[l];
        if (g < 0 || g >= n_global) return fail(AX_ERR_ARG, "l2g[%lld]=%d out of range", (long long)l, g);
        gptr[g + 1]++;
    }
    for (int64_t g = 0; g < n_global; ++g) gptr[g + 1] += gptr[g];
    std::vector<int64_t> fill(gptr, gptr + n_global);
    for (int64_t l = 0; l < n_local; ++l) gidx[fill[l2g[l]]++] = (int32_t)l;  // ascending l
    return AX_OK;
}

extern "C" int gs_assemble(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
                           const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, int dtype,
                           const void* in, void* out, void* stream)
{
    clear_error();
    if (n_local < 0 || n_global < 0) return fail(AX_ERR_ARG, "negative size");
    if (nrhs < 1 || nrhs > 65535) return fail(AX_ERR_ARG, "nrhs outside [1, 65535]");
    if (mode != GS_QT && mode != GS_Q && mode != GS_QQT) return fail(AX_ERR_UNSUPPORTED, "unknown mode %d", mode);
    if (dtype != AX_FP64 && dtype != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "dtype must be FP64 or FP32");
    if (n_local == 0 && n_global == 0) return AX_OK;
    if (!in || !out) return fail(AX_ERR_ARG, "in or out is NULL");
    if (in == out) return fail(AX_ERR_ARG, "in and out alias");
    if (mode != GS_Q && (!gptr || !gidx)) return fail(AX_ERR_ARG, "CSR arrays are NULL");
    if (mode != GS_QT && !l2g) return fail(AX_ERR_ARG, "l2g is NULL");
    return gs_apply(n_local, n_global, l2g, gptr, gidx, mask, mode, nrhs, dtype, in, out, as_stream(stream));
}
