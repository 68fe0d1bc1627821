// Gather-scatter: the binary matrix Q of Sec. 2.1 and its transpose, which assemble the global
// operator A = Q^T blockdiag(A_e) Q of Eq. (1).  Q^T is a segmented sum over the CSR inverse of
// the local-to-global map, taken in ascending local id by one thread per global node: no atomics,
// so the result is deterministic and independent of the launch shape.
#include <vector>

#include "ax_internal.h"

namespace ax {

template <typename T>
__global__ void __launch_bounds__(256)
gs_qt_kernel(int64_t n_local, int64_t n_global, int nrhs, const int64_t* __restrict__ gptr,
             const int32_t* __restrict__ gidx, const uint8_t* __restrict__ mask,
             const T* __restrict__ in, T* __restrict__ out)
{
    const int64_t total = n_global * nrhs;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / n_global, g = q - c * n_global;
        const T* x = in + c * n_local;
        T s = T(0);
        for (int64_t p = gptr[g]; p < gptr[g + 1]; ++p) s += x[gidx[p]];
        out[q] = (mask && mask[g]) ? T(0) : s;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
gs_q_kernel(int64_t n_local, int64_t n_global, int nrhs, const int32_t* __restrict__ l2g,
            const T* __restrict__ in, T* __restrict__ out)
{
    const int64_t total = n_local * nrhs;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / n_local, l = q - c * n_local;
        out[q] = in[c * n_global + l2g[l]];
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
gs_qqt_kernel(int64_t n_local, int nrhs, const int32_t* __restrict__ l2g,
              const int64_t* __restrict__ gptr, const int32_t* __restrict__ gidx,
              const uint8_t* __restrict__ mask, const T* __restrict__ in, T* __restrict__ out)
{
    const int64_t total = n_local * nrhs;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / n_local, l = q - c * n_local;
        const int32_t g = l2g[l];
        const T* x = in + c * n_local;
        T s = T(0);
        for (int64_t p = gptr[g]; p < gptr[g + 1]; ++p) s += x[gidx[p]];
        out[q] = (mask && mask[g]) ? T(0) : s;
    }
}

static unsigned gs_grid(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <typename T>
static int gs_launch(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
                     const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, const void* in,
                     void* out, hipStream_t st)
{
    switch (mode) {
    case GS_QT:
        hipLaunchKernelGGL(gs_qt_kernel<T>, dim3(gs_grid(n_global * nrhs)), dim3(256), 0, st, n_local,
                           n_global, nrhs, gptr, gidx, mask, (const T*)in, (T*)out);
        break;
    case GS_Q:
        hipLaunchKernelGGL(gs_q_kernel<T>, dim3(gs_grid(n_local * nrhs)), dim3(256), 0, st, n_local,
                           n_global, nrhs, l2g, (const T*)in, (T*)out);
        break;
    default:
        hipLaunchKernelGGL(gs_qqt_kernel<T>, dim3(gs_grid(n_local * nrhs)), dim3(256), 0, st, n_local,
                           nrhs, l2g, gptr, gidx, mask, (const T*)in, (T*)out);
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
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs < 1");
    if (mode != GS_QT && mode != GS_Q && mode != GS_QQT) return fail(AX_ERR_UNSUPPORTED, "unknown mode %d", mode);
    if (dtype != AX_FP64 && dtype != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "dtype must be FP64 or FP32");
    if (n_local == 0 && n_global == 0) return AX_OK;
    if (!in || !out) return fail(AX_ERR_ARG, "in or out is NULL");
    if (in == out) return fail(AX_ERR_ARG, "in and out alias");
    if (mode != GS_Q && (!gptr || !gidx)) return fail(AX_ERR_ARG, "CSR arrays are NULL");
    if (mode != GS_QT && !l2g) return fail(AX_ERR_ARG, "l2g is NULL");
    return gs_apply(n_local, n_global, l2g, gptr, gidx, mask, mode, nrhs, dtype, in, out, as_stream(stream));
}
