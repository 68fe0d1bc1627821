// Machine probes for the time-based roofline (Sec. 3.4): T_mem divides the kernel's memory
// traffic by the MEASURED bandwidth and T_cmp its flops by the peak of the units that execute
// them (the paper lists measured bandwidths beside the theoretical ones, Table 4).  These kernels
// measure, on the device they run on, the sustained HBM copy bandwidth and the sustained
// arithmetic rate of each execution path the AxLocal kernels could use: FP64 and FP32 fused
// multiply-add on the vector ALU (FP32 as this library is built: without packed FP32
// instructions) and on the matrix cores, and FP64 vector and matrix work issued together (to show
// whether the two overlap).  The caller times the launches.
#include <algorithm>
#include <type_traits>

#include "ax_internal.h"

namespace ax {

typedef double probe_d4 __attribute__((ext_vector_type(4)));
typedef float probe_f4 __attribute__((ext_vector_type(4)));

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;     // independent FMA chains per thread
constexpr int kProbeUnroll = 8;     // FMA steps per chain per iteration
constexpr int kProbeMfmaChains = 4; // independent MFMA accumulators per wave

// dst = src, 16 bytes per lane per step, grid-stride.
__global__ void __launch_bounds__(kProbeBlock)
probe_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, int64_t n16)
{
    for (int64_t q = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x; q < n16; q += (int64_t)gridDim.x * kProbeBlock)
        dst[q] = src[q];
}

// VALU: kProbeChains independent chains of kProbeUnroll fused multiply-adds per iteration.
// MFMA: kProbeMfmaChains independent 16x16x4 accumulations per iteration.  The result is stored
// so the work cannot be removed.
template <typename T, bool VALU, bool MFMA>
__global__ void __launch_bounds__(kProbeBlock)
probe_compute_kernel(T* __restrict__ out, int iters)
{
    T v[kProbeChains];
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) v[q] = T(1) + T(1e-3) * T(threadIdx.x + q);
    using V4 = typename std::conditional<sizeof(T) == 8, probe_d4, probe_f4>::type;
    V4 acc[kProbeMfmaChains];
#pragma unroll
    for (int q = 0; q < kProbeMfmaChains; ++q) acc[q] = V4{T(0), T(0), T(0), T(0)};
    const T a = T(1) + T(threadIdx.x) * T(1e-6), b = T(0.5);
    for (int it = 0; it < iters; ++it) {
        if constexpr (MFMA) {
#pragma unroll
            for (int q = 0; q < kProbeMfmaChains; ++q) {
                if constexpr (sizeof(T) == 8)
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[q], 0, 0, 0);
                else
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[q], 0, 0, 0);
            }
        }
        if constexpr (VALU) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
                for (int q = 0; q < kProbeChains; ++q) v[q] = fma(v[q], T(0.9999999), T(1e-9));
        }
    }
    T s = T(0);
#pragma unroll
    for (int q = 0; q < kProbeChains; ++q) s += v[q];
#pragma unroll
    for (int q = 0; q < kProbeMfmaChains; ++q) s += acc[q][0] + acc[q][1] + acc[q][2] + acc[q][3];
    out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = s;
}

static int probe_grid()
{
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus * 8;  // 32 waves per CU
}

}  // namespace ax

using namespace ax;

extern "C" int ax_probe_copy(const void* src, void* dst, size_t bytes, void* stream)
{
    clear_error();
    if (bytes == 0) return AX_OK;
    if (!src || !dst) return fail(AX_ERR_ARG, "src or dst is NULL");
    if (src == dst) return fail(AX_ERR_ARG, "src and dst alias");
    if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16)
        return fail(AX_ERR_ARG, "bytes and both pointers must be multiples of 16");
    const int64_t n16 = (int64_t)(bytes / 16);
    const int64_t want = (n16 + kProbeBlock - 1) / kProbeBlock;
    const unsigned grid = (unsigned)std::min<int64_t>(want, (int64_t)probe_grid() * 4);
    hipLaunchKernelGGL(probe_copy_kernel, dim3(grid), dim3(kProbeBlock), 0, as_stream(stream),
                       (const uint4*)src, (uint4*)dst, n16);
    return hip_check(hipGetLastError(), "probe copy launch");
}

extern "C" int ax_probe_compute_elems(size_t* n)
{
    clear_error();
    if (!n) return fail(AX_ERR_ARG, "n is NULL");
    *n = (size_t)probe_grid() * kProbeBlock;
    return AX_OK;
}

extern "C" int ax_probe_compute(int kind, int iters, void* out, double* flops, void* stream)
{
    clear_error();
    if (!out || !flops) return fail(AX_ERR_ARG, "out or flops is NULL");
    if (iters < 1) return fail(AX_ERR_ARG, "iters < 1");
    const int grid = probe_grid();
    const double threads = (double)grid * kProbeBlock, waves = threads / 64.0;
    const double valu = threads * iters * kProbeChains * kProbeUnroll * 2.0;
    const double mfma = waves * iters * kProbeMfmaChains * 2.0 * 16 * 16 * 4;
    hipStream_t st = as_stream(stream);
    switch (kind) {
    case AX_PROBE_FMA_F64:
        hipLaunchKernelGGL((probe_compute_kernel<double, true, false>), dim3(grid), dim3(kProbeBlock), 0, st,
                           (double*)out, iters);
        *flops = valu;
        break;
    case AX_PROBE_FMA_F32:
        hipLaunchKernelGGL((probe_compute_kernel<float, true, false>), dim3(grid), dim3(kProbeBlock), 0, st,
                           (float*)out, iters);
        *flops = valu;
        break;
    case AX_PROBE_MFMA_F64:
        hipLaunchKernelGGL((probe_compute_kernel<double, false, true>), dim3(grid), dim3(kProbeBlock), 0, st,
                           (double*)out, iters);
        *flops = mfma;
        break;
    case AX_PROBE_MFMA_F32:
        hipLaunchKernelGGL((probe_compute_kernel<float, false, true>), dim3(grid), dim3(kProbeBlock), 0, st,
                           (float*)out, iters);
        *flops = mfma;
        break;
    case AX_PROBE_MIX_F64:
        hipLaunchKernelGGL((probe_compute_kernel<double, true, true>), dim3(grid), dim3(kProbeBlock), 0, st,
                           (double*)out, iters);
        *flops = valu + mfma;
        break;
    default:
        return fail(AX_ERR_ARG, "unknown probe kind %d", kind);
    }
    return hip_check(hipGetLastError(), "probe launch");
}
