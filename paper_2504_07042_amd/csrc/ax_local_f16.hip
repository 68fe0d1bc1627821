// AxLocal with half-precision contraction operands and float accumulation on the gfx950
// matrix cores (v_mfma_f32_16x16x16_f16), for the inner operator of mixed-precision CG.
//
// Storage of X and Y is float.  Per element, X is scaled by a power of two so that |X| < 1 and
// rounded to half; the six D-contractions run on the matrix cores with float accumulation; the
// geometric factors (trilinear: Sec. 3.3 / Algorithm 2, parallelepiped: Algorithm 3, or stored)
// and the pointwise products stay in float (the factors would underflow in half); r, s, t are
// rescaled by a power of two before they are rounded to half for the transposed contractions.
// Power-of-two scalings are exact, so they only move the operands into half's normal range.
//
// Matrix-core formulation (N1 = 8): a contraction along one index is D (8x8) times an 8 x 64
// matrix whose columns are the 64 lines of the element along that index.  The 16x16x16 shape
// takes A = blockdiag(D, D) and a B whose two 8-row halves hold two different groups of 16
// lines, so one instruction contracts 32 lines and two cover the element.  Lane l supplies
// B[4(l/16) + q][l % 16], i.e. four consecutive points of one line, and receives the result at
// the same four points, so no re-layout is needed between input and output of a contraction.
#include "ax_internal.h"
#include "geom.h"

namespace ax {

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

enum { F16_TRI = 0, F16_PARA = 1, F16_STORED = 2 };

struct BasisF16 {
    float D[64];  // D[a * 8 + n]
    double xi[8];
    double w[8];
};

// node index of point `idx` on line `col` for a contraction along direction dir (0: r/i, 1: s/j,
// 2: t/k); lines are numbered by the two remaining indices, fastest first.
__device__ __forceinline__ int f16_node(int dir, int idx, int col)
{
    if (dir == 0) return idx + 8 * col;
    if (dir == 1) return (col & 7) + 8 * idx + 64 * (col >> 3);
    return col + 64 * idx;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// exponent e with |v| < 2^e for v = max |.| (0 -> 0)
__device__ __forceinline__ int pow2_bound(float m)
{
    int e = 0;
    if (m > 0.0f) frexpf(m, &e);
    return e;
}

// out[node] (float, LDS) = contraction of the half field `in` (LDS) along dir with A fragments
// a_frag; ACC: add to out instead of storing.
template <bool ACC>
__device__ __forceinline__ void f16_contract(const _Float16* __restrict__ in, float* __restrict__ out,
                                             int dir, half4_t afrag, int l)
{
    const int hb = (l >> 4) & 1;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int col = 32 * g + 16 * (l >> 5) + (l & 15);
        half4_t b;
#pragma unroll
        for (int q = 0; q < 4; ++q) b[q] = in[f16_node(dir, 4 * hb + q, col)];
        float4_t c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x16f16(afrag, b, c, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int nd = f16_node(dir, 4 * hb + q, col);
            if (ACC)
                out[nd] += c[q];
            else
                out[nd] = c[q];
        }
    }
}

template <int GEO>
__global__ void __launch_bounds__(64)
ax_local_f16_kernel(int64_t E, int nrhs, const double* __restrict__ geo, const float* __restrict__ Gs,
                    const float* __restrict__ X, float* __restrict__ Y, const BasisF16 bs)
{
    constexpr int NP = 512;
    __shared__ _Float16 hx[3][NP];  // X, then r, s, t (half)
    __shared__ float fb[3][NP];     // x0, x1, x2, then the accumulated output
    __shared__ double sv[24];
    lds_poison(hx, sizeof(hx));
    lds_poison(fb, sizeof(fb));
    lds_poison(sv, sizeof(sv));
    const int l = threadIdx.x;
    const int i = l & 7, j = l >> 3;

    // A fragments: blockdiag(D, D) and blockdiag(D^T, D^T); lane l holds A[l % 16][4 (l/16) + q]
    half4_t aD, aDT;
    {
        const int m = l & 15;
        const bool on = (m >> 3) == (l >> 5);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 4 * ((l >> 4) & 1) + q;
            aD[q] = (_Float16)(on ? bs.D[(m & 7) * 8 + k] : 0.0f);
            aDT[q] = (_Float16)(on ? bs.D[k * 8 + (m & 7)] : 0.0f);
        }
    }

    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        TriCoef tc;
        float h[6];
        if constexpr (GEO == F16_TRI) {
            if (l < 24) sv[l] = geo[e * 24 + l];
            __syncthreads();
            tri_prelude([&](int v, int q) { return sv[v * 3 + q]; }, bs.xi[i], bs.xi[j], bs.w[i], bs.w[j], tc);
        } else if constexpr (GEO == F16_PARA) {
            const double wij = bs.w[i] * bs.w[j];
#pragma unroll
            for (int q = 0; q < 6; ++q) h[q] = (float)(geo[e * 6 + q] * wij);
        }
        for (int c = 0; c < nrhs; ++c) {
            const float* x = X + ((int64_t)c * E + e) * NP;
            float xr[8];
            float mx = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                xr[k] = x[l + 64 * k];
                mx = fmaxf(mx, fabsf(xr[k]));
            }
            const int ex = pow2_bound(wave_max(mx));
#pragma unroll
            for (int k = 0; k < 8; ++k) hx[0][l + 64 * k] = (_Float16)ldexpf(xr[k], -ex);
            __syncthreads();
            f16_contract<false>(hx[0], fb[0], 0, aD, l);  // x0 = D_r x
            f16_contract<false>(hx[0], fb[1], 1, aD, l);  // x1 = D_s x
            f16_contract<false>(hx[0], fb[2], 2, aD, l);  // x2 = D_t x
            __syncthreads();
            float rr[8], ss[8], tt[8];
            float mr = 0.0f;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int nd = l + 64 * k;
                float x0 = fb[0][nd], x1 = fb[1][nd], x2 = fb[2][nd];
                float g[6];
                if constexpr (GEO == F16_TRI) {
                    float lam;
                    tri_adj<float>(tc, (float)bs.xi[k], (float)bs.w[k], g, lam);
                    x0 *= lam;
                    x1 *= lam;
                    x2 *= lam;
                } else if constexpr (GEO == F16_PARA) {
                    const float wk = (float)bs.w[k];
#pragma unroll
                    for (int q = 0; q < 6; ++q) g[q] = h[q] * wk;
                } else {
                    const float* ge = Gs + e * 6 * NP + nd;
#pragma unroll
                    for (int q = 0; q < 6; ++q) g[q] = ge[q * NP];
                }
                rr[k] = fmaf(g[0], x0, fmaf(g[1], x1, g[2] * x2));
                ss[k] = fmaf(g[1], x0, fmaf(g[3], x1, g[4] * x2));
                tt[k] = fmaf(g[2], x0, fmaf(g[4], x1, g[5] * x2));
                mr = fmaxf(mr, fmaxf(fabsf(rr[k]), fmaxf(fabsf(ss[k]), fabsf(tt[k]))));
            }
            const int er = pow2_bound(wave_max(mr));
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int nd = l + 64 * k;
                hx[0][nd] = (_Float16)ldexpf(rr[k], -er);
                hx[1][nd] = (_Float16)ldexpf(ss[k], -er);
                hx[2][nd] = (_Float16)ldexpf(tt[k], -er);
            }
            __syncthreads();
            f16_contract<false>(hx[0], fb[0], 0, aDT, l);  // D_r^T r
            __syncthreads();
            f16_contract<true>(hx[1], fb[0], 1, aDT, l);   // + D_s^T s
            __syncthreads();
            f16_contract<true>(hx[2], fb[0], 2, aDT, l);   // + D_t^T t
            __syncthreads();
            float* y = Y + ((int64_t)c * E + e) * NP;
#pragma unroll
            for (int k = 0; k < 8; ++k) y[l + 64 * k] = ldexpf(fb[0][l + 64 * k], ex + er);
            __syncthreads();
        }
    }
}

int ax_local_f16(int64_t E, int N, int geo_kind, const double* geo, const float* Gs, const double* D,
                 const double* xi, const double* w, int nrhs, const float* X, float* Y, hipStream_t st)
{
    if (N != 7)
        return fail(AX_ERR_UNSUPPORTED, "AX_FP16_ACC32 is implemented for N = 7 (8x8 matrix-core tiles) only");
    BasisF16 bs;
    for (int q = 0; q < 64; ++q) bs.D[q] = (float)D[q];
    for (int q = 0; q < 8; ++q) {
        bs.xi[q] = xi ? xi[q] : 0.0;
        bs.w[q] = w ? w[q] : 0.0;
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t cap = (int64_t)cus * 16;
    const unsigned grid = (unsigned)(E < cap ? E : cap);
    switch (geo_kind) {
    case 0:
        hipLaunchKernelGGL(ax_local_f16_kernel<F16_TRI>, dim3(grid), dim3(64), 0, st, E, nrhs, geo, Gs, X, Y, bs);
        break;
    case 1:
        hipLaunchKernelGGL(ax_local_f16_kernel<F16_PARA>, dim3(grid), dim3(64), 0, st, E, nrhs, geo, Gs, X, Y, bs);
        break;
    default:
        hipLaunchKernelGGL(ax_local_f16_kernel<F16_STORED>, dim3(grid), dim3(64), 0, st, E, nrhs, geo, Gs, X, Y, bs);
        break;
    }
    return hip_check(hipGetLastError(), "ax_local fp16 launch");
}

}  // namespace ax
