// AxLocal on gfx950: Y_e = D^T G_e D X_e (Eq. 3, Poisson) by sum factorisation (Algorithm 1),
// with the geometric factors recomputed in the kernel (trilinear: Sec. 3.3 / Algorithm 2;
// parallelepiped: Algorithm 3) or streamed from memory (the stored-factor baseline).
//
// Work decomposition (one wave64 per element at N1 = 8):
//   * A work-group owns EPB elements; each element gets N1*N1 lanes.  The "home" lane (i, j)
//     owns the node column X[i, j, :] in registers, as in the 2-D thread layer of Algorithm 4.
//   * Every one-dimensional contraction is done "pencil-wise": a lane holds N1 values along the
//     contracted direction and produces N1 outputs with N1^2 FMAs whose D operands are the same
//     for every lane (kernel arguments, read through the scalar unit).  Compared with the slice
//     scheme of Algorithm 4 (a lane-dependent row of D against N1 values of a shared slice), this
//     cuts LDS reads per FMA from 1 to 1/N1, which matters because a CDNA4 CU moves 16 doubles
//     per clock out of LDS but retires 64 FP64 FMAs per clock.
//   * The t-contractions run on the home lane's registers.  The r- and s-contractions read
//     pencils from an LDS copy of the element (row stride padded to an odd number of words so
//     both pencil directions are free of bank conflicts) and hand results back through LDS.
//   * The FP64 matrix cores of gfx950 run at the same rate as FP64 FMA on the vector unit and do
//     not overlap with it, so the FP64 contractions stay on the vector unit.
#include "ax_internal.h"
#include "geom.h"

namespace ax {

enum { GEO_TRI = 0, GEO_PARA = 1, GEO_STORED = 2 };

template <int N1>
struct Shape {
    static constexpr int NT = N1 * N1;                        // lanes per element
    static constexpr int SJ = (N1 % 2 == 0) ? N1 + 1 : N1;    // LDS row stride (odd)
    static constexpr int SK = N1 * SJ;                        // LDS slice stride
    static constexpr int FS = N1 * SK;                        // LDS words per field
    static constexpr int NP = N1 * N1 * N1;                   // nodes per element
    // elements per work-group: fill (nearly) whole waves while keeping LDS modest
    static constexpr int EPB = N1 == 2 ? 16 : N1 == 3 ? 7 : N1 == 4 ? 4 : N1 == 5 ? 5
                             : N1 == 6 ? 7 : N1 == 7 ? 5 : N1 == 9 ? 3 : N1 == 10 ? 3
                             : N1 == 11 ? 2 : 1;
    static constexpr int BLOCK = ((EPB * NT + 63) / 64) * 64;
    static constexpr int SLOTS = (BLOCK + NT - 1) / NT;
};

// out[a] = sum_n D[a][n] in[n]   (TRANS: out[a] = sum_n D[n][a] in[n])
template <int N1, bool TRANS, typename T>
__device__ __forceinline__ void contract(const T* __restrict__ D, const T* in, T* out)
{
#pragma unroll
    for (int a = 0; a < N1; ++a) {
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < N1; ++n) acc = fma(TRANS ? D[n * N1 + a] : D[a * N1 + n], in[n], acc);
        out[a] = acc;
    }
}

template <int N1, int GEO, typename T>
__global__ void __launch_bounds__(Shape<N1>::BLOCK)
ax_local_kernel(int64_t E, int nrhs, const double* __restrict__ geo, const T* __restrict__ Gs,
                const T* __restrict__ X, T* __restrict__ Y, const Basis<T> bs)
{
    using S = Shape<N1>;
    constexpr int NT = S::NT, SJ = S::SJ, SK = S::SK, FS = S::FS, NP = S::NP, EPB = S::EPB;
    __shared__ T smem[S::SLOTS * 3 * FS];

    const int tid = threadIdx.x;
    const int slot = (S::SLOTS == 1) ? 0 : tid / NT;
    const int lane = tid - slot * NT;
    const int64_t e0 = (int64_t)blockIdx.x * EPB;          // uniform across the work-group
    const int64_t e = (EPB == 1) ? e0 : e0 + slot;
    const bool active = (slot < EPB) && (e < E);
    T* __restrict__ A = smem + slot * 3 * FS;
    T* __restrict__ B = A + FS;
    T* __restrict__ C = B + FS;

    const int i = lane % N1, j = lane / N1;   // home lane: node column (i, j, :)
    const int pa = lane % N1, pb = lane / N1; // pencil lane: (j,k) for r, (i,k) for s

    // per-element geometry invariants of the home column
    TriCoef tc;
    double h[6];
    if constexpr (GEO == GEO_TRI) {
        double V[24];
        const double* Ve = geo + (active ? e : 0) * 24;
#pragma unroll
        for (int q = 0; q < 24; ++q) V[q] = Ve[q];
        tri_prelude(V, bs.xi[i], bs.xi[j], bs.w[i], bs.w[j], tc);
    } else if constexpr (GEO == GEO_PARA) {
        const double* he = geo + (active ? e : 0) * 6;
        const double wij = bs.w[i] * bs.w[j];
#pragma unroll
        for (int q = 0; q < 6; ++q) h[q] = he[q] * wij;
    }

    for (int c = 0; c < nrhs; ++c) {
        const int64_t base = ((int64_t)c * E + (active ? e : 0)) * NP;
        T xr[N1], x2[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = active ? X[base + i + j * N1 + k * NT] : T(0);
#pragma unroll
        for (int k = 0; k < N1; ++k) A[k * SK + j * SJ + i] = xr[k];
        contract<N1, false>(bs.D, xr, x2);  // x2 = D_t x (home column)
        __syncthreads();
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[pb * SK + pa * SJ + n];
            contract<N1, false>(bs.D, p, o);  // x0 = D_r x along i, pencil (j,k) = (pa,pb)
#pragma unroll
            for (int a = 0; a < N1; ++a) B[pb * SK + pa * SJ + a] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[pb * SK + n * SJ + pa];
            contract<N1, false>(bs.D, p, o);  // x1 = D_s x along j, pencil (i,k) = (pa,pb)
#pragma unroll
            for (int a = 0; a < N1; ++a) C[pb * SK + a * SJ + pa] = o[a];
        }
        __syncthreads();
        T tt[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            const int l = k * SK + j * SJ + i;
            T x0 = B[l], x1 = C[l], xx2 = x2[k];
            T g[6];
            if constexpr (GEO == GEO_TRI) {
                T lam;
                tri_adj<T>(tc, T(bs.xi[k]), T(bs.w[k]), g, lam);
                x0 *= lam;
                x1 *= lam;
                xx2 *= lam;
            } else if constexpr (GEO == GEO_PARA) {
                const T wk = T(bs.w[k]);
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = T(h[q]) * wk;
            } else {
                const T* ge = Gs + (active ? e : 0) * 6 * NP + i + j * N1 + k * NT;
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = active ? ge[q * NP] : T(0);
            }
            B[l] = fma(g[0], x0, fma(g[1], x1, g[2] * xx2));
            C[l] = fma(g[1], x0, fma(g[3], x1, g[4] * xx2));
            tt[k] = fma(g[2], x0, fma(g[4], x1, g[5] * xx2));
        }
        T y2[N1];
        contract<N1, true>(bs.D, tt, y2);  // D_t^T t (home column)
        __syncthreads();
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = B[pb * SK + pa * SJ + n];
            contract<N1, true>(bs.D, p, o);  // D_r^T r along i
#pragma unroll
            for (int a = 0; a < N1; ++a) A[pb * SK + pa * SJ + a] = o[a];
        }
        __syncthreads();
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = C[pb * SK + n * SJ + pa];
            contract<N1, true>(bs.D, p, o);  // D_s^T s along j
#pragma unroll
            for (int a = 0; a < N1; ++a) A[pb * SK + a * SJ + pa] += o[a];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k) Y[base + i + j * N1 + k * NT] = A[k * SK + j * SJ + i] + y2[k];
        }
    }
}

template <int N1, int GEO, typename T>
static int launch_n1(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                     const double* D, const double* xi, const double* w, hipStream_t st)
{
    using S = Shape<N1>;
    Basis<T> bs;
    fill_basis(bs, N1, D, xi, w);
    const int64_t blocks = (E + S::EPB - 1) / S::EPB;
    if (blocks > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many elements for one launch");
    hipLaunchKernelGGL((ax_local_kernel<N1, GEO, T>), dim3((unsigned)blocks), dim3(S::BLOCK), 0, st,
                       E, nrhs, geo, Gs, X, Y, bs);
    return hip_check(hipGetLastError(), "ax_local launch");
}

template <int GEO, typename T>
static int dispatch(int N, int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                    const double* D, const double* xi, const double* w, hipStream_t st)
{
    switch (N + 1) {
#define AX_CASE(n1) \
    case n1: return launch_n1<n1, GEO, T>(E, nrhs, geo, Gs, X, Y, D, xi, w, st);
        AX_CASE(2) AX_CASE(3) AX_CASE(4) AX_CASE(5) AX_CASE(6) AX_CASE(7) AX_CASE(8) AX_CASE(9)
        AX_CASE(10) AX_CASE(11) AX_CASE(12) AX_CASE(13) AX_CASE(14) AX_CASE(15) AX_CASE(16)
#undef AX_CASE
    default:
        return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    }
}

static int check_common(int64_t E, int N, int nrhs, int prec, const void* X, const void* Y,
                        const double* D)
{
    if (E < 0) return fail(AX_ERR_ARG, "E=%lld < 0", (long long)E);
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs=%d < 1", nrhs);
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (prec != AX_FP64 && prec != AX_FP32 && prec != AX_FP16_ACC32)
        return fail(AX_ERR_UNSUPPORTED, "unknown precision %d", prec);
    if (!D) return fail(AX_ERR_ARG, "D is NULL");
    if (E > 0 && (!X || !Y)) return fail(AX_ERR_ARG, "X or Y is NULL");
    if (E > 0 && X == Y) return fail(AX_ERR_ARG, "X and Y alias (in-place is not supported)");
    return AX_OK;
}

// FP16-input / FP32-accumulate variants live in ax_local_f16.hip.
int ax_local_f16(int64_t E, int N, int geo_kind, const double* geo, const float* Gs,
                 const double* D, const double* xi, const double* w, int nrhs, const float* X,
                 float* Y, hipStream_t st);

}  // namespace ax

using namespace ax;

extern "C" int ax_local(int64_t E, int N, int geom, const double* geo, const double* D,
                        const double* xi, const double* w, int nrhs, int prec, const void* X,
                        void* Y, void* stream)
{
    clear_error();
    AX_TRY(check_common(E, N, nrhs, prec, X, Y, D));
    if (geom != AX_TRILINEAR && geom != AX_PARALLELEPIPED)
        return fail(AX_ERR_UNSUPPORTED, "unknown geometry %d", geom);
    if (!w) return fail(AX_ERR_ARG, "w is NULL");
    if (geom == AX_TRILINEAR && !xi) return fail(AX_ERR_ARG, "xi is NULL (needed for trilinear)");
    if (E == 0) return AX_OK;
    if (!geo) return fail(AX_ERR_ARG, "geo is NULL");
    hipStream_t st = as_stream(stream);
    const int gk = geom == AX_TRILINEAR ? GEO_TRI : GEO_PARA;
    if (prec == AX_FP64) {
        if (gk == GEO_TRI)
            return dispatch<GEO_TRI, double>(N, E, nrhs, geo, nullptr, (const double*)X, (double*)Y, D, xi, w, st);
        return dispatch<GEO_PARA, double>(N, E, nrhs, geo, nullptr, (const double*)X, (double*)Y, D, xi, w, st);
    }
    if (prec == AX_FP32) {
        if (gk == GEO_TRI)
            return dispatch<GEO_TRI, float>(N, E, nrhs, geo, nullptr, (const float*)X, (float*)Y, D, xi, w, st);
        return dispatch<GEO_PARA, float>(N, E, nrhs, geo, nullptr, (const float*)X, (float*)Y, D, xi, w, st);
    }
    return ax_local_f16(E, N, gk, geo, nullptr, D, xi, w, nrhs, (const float*)X, (float*)Y, st);
}

extern "C" int ax_local_precomputedG(int64_t E, int N, const void* G, const double* D, int nrhs,
                                     int prec, const void* X, void* Y, void* stream)
{
    clear_error();
    AX_TRY(check_common(E, N, nrhs, prec, X, Y, D));
    if (E == 0) return AX_OK;
    if (!G) return fail(AX_ERR_ARG, "G is NULL");
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        return dispatch<GEO_STORED, double>(N, E, nrhs, nullptr, (const double*)G, (const double*)X, (double*)Y, D, nullptr, nullptr, st);
    if (prec == AX_FP32)
        return dispatch<GEO_STORED, float>(N, E, nrhs, nullptr, (const float*)G, (const float*)X, (float*)Y, D, nullptr, nullptr, st);
    return ax_local_f16(E, N, GEO_STORED, nullptr, (const float*)G, D, nullptr, nullptr, nrhs, (const float*)X, (float*)Y, st);
}
