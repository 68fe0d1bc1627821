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
#include "ax_kernels.h"
#include "geom.h"

namespace ax {

template <int N1, int GEO, bool EO, typename T>
__global__ void __launch_bounds__(Shape<N1>::BLOCK, Shape<N1>::MINW)
ax_local_kernel(int64_t E, int nrhs, const double* __restrict__ geo, const T* __restrict__ Gs,
                const T* __restrict__ X, T* __restrict__ Y, const Basis<T> bs)
{
    using S = Shape<N1>;
    constexpr int NT = S::NT, SJ = S::SJ, SK = S::SK, FS = S::FS, NP = S::NP, EPB = S::EPB;
    constexpr int BLOCK = S::BLOCK;
    constexpr int NV = (GEO == GEO_TRI) ? 24 : 0;                // vertex words per element
    constexpr int VPT = (EPB * NV + BLOCK - 1) / BLOCK;          // vertex words per thread
    __shared__ T smem[S::SLOTS * 2 * FS];
    __shared__ double svert[(GEO == GEO_TRI) ? EPB * 24 : 1];
    // (xi_k, w_k) pairs: read per node from LDS rather than held in scalar registers, which
    // leaves the scalar file to the contraction coefficients
    __shared__ double sxw[2 * N1];

    const int tid = threadIdx.x;
    const int slot = (S::SLOTS == 1) ? 0 : tid / NT;
    const int lane = tid - slot * NT;
    T* __restrict__ A = smem + slot * 2 * FS;
    T* __restrict__ B = A + FS;
    const int i = lane % N1, j = lane / N1;    // home lane: node column (i, j, :)
    const int pa = lane % N1, pb = lane / N1;  // pencil lane: (j,k) for r, (i,k) for s
    const int64_t nblk = (E + EPB - 1) / EPB;
    if (tid < 2 * N1) sxw[tid] = (tid & 1) ? bs.w[tid >> 1] : bs.xi[tid >> 1];

    // Items are (element group, column) pairs walked in order; each work-group strides over the
    // element groups.  The next item's X (and vertices) are fetched into registers while the
    // current one is computed, so HBM latency overlaps with the contraction work.
    int64_t eb = blockIdx.x;
    int c = 0;
    auto x_base = [&](int64_t ebq, int cq, bool& act) -> int64_t {
        const int64_t eq = ebq * EPB + slot;
        act = (ebq < nblk) && (slot < EPB) && (eq < E);
        return ((int64_t)cq * E + (act ? eq : 0)) * NP;
    };
    T xr[N1];
    double vr[VPT > 0 ? VPT : 1];
    {
        bool act;
        const int64_t b0 = x_base(eb, c, act);
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = act ? X[b0 + i + j * N1 + k * NT] : T(0);
        if constexpr (GEO == GEO_TRI) {
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                const int idx = tid + q * BLOCK;
                const int64_t off = eb * EPB * 24 + idx;
                vr[q] = (idx < EPB * 24 && eb < nblk && off < E * 24) ? geo[off] : 0.0;
            }
        }
    }

    TriCoef tc;
    double h[6];
    while (eb < nblk) {
        bool active;
        const int64_t base = x_base(eb, c, active);
        const int64_t e = eb * EPB + slot;
        if constexpr (GEO == GEO_PARA) {
            if (c == 0) {
                const double* he = geo + (active ? e : 0) * 6;
                const double wij = bs.w[i] * bs.w[j];
#pragma unroll
                for (int q = 0; q < 6; ++q) h[q] = he[q] * wij;
            }
        }
        // P0: stage X (and the vertices), prefetch the next item, t-contraction in registers
#pragma unroll
        for (int k = 0; k < N1; ++k) A[k * SK + j * SJ + i] = xr[k];
        if constexpr (GEO == GEO_TRI) {
            if (c == 0) {
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const int idx = tid + q * BLOCK;
                    if (idx < EPB * 24) svert[idx] = vr[q];
                }
            }
        }
        const bool last_col = (c + 1 == nrhs);
        const int64_t eb_n = last_col ? eb + gridDim.x : eb;
        const int c_n = last_col ? 0 : c + 1;
        T xn[N1];
        {
            bool act_n;
            const int64_t bn = x_base(eb_n, c_n, act_n);
            // inactive lanes re-read a valid line of the current element and discard it, which
            // keeps the loads free of per-load branches
            const T* src = X + (act_n ? bn : base) + i + j * N1;
#pragma unroll
            for (int k = 0; k < N1; ++k) xn[k] = src[k * NT];
            if (!act_n) {
#pragma unroll
                for (int k = 0; k < N1; ++k) xn[k] = T(0);
            }
            if constexpr (GEO == GEO_TRI) {
                if (last_col) {
#pragma unroll
                    for (int q = 0; q < VPT; ++q) {
                        const int idx = tid + q * BLOCK;
                        const int64_t off = eb_n * EPB * 24 + idx;
                        vr[q] = (idx < EPB * 24 && eb_n < nblk && off < E * 24) ? geo[off] : 0.0;
                    }
                }
            }
        }
        T x2[N1];
        contract<N1, false, EO>(bs, xr, x2);  // x2 = D_t x
        __syncthreads();
        // P1: r-pencils (j,k) -> x0 in B; s-pencils (i,k) -> x1 held in registers
        T o1[N1];
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[pb * SK + pa * SJ + n];
            contract<N1, false, EO>(bs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[pb * SK + pa * SJ + a] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[pb * SK + n * SJ + pa];
            contract<N1, false, EO>(bs, p, o1);
        }
        __syncthreads();
        // P2: x1 -> A; per-element geometry invariants of the home column from the staged vertices
#pragma unroll
        for (int a = 0; a < N1; ++a) A[pb * SK + a * SJ + pa] = o1[a];
        if constexpr (GEO == GEO_TRI) {
            if (c == 0) {
                const double* sv = svert + (slot < EPB ? slot : 0) * 24;
                tri_prelude([&](int v, int q) { return sv[v * 3 + q]; }, bs.xi[i], bs.xi[j], bs.w[i],
                            bs.w[j], tc);
            }
        }
        __syncthreads();
        // P3: pointwise factors at the home column; r -> B, s -> A, t stays in registers
        T tt[N1];
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            const int l = k * SK + j * SJ + i;
            T x0 = B[l], x1 = A[l], xx2 = x2[k];
            T g[6];
            if constexpr (GEO == GEO_TRI) {
                T lam;
                tri_adj<T>(tc, T(sxw[2 * k]), T(sxw[2 * k + 1]), g, lam);
                x0 *= lam;
                x1 *= lam;
                xx2 *= lam;
            } else if constexpr (GEO == GEO_PARA) {
                const T wk = T(sxw[2 * k + 1]);
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = T(h[q]) * wk;
            } else {
                const T* ge = Gs + (active ? e : 0) * 6 * NP + i + j * N1 + k * NT;
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = active ? ge[q * NP] : T(0);
            }
            B[l] = fma(g[0], x0, fma(g[1], x1, g[2] * xx2));
            A[l] = fma(g[1], x0, fma(g[3], x1, g[4] * xx2));
            tt[k] = fma(g[2], x0, fma(g[4], x1, g[5] * xx2));
        }
        T y2[N1];
        contract<N1, true, EO>(bs, tt, y2);  // D_t^T t
        __syncthreads();
        // P4: D_r^T r in place on the r-pencils; D_s^T s into registers
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = B[pb * SK + pa * SJ + n];
            contract<N1, true, EO>(bs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[pb * SK + pa * SJ + a] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[pb * SK + n * SJ + pa];
            contract<N1, true, EO>(bs, p, o1);
        }
        __syncthreads();
        // P5: add D_s^T s on the s-pencils
#pragma unroll
        for (int a = 0; a < N1; ++a) B[pb * SK + a * SJ + pa] += o1[a];
        __syncthreads();
        // P6: Y = (D_r^T r + D_s^T s) + D_t^T t
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k) Y[base + i + j * N1 + k * NT] = B[k * SK + j * SJ + i] + y2[k];
        }
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = xn[k];
        eb = eb_n;
        c = c_n;
    }
}

template <int N1, int GEO, typename T>
static int64_t persistent_groups()
{
    static int64_t g = 0;
    if (g == 0) {
        int dev = 0, cus = 256, per = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, ax_local_kernel<N1, GEO, true, T>,
                                                         Shape<N1>::BLOCK, 0) != hipSuccess || per < 1)
            per = 1;
        g = (int64_t)cus * per * AX_PERSIST_MULT;
    }
    return g;
}

template <int N1, int GEO, typename T>
static int launch_n1(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                     const double* D, const double* xi, const double* w, hipStream_t st)
{
    using S = Shape<N1>;
    Basis<T> bs;
    fill_basis(bs, N1, D, xi, w);
    const int64_t nblk = (E + S::EPB - 1) / S::EPB;
    // persistent work-groups: enough to fill every CU several times over, never more than the
    // number of element groups
    const int64_t blocks = nblk < persistent_groups<N1, GEO, T>() ? nblk : persistent_groups<N1, GEO, T>();
    if (centro_antisymmetric(N1, D))
        hipLaunchKernelGGL((ax_local_kernel<N1, GEO, true, T>), dim3((unsigned)blocks), dim3(S::BLOCK), 0,
                           st, E, nrhs, geo, Gs, X, Y, bs);
    else
        hipLaunchKernelGGL((ax_local_kernel<N1, GEO, false, T>), dim3((unsigned)blocks), dim3(S::BLOCK), 0,
                           st, E, nrhs, geo, Gs, X, Y, bs);
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
