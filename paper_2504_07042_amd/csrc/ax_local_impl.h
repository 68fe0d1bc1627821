// AxLocal kernel template and its launch dispatch (internal header, instantiated per arithmetic
// type in ax_local_f64.hip and ax_local_f32.hip).
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
#pragma once

#include "ax_internal.h"
#include "ax_kernels.h"
#include "geom.h"

// Issue point of the next item's loads: 0 = before the first contraction (longest overlap),
// 1 = after the pointwise stage (shorter overlap, fewer live registers at the pointwise peak).
#ifndef AX_PREFETCH_LATE
#define AX_PREFETCH_LATE 0
#endif

namespace ax {

// Work-group shape for EPBX elements of order N1 - 1.
template <int N1, int EPBX>
struct Tile {
    static constexpr int NT = N1 * N1;
    static constexpr int EPB = EPBX;
    static constexpr int BLOCK = ((EPB * NT + 63) / 64) * 64;
    static constexpr int SLOTS = (BLOCK + NT - 1) / NT;
};

// GATHER: X is a global vector [nrhs][ldg] read through the local-to-global map l2g (the Q of
// Sec. 2.1 fused into the load), so the solver never materialises Q x.
template <int N1, int GEO, bool EO, bool GATHER, int EPBX, typename T>
__global__ void __launch_bounds__((Tile<N1, EPBX>::BLOCK), Shape<N1>::MINW)
ax_local_kernel(int64_t E, int nrhs, const double* __restrict__ geo, const T* __restrict__ Gs,
                const T* __restrict__ X, T* __restrict__ Y, const Basis<T> bs,
                const int32_t* __restrict__ l2g, int64_t ldg)
{
    using S = Shape<N1>;
    using TL = Tile<N1, EPBX>;
    constexpr int NT = S::NT, FS = S::FS, NP = S::NP, EPB = TL::EPB;
    constexpr int BLOCK = TL::BLOCK;
    constexpr int NV = (GEO == GEO_TRI) ? 24 : 0;                // vertex words per element
    constexpr int VPT = (EPB * NV + BLOCK - 1) / BLOCK;          // vertex words per thread
    __shared__ T smem[TL::SLOTS * 2 * FS];
    __shared__ double svert[(GEO == GEO_TRI) ? EPB * 24 : 1];
    // (xi_k, w_k) pairs: read per node from LDS rather than held in scalar registers, which
    // leaves the scalar file to the contraction coefficients
    __shared__ double sxw[2 * N1];

    const int tid = threadIdx.x;
    const int slot = (TL::SLOTS == 1) ? 0 : tid / NT;
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
    // node column (i, j, :) of item (ebq, cq); inactive lanes read element 0 and discard it,
    // which keeps the loads free of per-load branches
    auto load_x = [&](int64_t ebq, int cq, T* dst) {
        const int64_t eq = ebq * EPB + slot;
        const bool act = (ebq < nblk) && (slot < EPB) && (eq < E);
        const int64_t le = (act ? eq : 0) * NP + i + j * N1;
        if constexpr (GATHER) {
            int32_t gi[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) gi[k] = l2g[le + k * NT];
            const T* xc = X + (int64_t)cq * ldg;
#pragma unroll
            for (int k = 0; k < N1; ++k) dst[k] = xc[gi[k]];
        } else {
            const T* src = X + (int64_t)cq * E * NP + le;
#pragma unroll
            for (int k = 0; k < N1; ++k) dst[k] = src[k * NT];
        }
        if (!act) {
#pragma unroll
            for (int k = 0; k < N1; ++k) dst[k] = T(0);
        }
    };
    T xr[N1];
    double vr[VPT > 0 ? VPT : 1];
    load_x(eb, c, xr);
    if constexpr (GEO == GEO_TRI) {
#pragma unroll
        for (int q = 0; q < VPT; ++q) {
            const int idx = tid + q * BLOCK;
            const int64_t off = eb * EPB * 24 + idx;
            vr[q] = (idx < EPB * 24 && eb < nblk && off < E * 24) ? geo[off] : 0.0;
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
        for (int k = 0; k < N1; ++k) A[S::pos(i, j, k)] = xr[k];
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
        auto prefetch = [&]() {
            load_x(eb_n, c_n, xn);
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
        };
        if constexpr (AX_PREFETCH_LATE == 0) prefetch();
        T x2[N1];
        contract<N1, false, EO>(bs, xr, x2);  // x2 = D_t x
        __syncthreads();
        // P1: r-pencils (j,k) -> x0 in B; s-pencils (i,k) -> x1 held in registers
        T o1[N1];
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[S::pos(n, pa, pb)];
            contract<N1, false, EO>(bs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[S::pos(a, pa, pb)] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[S::pos(pa, n, pb)];
            contract<N1, false, EO>(bs, p, o1);
        }
        __syncthreads();
        // P2: x1 -> A; per-element geometry invariants of the home column from the staged vertices
#pragma unroll
        for (int a = 0; a < N1; ++a) A[S::pos(pa, a, pb)] = o1[a];
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
            const int l = S::pos(i, j, k);
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
        if constexpr (AX_PREFETCH_LATE != 0) prefetch();
        __syncthreads();
        // P4: D_r^T r in place on the r-pencils; D_s^T s into registers
        {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = B[S::pos(n, pa, pb)];
            contract<N1, true, EO>(bs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[S::pos(a, pa, pb)] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[S::pos(pa, n, pb)];
            contract<N1, true, EO>(bs, p, o1);
        }
        __syncthreads();
        // P5: add D_s^T s on the s-pencils
#pragma unroll
        for (int a = 0; a < N1; ++a) B[S::pos(pa, a, pb)] += o1[a];
        __syncthreads();
        // P6: Y = (D_r^T r + D_s^T s) + D_t^T t
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k) Y[base + i + j * N1 + k * NT] = B[S::pos(i, j, k)] + y2[k];
        }
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = xn[k];
        eb = eb_n;
        c = c_n;
    }
}

template <int N1, int GEO, bool EO, bool GATHER, int EPBX, typename T>
static int launch_tile(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y, const Basis<T>& bs,
                       int grid_mult, hipStream_t st, const int32_t* l2g, int64_t ldg)
{
    using TL = Tile<N1, EPBX>;
    static int per = 0;  // resident work-groups per CU for this instantiation
    static int cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, ax_local_kernel<N1, GEO, EO, GATHER, EPBX, T>,
                                                         TL::BLOCK, 0) != hipSuccess || q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t nblk = (E + TL::EPB - 1) / TL::EPB;
    // persistent work-groups: grid_mult times the resident capacity, never more than the number
    // of element groups
    const int64_t cap = (int64_t)cus * per * (grid_mult > 0 ? grid_mult : 1);
    const int64_t blocks = nblk < cap ? nblk : cap;
    if (blocks > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many elements for one launch");
    hipLaunchKernelGGL((ax_local_kernel<N1, GEO, EO, GATHER, EPBX, T>), dim3((unsigned)blocks), dim3(TL::BLOCK),
                       0, st, E, nrhs, geo, Gs, X, Y, bs, l2g, ldg);
    return hip_check(hipGetLastError(), "ax_local launch");
}

template <int N1, int GEO, typename T>
static int launch_n1(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                     const double* D, const double* xi, const double* w, hipStream_t st,
                     const int32_t* l2g, int64_t ldg)
{
    using S = Shape<N1>;
    Basis<T> bs;
    fill_basis(bs, N1, D, xi, w);
    const bool eo = centro_antisymmetric(N1, D);
    const TuneEntry tu = tune_get(N1, GEO, sizeof(T) == 8 ? AX_FP64 : AX_FP32);
    if (l2g) {
        if (!eo) return fail(AX_ERR_UNSUPPORTED, "gathering AxLocal needs a GLL differentiation matrix");
        if constexpr (GEO != GEO_STORED)
            return launch_tile<N1, GEO, true, true, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, l2g, ldg);
        return fail(AX_ERR_UNSUPPORTED, "gathering AxLocal needs on-the-fly factors");
    }
    if (!eo)
        return launch_tile<N1, GEO, false, false, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, nullptr, 0);
    if constexpr (S::EPB_ALT != S::EPB) {
        if (tu.epb_alt)
            return launch_tile<N1, GEO, true, false, S::EPB_ALT, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st,
                                                                    nullptr, 0);
    }
    return launch_tile<N1, GEO, true, false, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, nullptr, 0);
}

template <int GEO, typename T>
static int dispatch(int N, int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                    const double* D, const double* xi, const double* w, hipStream_t st,
                    const int32_t* l2g, int64_t ldg)
{
    switch (N + 1) {
#define AX_CASE(n1) \
    case n1: return launch_n1<n1, GEO, T>(E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg);
        AX_CASE(2) AX_CASE(3) AX_CASE(4) AX_CASE(5) AX_CASE(6) AX_CASE(7) AX_CASE(8) AX_CASE(9)
        AX_CASE(10) AX_CASE(11) AX_CASE(12) AX_CASE(13) AX_CASE(14) AX_CASE(15) AX_CASE(16)
#undef AX_CASE
    default:
        return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    }
}
}  // namespace ax
