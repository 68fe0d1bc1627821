// Per-item building blocks of the trilinear on-the-fly operator (internal header): one element
// per N1^2 lanes (each lane owns a node column, then an r- and an s-pencil), several elements per
// work-group.  Shared by the batched kernels (one persistent launch per order over a work list
// of many meshes) and the single-mesh per-item kernels of ax_local; the work-group shape is a
// run-time variant (item_shape) chosen by the tuning table.
//
// Per item the work is the trilinear on-the-fly operator of ax_local (geometric factors of
// Sec. 3.3 / Algorithm 2, contractions of Algorithm 1) with the basis tables read per output row.
#pragma once

#include "ax_internal.h"
#include "ax_kernels.h"
#include "geom.h"

namespace ax {

constexpr int kBMaxN1 = 10;  // highest order (N1 = N + 1) of the batched launches

// One mesh of a batch (device descriptor) and one work item (element group eb of mesh `mesh`).
struct BMesh {
    int64_t E;
    int64_t ld;  // stride between columns of X and Y (values)
    const double* verts;
    const void* X;
    void* Y;
    int N1;
    int wgs;     // slice form of the batched tile kernel: work-groups given to this mesh
    int64_t es;  // stride between elements of X and Y (values): N1^3, or ncol N1^3 interleaved
    // gathering form (kernels instantiated with GATHER): X is a global vector read through l2g
    // (this mesh's part of the map, local element-major numbering), columns ldg values apart
    const int32_t* l2g;
    int64_t ldg;
};

struct BItem {
    int mesh;
    int eb;  // element group within the mesh
};

// Work-group shape of variant V of order N1: EPB elements on BLOCK lanes (item_shape), and the
// LDS per work-group: two fields per element plus its 24 vertex words.
template <int N1, int V>
struct BShape {
    static constexpr int NT = N1 * N1;
    static constexpr int EPB = item_shape(N1, V).epb;
    static constexpr int BLOCK = item_shape(N1, V).block;
    static constexpr int NP = Shape<N1>::NP;
    static_assert(EPB * NT <= BLOCK && BLOCK % 64 == 0 && BLOCK <= 1024, "item shape");
    template <typename T>
    static constexpr int FS = Shape<N1, sizeof(T)>::FS;
    template <typename T>
    static constexpr size_t lds_bytes() { return (size_t)EPB * 2 * FS<T> * sizeof(T) + (size_t)EPB * 24 * 8; }
};

// cs: source of the basis tables (CoefResident or CoefReload)
// PL: partial recomputation (Sec. 4.2.2), the per-node scale read from lam [E][N1^3].
template <int N1, int V, typename T, bool PL = false, bool GATHER = false, typename C>
__device__ __forceinline__ void batched_item(const BMesh& m, int64_t eb, int nrhs, const C& cs, char* lds,
                                             const T* __restrict__ lamp = nullptr)
{
    using S = BShape<N1, V>;
    constexpr int NT = S::NT, EPB = S::EPB, FS = S::template FS<T>, NP = S::NP;
    T* smem = reinterpret_cast<T*>(lds);
    double* svert = reinterpret_cast<double*>(lds + (size_t)EPB * 2 * FS * sizeof(T));
    const int tid = threadIdx.x;
    const int slot = tid / NT;
    const int lane = tid - slot * NT;
    const bool inslot = slot < EPB;
    const int64_t e = eb * EPB + slot;
    const bool active = inslot && e < m.E;
    T* A = smem + (inslot ? slot : 0) * 2 * FS;
    T* B = A + FS;
    const int i = lane % N1, j = lane / N1;
    const int pa = i, pb = j;
    const T* X = reinterpret_cast<const T*>(m.X);
    T* Y = reinterpret_cast<T*>(m.Y);

    for (int q = tid; q < EPB * 24; q += S::BLOCK) {
        const int64_t off = eb * EPB * 24 + q;
        svert[q] = off < m.E * 24 ? m.verts[off] : 0.0;
    }
    __syncthreads();
    TriCoefT<T> tc;
    if (inslot) {
        const double* sv = svert + slot * 24;
        const C b = cs.row();
        TriCoef t64;
        tri_prelude([&](int v, int q) { return sv[v * 3 + q]; }, b.xi(i), b.xi(j), b.w(i), b.w(j), t64);
        tri_narrow(t64, tc);
    }
    for (int c = 0; c < nrhs; ++c) {
        const int64_t base = (int64_t)c * m.ld + (active ? e : 0) * m.es;
        T xr[N1], x2[N1];
        if constexpr (GATHER) {
            const int32_t* lm = m.l2g + (active ? e : 0) * NP + i + j * N1;
            int32_t gi[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) gi[k] = active ? lm[k * NT] : 0;
            const T* xc = X + (int64_t)c * m.ldg;
#pragma unroll
            for (int k = 0; k < N1; ++k) xr[k] = active ? xc[gi[k]] : T(0);
        } else {
#pragma unroll
            for (int k = 0; k < N1; ++k) xr[k] = active ? X[base + i + j * N1 + k * NT] : T(0);
        }
        if (inslot) {
#pragma unroll
            for (int k = 0; k < N1; ++k) A[Shape<N1, sizeof(T)>::pos(i, j, k)] = xr[k];
        }
        contract<N1, false, true>(cs, xr, x2);
        __syncthreads();
        T o1[N1];
        if (inslot) {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[Shape<N1, sizeof(T)>::pos(n, pa, pb)];
            contract<N1, false, true>(cs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[Shape<N1, sizeof(T)>::pos(a, pa, pb)] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[Shape<N1, sizeof(T)>::pos(pa, n, pb)];
            contract<N1, false, true>(cs, p, o1);
        }
        // Partial recomputation: all N1 scale loads of the column issued before the barrier
        // instead of one per node inside the loop below, so their latency overlaps the barrier
        // wait (measured interleaved, FP64: +12 % at N1 = 9, +28-30 % at N1 = 10, 11, 14, 15, and
        // at N1 = 12, 13 the extra registers cost a wave per SIMD and it is 9-10 % slower; FP32:
        // +16-20 % at N1 = 13..15).
        constexpr bool kEarly = PL && (sizeof(T) == 4 || (N1 != 12 && N1 != 13));
        T lv[N1];
        if constexpr (kEarly) {
#pragma unroll
            for (int k = 0; k < N1; ++k) lv[k] = lamp[(active ? e : 0) * NP + i + j * N1 + k * NT];
        }
        __syncthreads();
        if (inslot) {
#pragma unroll
            for (int a = 0; a < N1; ++a) A[Shape<N1, sizeof(T)>::pos(pa, a, pb)] = o1[a];
        }
        __syncthreads();
        T tt[N1];
        if (inslot) {
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                const int l = Shape<N1, sizeof(T)>::pos(i, j, k);
                T x0 = B[l], x1 = A[l], xx2 = x2[k];
                T g[6], lam;
                const C b = cs.row();
                if constexpr (PL) {
                    lam = kEarly ? lv[k] : lamp[(active ? e : 0) * NP + i + j * N1 + k * NT];
                    tri_adj_k<T>(tc, T(b.xi(k)), g);
                } else {
                    tri_adj<T>(tc, T(b.xi(k)), T(b.w(k)), g, lam);
                }
                x0 *= lam;
                x1 *= lam;
                xx2 *= lam;
                B[l] = fma(g[0], x0, fma(g[1], x1, g[2] * xx2));
                A[l] = fma(g[1], x0, fma(g[3], x1, g[4] * xx2));
                tt[k] = fma(g[2], x0, fma(g[4], x1, g[5] * xx2));
            }
        } else {
#pragma unroll
            for (int k = 0; k < N1; ++k) tt[k] = T(0);
        }
        T y2[N1];
        contract<N1, true, true>(cs, tt, y2);
        __syncthreads();
        if (inslot) {
            T p[N1], o[N1];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = B[Shape<N1, sizeof(T)>::pos(n, pa, pb)];
            contract<N1, true, true>(cs, p, o);
#pragma unroll
            for (int a = 0; a < N1; ++a) B[Shape<N1, sizeof(T)>::pos(a, pa, pb)] = o[a];
#pragma unroll
            for (int n = 0; n < N1; ++n) p[n] = A[Shape<N1, sizeof(T)>::pos(pa, n, pb)];
            contract<N1, true, true>(cs, p, o1);
        }
        __syncthreads();
        if (inslot) {
#pragma unroll
            for (int a = 0; a < N1; ++a) B[Shape<N1, sizeof(T)>::pos(pa, a, pb)] += o1[a];
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k) Y[base + i + j * N1 + k * NT] = B[Shape<N1, sizeof(T)>::pos(i, j, k)] + y2[k];
        }
        __syncthreads();
    }
}

// The per-item path above as a single-mesh persistent kernel (no work list): work-group g takes
// element groups g, g + grid, ...  Used by ax_local (and its partial-recomputation form) for the
// trilinear orders whose register footprint the prefetching kernel exceeds (FP64 N1 = 9..15:
// 118-162 VGPRs here against 256 plus spills there; measured 1.4-3.2x faster) or fills only at
// two waves per SIMD (N1 = 6, 7), with the tables reloaded per output row; which kernel runs is
// a run-time choice (item_default, or the tuning table).  V: shape variant (item_shape); W:
// register budget variant (item_waves).
template <typename T>
struct ItemArgs {
    BMesh m;
    int nrhs;
    Basis<T> bs;
    const T* lam;  // per-node scale of the partial recomputation (PL), else unused
};

// The register budget (item_waves): the FP32 full form fits five waves per SIMD (88-96 VGPRs;
// measured 3-8% faster than four at N1 = 10, 11, 12, 14, 15, 2% slower at 13); the FP32 partial
// form spills at five and keeps the default budget (measured 12% faster at N1 = 14, even at 13
// and 15).
template <int N1, typename T, bool PL, int V, int W>
__global__ void __launch_bounds__((BShape<N1, V>::BLOCK), (item_waves(N1, sizeof(T) == 4, PL, W)))
tri_item_kernel(const ItemArgs<T> a)
{
    __shared__ __attribute__((aligned(16))) char lds[BShape<N1, V>::template lds_bytes<T>()];
    lds_poison(lds, sizeof(lds));
    const int64_t ng = (a.m.E + BShape<N1, V>::EPB - 1) / BShape<N1, V>::EPB;
    const CoefReload<T> cs = karg_coefs<T, ItemArgs<T>>();
    for (int64_t eb = blockIdx.x; eb < ng; eb += gridDim.x)
        batched_item<N1, V, T, PL>(a.m, eb, a.nrhs, cs, lds, a.lam);
}

template <int N1, typename T, bool PL, int V, int W>
static int tri_item_launch(int64_t E, int nrhs, const double* verts, const T* X, T* Y, const Basis<T>& bs,
                           const T* lam, int grid_mult, hipStream_t st, int64_t es, int64_t ccs)
{
    static int per = 0, cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, tri_item_kernel<N1, T, PL, V, W>, BShape<N1, V>::BLOCK, 0) != hipSuccess ||
            q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t ng = (E + BShape<N1, V>::EPB - 1) / BShape<N1, V>::EPB;
    const int64_t cap = (int64_t)cus * per * (grid_mult > 0 ? grid_mult : 1);
    const int64_t blocks = ng < cap ? ng : cap;
    if (blocks <= 0) return AX_OK;
    const ItemArgs<T> a{BMesh{E, ccs, verts, X, Y, N1, 0, es}, nrhs, bs, lam};
    hipLaunchKernelGGL((tri_item_kernel<N1, T, PL, V, W>), dim3((unsigned)blocks), dim3(BShape<N1, V>::BLOCK), 0, st, a);
    return hip_check(hipGetLastError(), "ax_local (item kernel) launch");
}


// Single-mesh per-item AxLocal (defined in item_f64.hip / item_f32.hip): order N1 (2..16; the
// partial form, lam != nullptr, 9..16), shape variant `variant` and register budget variant
// `waves` (0 or 1 each; a variant an order does not have falls back to 0).
int tri_item_dispatch_f64(int N1, int64_t E, int nrhs, const double* verts, const double* X, double* Y,
                          const Basis<double>& bs, int grid_mult, int variant, int waves, hipStream_t st,
                          const double* lam, int64_t es, int64_t ccs);
int tri_item_dispatch_f32(int N1, int64_t E, int nrhs, const double* verts, const float* X, float* Y,
                          const Basis<float>& bs, int grid_mult, int variant, int waves, hipStream_t st,
                          const float* lam, int64_t es, int64_t ccs);

// Dispatch of one order over the four (shape, budget) variants.
template <int N1, typename T, bool PL>
static int tri_item_variants(int64_t E, int nrhs, const double* verts, const T* X, T* Y, const Basis<T>& bs,
                             const T* lam, int grid_mult, int variant, int waves, hipStream_t st, int64_t es,
                             int64_t ccs)
{
    if constexpr (item_has_alt(N1)) {
        if (variant)
            return waves ? tri_item_launch<N1, T, PL, 1, 1>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs)
                         : tri_item_launch<N1, T, PL, 1, 0>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs);
    }
    return waves ? tri_item_launch<N1, T, PL, 0, 1>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs)
                 : tri_item_launch<N1, T, PL, 0, 0>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs);
}

template <typename T>
static int tri_item_dispatch(int N1, int64_t E, int nrhs, const double* verts, const T* X, T* Y, const Basis<T>& bs,
                             int grid_mult, int variant, int waves, hipStream_t st, const T* lam, int64_t es,
                             int64_t ccs)
{
    if (lam) {
        switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_variants<n, T, true>(E, nrhs, verts, X, Y, bs, lam, grid_mult, variant, waves, st, es, ccs);
            AX_ITEM_CASE(9) AX_ITEM_CASE(10) AX_ITEM_CASE(11) AX_ITEM_CASE(12) AX_ITEM_CASE(13) AX_ITEM_CASE(14)
            AX_ITEM_CASE(15) AX_ITEM_CASE(16)
#undef AX_ITEM_CASE
        default: return fail(AX_ERR_UNSUPPORTED, "partial item kernel for N1=%d", N1);
        }
    }
    switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_variants<n, T, false>(E, nrhs, verts, X, Y, bs, nullptr, grid_mult, variant, waves, st, es, ccs);
        AX_ITEM_CASE(2) AX_ITEM_CASE(3) AX_ITEM_CASE(4) AX_ITEM_CASE(5) AX_ITEM_CASE(6) AX_ITEM_CASE(7)
        AX_ITEM_CASE(8) AX_ITEM_CASE(9) AX_ITEM_CASE(10) AX_ITEM_CASE(11) AX_ITEM_CASE(12) AX_ITEM_CASE(13)
        AX_ITEM_CASE(14) AX_ITEM_CASE(15) AX_ITEM_CASE(16)
#undef AX_ITEM_CASE
    default: return fail(AX_ERR_UNSUPPORTED, "item kernel for N1=%d", N1);
    }
}

}  // namespace ax
