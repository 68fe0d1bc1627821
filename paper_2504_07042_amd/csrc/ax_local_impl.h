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

#include <type_traits>

#include "ax_internal.h"
#include "ax_kernels.h"
#include "geom.h"

// 1: the even-odd kernels (mirror-symmetric nodes) read xi_k and w_k of the node loop from the
// first half of the kernel-argument tables, which stays resident in scalar registers next to
// the contraction coefficients; 0: every node reads them from an LDS table.
#ifndef AX_XW_SCALAR
#define AX_XW_SCALAR 1
#endif
// 1: the trilinear per-element prelude runs at the start of each item (fewest live registers);
// 0: between the forward r/s contractions and the pointwise stage.
#ifndef AX_EARLY_PRELUDE
#define AX_EARLY_PRELUDE 1
#endif
// 1: the s-direction transpose contraction goes back to LDS in place and the output stage sums
// the two fields (one barrier and one read-modify-write pass fewer); 0: it is added into the
// r-field through a separate pass.
#ifndef AX_MERGE_RS
#define AX_MERGE_RS 1
#endif

// 1: the FP32 N1 = 8 kernels run their D-contractions on the matrix cores (contract_mfma, 96
// v_mfma_f32_4x4x1f32 per element instead of 288 vector instructions); 0: on the vector ALU.
// Measured interleaved on gfx950 (trilinear, N = 7, 32^3): 65.8 us with the matrix cores against
// 52.0 us on the vector ALU, i.e. each 4x4x1 instruction costs about as much issue time as the
// vector work it replaces plus register pressure (128 VGPRs and spills); so 0.
#ifndef AX_F32_MFMA
#define AX_F32_MFMA 0
#endif

namespace ax {

template <int N1, bool EO, typename T>
constexpr bool use_mfma() { return AX_F32_MFMA && EO && sizeof(T) == 4 && N1 == 8; }

// Work-group shape for EPBX elements of order N1 - 1.
template <int N1, int EPBX>
struct Tile {
    static constexpr int NT = N1 * N1;
    static constexpr int EPB = EPBX;
    static constexpr int BLOCK = ((EPB * NT + 63) / 64) * 64;
    static constexpr int SLOTS = (BLOCK + NT - 1) / NT;
};

// Kernel argument block (one by-value struct, so that the contraction tables can also be read
// through the kernel-argument segment pointer; see CoefReload).
template <typename T>
struct AxArgs {
    int64_t E;
    int nrhs;
    const double* geo;
    const T* Gs;
    const T* X;
    T* Y;
    const int32_t* l2g;
    int64_t ldg;
    int64_t es, ccs;
    double* epart;
    Basis<T> bs;
};

// Orders whose contraction tables are read per output row instead of held in scalar registers.
// (measured on gfx950: the FP64 trilinear kernel at N1 = 10 is faster with resident tables)
template <int N1, int GEO, typename T>
constexpr bool reload_coefs() { return sizeof(T) == 8 ? N1 >= (is_trilinear(GEO) ? 11 : 10) : N1 >= 13; }

// (xi_k, w_k) of node k for the pointwise stage
template <int N1, int GEO, bool EO, typename T, typename B>
__device__ __forceinline__ void node_xw(const B& bs, const double* sxw, int k, T& t, T& wk)
{
    if constexpr (EO && AX_XW_SCALAR && !reload_coefs<N1, GEO, T>()) {
        const int m = k < N1 - 1 - k ? k : N1 - 1 - k;
        const double x = bs.xi[m];
        t = T(k == m ? x : -x);
        wk = T(bs.w[m]);
    } else {
        t = T(sxw[2 * k]);
        wk = T(sxw[2 * k + 1]);
    }
}

// Element at byte offset `off` (32-bit, non-negative) from a work-group-uniform base: the form
// the global loads and stores take with a scalar base register and a 32-bit lane offset.
template <typename P>
__device__ __forceinline__ P* at_bytes(P* base, uint32_t off)
{
    using C = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return reinterpret_cast<P*>(reinterpret_cast<C*>(base) + off);
}

// The r-pencil (., j, k) of a field: contiguous words i = 0..N1-1.  With layout 2 every pencil
// starts on a 16-byte boundary and moves as 16-byte accesses (two doubles or four floats each).
template <typename S, typename T>
__device__ __forceinline__ void rpencil_read(const T* F, int j, int k, T* p)
{
    constexpr int N1 = S::NN;
    if constexpr (S::L2) {
        constexpr int W = 16 / sizeof(T);  // values per 16-byte access
        typedef T v16 __attribute__((ext_vector_type(W)));
        const v16* q = reinterpret_cast<const v16*>(F + S::pos(0, j, k));
#pragma unroll
        for (int m = 0; m < N1 / W; ++m) {
            const v16 v = q[m];
#pragma unroll
            for (int u = 0; u < W; ++u) p[W * m + u] = v[u];
        }
    } else {
#pragma unroll
        for (int n = 0; n < N1; ++n) p[n] = F[S::pos(n, j, k)];
    }
}

template <typename S, typename T>
__device__ __forceinline__ void rpencil_write(T* F, int j, int k, const T* o)
{
    constexpr int N1 = S::NN;
    if constexpr (S::L2) {
        constexpr int W = 16 / sizeof(T);
        typedef T v16 __attribute__((ext_vector_type(W)));
        v16* q = reinterpret_cast<v16*>(F + S::pos(0, j, k));
#pragma unroll
        for (int m = 0; m < N1 / W; ++m) {
            v16 v;
#pragma unroll
            for (int u = 0; u < W; ++u) v[u] = o[W * m + u];
            q[m] = v;
        }
    } else {
#pragma unroll
        for (int a = 0; a < N1; ++a) F[S::pos(a, j, k)] = o[a];
    }
}

// Synchronisation of the work-group between LDS phases.  A work-group of one wave (N1 = 8 with one
// element per group) needs no hardware barrier and no wait for its LDS writes: the LDS performs the
// accesses of one wave in issue order, so a later read by any lane sees an earlier write by any
// lane.  Only the compiler must keep the order, which the wavefront-scope fences and the wave
// barrier enforce; no instruction is emitted, so the wave waits on LDS only where it uses a value.
#ifndef AX_WAVE_SYNC
#define AX_WAVE_SYNC 1
#endif
// Reading the s-pencil before the r-contraction of the same phase (so that its LDS latency
// overlaps the r-contraction) costs 16 or 8 live registers.  Measured on gfx950 at N1 = 8
// (interleaved): FP64 partial recomputation +8 %, FP32 trilinear and parallelepiped +4 %, FP64
// trilinear -8 % in both phases, FP64 parallelepiped -2 %; the other orders within 1-2 %.  AX_S_HOIST forces it
// on (1) or off (0) everywhere; by default it is used where it measured faster.
#ifndef AX_S_HOIST
#define AX_S_HOIST -1
#endif
// FP64 trilinear: in the forward phase only (measured +0.9 % at N1 = 8; in the transposed phase
// -10 %)
#ifndef AX_S_HOIST_F64_TRI
#define AX_S_HOIST_F64_TRI 1
#endif
// bit 0: the forward phase, bit 1: the transposed phase
template <int N1, int GEO, typename T>
constexpr int s_hoist()
{
    if constexpr (AX_S_HOIST >= 0) return AX_S_HOIST != 0 ? 3 : 0;
    if constexpr (N1 == 8 && sizeof(T) == 8 && GEO == GEO_TRI) return AX_S_HOIST_F64_TRI;
    return N1 == 8 && (sizeof(T) == 4 ? (GEO == GEO_TRI || GEO == GEO_PARA) : GEO == GEO_TRIL) ? 3 : 0;
}
template <int BLOCK>
__device__ __forceinline__ void group_sync()
{
    if constexpr (AX_WAVE_SYNC && BLOCK <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

#ifndef AX_GATHER_XCD
#define AX_GATHER_XCD 1
#endif

// Element groups of one mesh walked in order (group g holds elements [g EPB, g EPB + EPB)): the
// single-mesh launches, work-group b taking groups b, b + gridDim.x, ...  The batched launches
// pass either a work list of (mesh, group) items over many meshes of one order (kList), which
// supplies each group's addresses, or a slice of one mesh (kSlice: the work-group takes groups
// first, first + stride, ... of the mesh given to it).
struct OneMeshWalk {
    static constexpr bool kList = false;
    static constexpr bool kSlice = false;
};

// Kernel body.  GATHER 1: X is a global vector [nrhs][ldg] read through the local-to-global map
// l2g (the Q of Sec. 2.1 fused into the load), so the solver never materialises Q x.  GATHER 2
// (one column, the CG's operator): as 1, and each work-group also writes the sum of its
// elements' energies (D X_e)^T G_e (D X_e) = X_e^T Y_e to epart[blockIdx.x], which sums to
// p^T A p when X = Q p and p vanishes on the masked nodes.  `cs` is the source of the
// contraction coefficients (CoefResident, CoefReload or CoefConst).  Local vectors: node l of column c of
// element e at c * ccs + e * es + l (es = N1^3, ccs = E N1^3 for [nrhs][E][N1^3];
// es = nrhs N1^3, ccs = N1^3 for the component-interleaved [E][nrhs][N1^3] of a vector field).
// With a work list `wl` (W::kList, trilinear only, es = N1^3) the element groups and their
// addresses come from the list; E, geo, X, Y, l2g, ldg and ccs are then unused.
template <int N1, int GEO, bool EO, int GATHER, int EPBX, typename T, typename C, typename W = OneMeshWalk>
__device__ __forceinline__ void
ax_local_body(int64_t E, int nrhs, const double* __restrict__ geo, const T* __restrict__ Gs,
              const T* __restrict__ X, T* __restrict__ Y, const Basis<T>& bs,
              const int32_t* __restrict__ l2g, int64_t ldg, int64_t es, int64_t ccs, double* __restrict__ epart,
              const C& cs, const W& wl = W{})
{
    static_assert(!W::kList || GEO == GEO_TRI, "work lists carry trilinear meshes");
    using S = Shape<N1, sizeof(T)>;
    using TL = Tile<N1, EPBX>;
    constexpr int NT = S::NT, FS = S::FS, NP = S::NP, EPB = TL::EPB;
    constexpr int BLOCK = TL::BLOCK;
    constexpr int NV = is_trilinear(GEO) ? 24 : 0;               // vertex words per element
    constexpr int VPT = (EPB * NV + BLOCK - 1) / BLOCK;          // vertex words per thread
    __shared__ __attribute__((aligned(16))) T smem[TL::SLOTS * 2 * FS];
    __shared__ double svert[is_trilinear(GEO) ? EPB * 24 : 1];
    // (xi_k, w_k) pairs: the per-lane (xi_i, w_i), (xi_j, w_j) of the home columns, and xi_k, w_k
    // of the node loop for the kernels that do not keep them in scalar registers
    __shared__ double sxw[2 * N1];
    // GATHER 2: per-lane energy sums, kept in LDS so that they hold no register over the item
    __shared__ double sen[GATHER == 2 ? BLOCK : 1];
    lds_poison(smem, sizeof(smem));
    lds_poison(svert, sizeof(svert));
    lds_poison(sxw, sizeof(sxw));

    const int tid = threadIdx.x;
    if constexpr (GATHER == 2) sen[tid] = 0.0;
    const int slot = (TL::SLOTS == 1) ? 0 : tid / NT;
    const int lane = tid - slot * NT;
    T* __restrict__ A = smem + slot * 2 * FS;
    T* __restrict__ B = A + FS;
    const int i = lane % N1, j = lane / N1;    // home lane: node column (i, j, :)
    const int pa = S::spa(lane), pb = S::spb(lane);  // s-pencil lane (i, k)
    const int ra = S::rpa(lane), rb = S::rpb(lane);  // r-pencil lane (j, k)
    int64_t nblk;
    if constexpr (W::kList)
        nblk = wl.groups();
    else
        nblk = (E + EPB - 1) / EPB;
    if (tid < 2 * N1) sxw[tid] = (tid & 1) ? bs.w[tid >> 1] : bs.xi[tid >> 1];
    group_sync<BLOCK>();   // sxw is read by every wave from the first element on
    // the D-contractions: forward (D) and transposed (D^T), on the matrix cores or the vector ALU
    constexpr bool MF = use_mfma<N1, EO, T>();
    MfmaCoef<MF ? N1 : 2> kD, kT;
    if constexpr (MF) {
        mfma_coef_init<N1, false>(bs, (int)(threadIdx.x & 63), kD);
        mfma_coef_init<N1, true>(bs, (int)(threadIdx.x & 63), kT);
    }
    auto fwd = [&](const T* in, T* out) {
        if constexpr (MF)
            contract_mfma<N1>(kD, in, out);
        else
            contract<N1, false, EO>(cs, in, out);
    };
    auto bwd = [&](const T* in, T* out) {
        if constexpr (MF)
            contract_mfma<N1>(kT, in, out);
        else
            contract<N1, true, EO>(cs, in, out);
    };

    // Items are (element group, column) pairs walked in order; each work-group strides over the
    // element groups.  The next item's X (and vertices) are fetched into registers while the
    // current one is computed and staged into LDS at the end of the current item, so HBM latency
    // overlaps with a whole item of contraction work.  Addresses are a group-uniform base plus a
    // 32-bit lane offset; a group past the end is clamped to group 0 and slots past the last
    // element read the group's first element (results of such slots are never stored).
    auto clamp_group = [&](int64_t ebq) -> int64_t { return ebq < nblk ? ebq : 0; };
    auto slot_active = [&](int64_t g) -> bool {
        if constexpr (W::kList)
            return (slot < EPB) && wl.has(g, slot);
        else
            return (slot < EPB) && (g * EPB + slot < E);
    };
    // byte offset of node (i, j, 0) of this lane's element from the group's first node
    auto home_off = [&](bool act) -> uint32_t {
        return (uint32_t)(((act ? slot * es : 0) + i + j * N1) * (int64_t)sizeof(T));
    };
    auto load_x = [&](int64_t ebq, int cq, T* dst) {
        const int64_t g = clamp_group(ebq);
        const uint32_t lo = home_off(slot_active(g));
        if constexpr (GATHER) {
            const int32_t* mb;
            const T* xc;
            if constexpr (W::kList) {
                mb = wl.map(g);
                xc = wl.template xglob<T>(g, cq);
            } else {
                mb = l2g + g * EPB * NP;
                xc = X + (int64_t)cq * ldg;
            }
            int32_t gi[N1];
#pragma unroll
            for (int k = 0; k < N1; ++k) gi[k] = *at_bytes(mb, lo / sizeof(T) * 4 + k * NT * 4);
#pragma unroll
            for (int k = 0; k < N1; ++k) dst[k] = xc[gi[k]];
        } else {
            const T* src;
            if constexpr (W::kList)
                src = wl.template xsrc<T>(g, cq);
            else
                src = X + (int64_t)cq * ccs + g * EPB * es;
#pragma unroll
            for (int k = 0; k < N1; ++k) dst[k] = *at_bytes(src, lo + k * NT * (uint32_t)sizeof(T));
        }
    };
    auto load_v = [&](int64_t ebq, double* dst) {
        if constexpr (is_trilinear(GEO)) {
            const int64_t g = clamp_group(ebq);
            const double* src;
            int64_t lim;   // vertex words left from the group start
            if constexpr (W::kList) {
                src = wl.verts(g);
                lim = wl.left(g) * 24;
            } else {
                src = geo + g * EPB * 24;
                lim = (E - g * EPB) * 24;
            }
#pragma unroll
            for (int q = 0; q < VPT; ++q) {
                const int idx = tid + q * BLOCK;
                dst[q] = *at_bytes(src, (uint32_t)((idx < EPB * 24 && idx < lim ? idx : 0) * 8));
            }
        }
    };
    auto stage = [&](const T* x, const double* v, bool new_elem) {
#pragma unroll
        for (int k = 0; k < N1; ++k) A[S::pos(i, j, k)] = x[k];
        if constexpr (is_trilinear(GEO)) {
            if (new_elem) {
#pragma unroll
                for (int q = 0; q < VPT; ++q) {
                    const int idx = tid + q * BLOCK;
                    if (idx < EPB * 24) svert[idx] = v[q];
                }
            }
        }
    };

    // The gathering forms read shared nodes through l2g: elements adjacent in the mesh touch the
    // same cache lines of the global vector, so the work-groups of one XCD (one L2) take runs of
    // consecutive element groups (xcd_tile) instead of every eighth one.
    int64_t eb;
    if constexpr (W::kSlice)
        eb = wl.first;
    else if constexpr (GATHER != 0 && AX_GATHER_XCD)
        eb = xcd_tile(blockIdx.x, gridDim.x);
    else
        eb = blockIdx.x;
    int c = 0;
    T xr[N1];
    double vr[VPT > 0 ? VPT : 1];
    load_x(eb, 0, xr);
    load_v(eb, vr);
    stage(xr, vr, true);

    // where the trilinear prelude runs: at the item start (before the prefetch registers are
    // live) or between the forward r/s contractions and the pointwise stage
    constexpr bool EARLY = AX_EARLY_PRELUDE;
    TriCoefT<T> tc;
    double h[6];
    while (eb < nblk) {
        const bool active = slot_active(eb);
        const int64_t e = eb * EPB + slot;
        const bool last_col = (c + 1 == nrhs);
        int64_t eb_n;
        if constexpr (W::kSlice)
            eb_n = last_col ? eb + wl.stride : eb;
        else
            eb_n = last_col ? eb + gridDim.x : eb;
        const int c_n = last_col ? 0 : c + 1;
        if constexpr (GEO == GEO_PARA) {
            if (c == 0) {
                const double* he = geo + (active ? e : 0) * 6;
                const double wij = sxw[2 * i + 1] * sxw[2 * j + 1];
#pragma unroll
                for (int q = 0; q < 6; ++q) h[q] = he[q] * wij;
            }
        }
        // P0: (per-element geometry invariants of the home column from the staged vertices, at
        // the point of the item where the fewest registers are live,) t-contraction in
        // registers, then the next item's loads
        if constexpr (EARLY) {
            group_sync<BLOCK>();
            if constexpr (is_trilinear(GEO)) {
                if (c == 0) {
                    const double* sv = svert + (slot < EPB ? slot : 0) * 24;
                    TriCoef t64;
                    tri_prelude([&](int v, int q) { return sv[v * 3 + q]; }, sxw[2 * i], sxw[2 * j],
                                sxw[2 * i + 1], sxw[2 * j + 1], t64);
                    tri_narrow(t64, tc);
                }
            }
        }
        T x2[N1];
        fwd(xr, x2);  // x2 = D_t x
        T xn[N1];
        load_x(eb_n, c_n, xn);
        if (last_col) load_v(eb_n, vr);
        if constexpr (!EARLY) group_sync<BLOCK>();
        // P1: r-pencils (j,k) -> x0 in B; s-pencils (i,k) -> x1 held in registers
        T o1[N1];
        {
            T p[N1], o[N1];
            rpencil_read<S>(A, ra, rb, p);
            if constexpr ((s_hoist<N1, GEO, T>() & 1) != 0) {
                // the s-pencil is read before the r-contraction so that its latency overlaps it
                T q[N1];
#pragma unroll
                for (int n = 0; n < N1; ++n) q[n] = A[S::pos(pa, n, pb)];
                fwd(p, o);
                rpencil_write<S>(B, ra, rb, o);
                fwd(q, o1);
            } else {
                fwd(p, o);
                rpencil_write<S>(B, ra, rb, o);
#pragma unroll
                for (int n = 0; n < N1; ++n) p[n] = A[S::pos(pa, n, pb)];
                fwd(p, o1);
            }
        }
        group_sync<BLOCK>();
        // P2: x1 -> A; (per-element geometry invariants of the home column from the staged vertices)
#pragma unroll
        for (int a = 0; a < N1; ++a) A[S::pos(pa, a, pb)] = o1[a];
        if constexpr (is_trilinear(GEO) && !EARLY) {
            if (c == 0) {
                const double* sv = svert + (slot < EPB ? slot : 0) * 24;
                TriCoef t64;
                tri_prelude([&](int v, int q) { return sv[v * 3 + q]; }, sxw[2 * i], sxw[2 * j], sxw[2 * i + 1],
                            sxw[2 * j + 1], t64);
                tri_narrow(t64, tc);
            }
        }
        group_sync<BLOCK>();
        // P3: pointwise factors at the home column; r -> B, s -> A, t stays in registers
        T tt[N1];
        T ei = T(0);  // GATHER 2: this item's energy at the home column
#pragma unroll
        for (int k = 0; k < N1; ++k) {
            const int l = S::pos(i, j, k);
            T x0 = B[l], x1 = A[l], xx2 = x2[k];
            T g[6];
            T lam_out = T(1);  // GATHER 2: lambda applied to the outputs, after the energy
            if constexpr (GEO == GEO_TRI) {
                T lam;
                T tk, wk;
                node_xw<N1, GEO, EO>(bs, sxw, k, tk, wk);
                tri_adj<T>(tc, tk, wk, g, lam);
                if constexpr (GATHER == 2) {
                    lam_out = lam;
                } else {
                    x0 *= lam;
                    x1 *= lam;
                    xx2 *= lam;
                }
            } else if constexpr (GEO == GEO_TRIL || GEO == GEO_HELM) {
                T tk, wk;
                node_xw<N1, GEO, EO>(bs, sxw, k, tk, wk);
                constexpr int LS = GEO == GEO_HELM ? 2 : 1;  // fields per element in Gs
                const T lam = Gs[(active ? e : 0) * LS * NP + i + j * N1 + k * NT];
                tri_adj_k<T>(tc, tk, g);
                x0 *= lam;
                x1 *= lam;
                xx2 *= lam;
            } else if constexpr (GEO == GEO_PARA) {
                T tk, wk;
                node_xw<N1, GEO, EO>(bs, sxw, k, tk, wk);
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = T(h[q]) * wk;
            } else {
                const T* ge = Gs + (active ? e : 0) * 6 * NP + i + j * N1 + k * NT;
#pragma unroll
                for (int q = 0; q < 6; ++q) g[q] = active ? ge[q * NP] : T(0);
            }
            if constexpr (GATHER == 2) {
                T bo = fma(g[0], x0, fma(g[1], x1, g[2] * xx2));
                T ao = fma(g[1], x0, fma(g[3], x1, g[4] * xx2));
                T to = fma(g[2], x0, fma(g[4], x1, g[5] * xx2));
                // the node's energy (D X)^T G (D X) with G = lambda g, then G (D X) itself
                if (active) ei += lam_out * fma(x0, bo, fma(x1, ao, xx2 * to));
                if constexpr (GEO == GEO_TRI) {
                    bo *= lam_out;
                    ao *= lam_out;
                    to *= lam_out;
                }
                B[l] = bo;
                A[l] = ao;
                tt[k] = to;
            } else {
                B[l] = fma(g[0], x0, fma(g[1], x1, g[2] * xx2));
                A[l] = fma(g[1], x0, fma(g[3], x1, g[4] * xx2));
                tt[k] = fma(g[2], x0, fma(g[4], x1, g[5] * xx2));
            }
        }
        if constexpr (GATHER == 2) sen[tid] += (double)ei;
        T y2[N1];
        bwd(tt, y2);  // D_t^T t
        // Helmholtz: Lambda3 and this item's X at the home column for the mass term, loaded here
        // (X again, now from the cache) so that they are in flight during the next phase
        T l3v[GEO == GEO_HELM ? N1 : 1], xv[GEO == GEO_HELM ? N1 : 1];
        if constexpr (GEO == GEO_HELM) {
            const T* l3 = Gs + ((active ? e : 0) * 2 + 1) * NP + i + j * N1;
#pragma unroll
            for (int k = 0; k < N1; ++k) l3v[k] = l3[k * NT];
            load_x(eb, c, xv);
        }
        group_sync<BLOCK>();
        // P4: D_r^T r in place on the r-pencils; D_s^T s into registers
        {
            T p[N1], o[N1];
            rpencil_read<S>(B, ra, rb, p);
            if constexpr ((s_hoist<N1, GEO, T>() & 2) != 0) {
                T q[N1];
#pragma unroll
                for (int n = 0; n < N1; ++n) q[n] = A[S::pos(pa, n, pb)];
                bwd(p, o);
                rpencil_write<S>(B, ra, rb, o);
                bwd(q, o1);
            } else {
                bwd(p, o);
                rpencil_write<S>(B, ra, rb, o);
#pragma unroll
                for (int n = 0; n < N1; ++n) p[n] = A[S::pos(pa, n, pb)];
                bwd(p, o1);
            }
#if AX_MERGE_RS
            // each s-pencil is read and written by its own lane only
#pragma unroll
            for (int a = 0; a < N1; ++a) A[S::pos(pa, a, pb)] = o1[a];
#endif
        }
        group_sync<BLOCK>();
        if constexpr (GEO == GEO_HELM) {
#pragma unroll
            for (int k = 0; k < N1; ++k) y2[k] = fma(l3v[k], xv[k], y2[k]);
        }
        T* yb;
        if constexpr (W::kList)
            yb = wl.template ydst<T>(eb, c);
        else
            yb = Y + (int64_t)c * ccs + eb * EPB * es;
        const uint32_t lo = home_off(true);
#if AX_MERGE_RS
        // P5: Y = (D_r^T r + D_s^T s) + D_t^T t
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k) {
                const int l = S::pos(i, j, k);
                *at_bytes(yb, lo + k * NT * (uint32_t)sizeof(T)) = (B[l] + A[l]) + y2[k];
            }
        }
#else
        // P5: add D_s^T s on the s-pencils
#pragma unroll
        for (int a = 0; a < N1; ++a) B[S::pos(pa, a, pb)] += o1[a];
        group_sync<BLOCK>();
        // P6: Y = (D_r^T r + D_s^T s) + D_t^T t
        if (active) {
#pragma unroll
            for (int k = 0; k < N1; ++k)
                *at_bytes(yb, lo + k * NT * (uint32_t)sizeof(T)) = B[S::pos(i, j, k)] + y2[k];
        }
#endif
        // stage the next item: this lane's own home positions (read above by this lane only)
        // and the vertex table (last read before the barriers of P3 and P4)
        stage(xn, vr, last_col);
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = xn[k];
        eb = eb_n;
        c = c_n;
    }
    if constexpr (GATHER == 2) {
        // the work-group's energy: wave sums, then the waves in order (a fixed combination)
        double en = sen[tid];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) en += __shfl_xor(en, off);
        if constexpr (BLOCK == 64) {
            if (tid == 0) epart[blockIdx.x] = en;
        } else {
            __shared__ double ered[BLOCK / 64];
            if ((tid & 63) == 0) ered[tid >> 6] = en;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < BLOCK / 64; ++q) s += ered[q];
                epart[blockIdx.x] = s;
            }
        }
    }
}

template <int N1, int GEO, typename T>
constexpr int min_waves()
{
    return tile_waves(N1, GEO, sizeof(T) == 4);
}

// Entry points: the tables of orders that fit the scalar register file stay resident; the
// others are reloaded per output row through the kernel-argument segment (one struct argument).
template <int N1, int GEO, bool EO, int GATHER, int EPBX, typename T>
__global__ void __launch_bounds__((Tile<N1, EPBX>::BLOCK), (min_waves<N1, GEO, T>()))
ax_local_kernel(int64_t E, int nrhs, const double* __restrict__ geo, const T* __restrict__ Gs,
                const T* __restrict__ X, T* __restrict__ Y, const Basis<T> bs,
                const int32_t* __restrict__ l2g, int64_t ldg, int64_t es, int64_t ccs, double* __restrict__ epart)
{
    ax_local_body<N1, GEO, EO, GATHER, EPBX, T>(E, nrhs, geo, Gs, X, Y, bs, l2g, ldg, es, ccs, epart,
                                                CoefResident<T>{bs});
}

template <int N1, int GEO, bool EO, int GATHER, int EPBX, typename T>
__global__ void __launch_bounds__((Tile<N1, EPBX>::BLOCK), (min_waves<N1, GEO, T>()))
ax_local_kernel_rl(const AxArgs<T> ka)
{
    const CoefReload<T> cs = karg_coefs<T, AxArgs<T>>();
    ax_local_body<N1, GEO, EO, GATHER, EPBX, T>(ka.E, ka.nrhs, ka.geo, ka.Gs, ka.X, ka.Y, ka.bs, ka.l2g, ka.ldg, ka.es,
                                                ka.ccs, ka.epart, cs);
}

// fo (GATHER 2 only): the energy partials; fo->nparts gets the grid size.
template <int N1, int GEO, bool EO, int GATHER, int EPBX, typename T>
static int launch_tile(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y, const Basis<T>& bs,
                       int grid_mult, hipStream_t st, const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs,
                       FusedOut* fo = nullptr)
{
    using TL = Tile<N1, EPBX>;
    static int per = 0;  // resident work-groups per CU for this instantiation
    static int cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        const void* kf;
        if constexpr (reload_coefs<N1, GEO, T>())
            kf = reinterpret_cast<const void*>(ax_local_kernel_rl<N1, GEO, EO, GATHER, EPBX, T>);
        else
            kf = reinterpret_cast<const void*>(ax_local_kernel<N1, GEO, EO, GATHER, EPBX, T>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, kf, TL::BLOCK, 0) != hipSuccess || q < 1)
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
    double* epart = nullptr;
    if constexpr (GATHER == 2) {
        if (!fo || !fo->epart) return fail(AX_ERR_ARG, "internal: fused AxLocal without its energy partials");
        if (blocks > fo->epart_cap) return fail(AX_ERR_ARG, "internal: energy partials hold %lld, need %lld",
                                                (long long)fo->epart_cap, (long long)blocks);
        epart = fo->epart;
        fo->nparts = blocks;
    }
    if constexpr (reload_coefs<N1, GEO, T>()) {
        const AxArgs<T> ka{E, nrhs, geo, Gs, X, Y, l2g, ldg, es, ccs, epart, bs};
        hipLaunchKernelGGL((ax_local_kernel_rl<N1, GEO, EO, GATHER, EPBX, T>), dim3((unsigned)blocks),
                           dim3(TL::BLOCK), 0, st, ka);
    } else {
        hipLaunchKernelGGL((ax_local_kernel<N1, GEO, EO, GATHER, EPBX, T>), dim3((unsigned)blocks), dim3(TL::BLOCK),
                           0, st, E, nrhs, geo, Gs, X, Y, bs, l2g, ldg, es, ccs, epart);
    }
    return hip_check(hipGetLastError(), "ax_local launch");
}

int tri_item_dispatch_f64(int N1, int64_t E, int nrhs, const double* verts, const double* X, double* Y,
                          const Basis<double>& bs, int grid_mult, int variant, int waves, hipStream_t st,
                          const double* lam, int64_t es, int64_t ccs);
int tri_item_dispatch_f32(int N1, int64_t E, int nrhs, const double* verts, const float* X, float* Y,
                          const Basis<float>& bs, int grid_mult, int variant, int waves, hipStream_t st,
                          const float* lam, int64_t es, int64_t ccs);

template <int N1, int GEO, typename T>
static int launch_n1(int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                     const double* D, const double* xi, const double* w, hipStream_t st,
                     const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs, FusedOut* fo)
{
    using S = Shape<N1>;
    Basis<T> bs;
    fill_basis(bs, N1, D, xi, w);
    // the even-odd kernels also take the nodes as mirror-symmetric (the factors need none)
    const bool eo = centro_antisymmetric(N1, D) && (GEO == GEO_STORED || symmetric_nodes(N1, xi, w));
    const TuneEntry tu = tune_get(N1, tune_kind_of(GEO), sizeof(T) == 8 ? AX_FP64 : AX_FP32);
    if (l2g) {
        if (!eo) return fail(AX_ERR_UNSUPPORTED, "gathering AxLocal needs a GLL differentiation matrix");
        if constexpr (GEO == GEO_TRI || GEO == GEO_PARA) {
            if (fo) {
                // energies fused in FP32 only: in FP64 the kernel's extra register pressure cost as
                // much as the p read it saves in Q^T
                if constexpr (sizeof(T) == 4)
                    return launch_tile<N1, GEO, true, 2, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, l2g,
                                                                    ldg, es, ccs, fo);
                return fail(AX_ERR_UNSUPPORTED, "internal: the fused operator is FP32");
            }
            return launch_tile<N1, GEO, true, 1, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, l2g, ldg, es, ccs);
        }
        return fail(AX_ERR_UNSUPPORTED, "gathering AxLocal needs on-the-fly factors");
    }
    // the per-item kernel where the tuning table (or the measured default) picks it
    if constexpr (item_available(N1, GEO)) {
        const bool item = tu.kernel == AX_KERNEL_ITEM ||
                          (tu.kernel == AX_KERNEL_AUTO && item_default(N1, GEO, sizeof(T) == 4));
        if (eo && item) {
            if constexpr (sizeof(T) == 8)
                return tri_item_dispatch_f64(N1, E, nrhs, geo, (const double*)X, (double*)Y, bs, tu.grid_mult,
                                             tu.item_alt, tu.waves_alt, st,
                                             GEO == GEO_TRIL ? (const double*)Gs : nullptr, es, ccs);
            else
                return tri_item_dispatch_f32(N1, E, nrhs, geo, X, Y, bs, tu.grid_mult, tu.item_alt, tu.waves_alt, st,
                                             GEO == GEO_TRIL ? (const float*)Gs : nullptr, es, ccs);
        }
    }
    if (!eo)
        return launch_tile<N1, GEO, false, false, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, nullptr, 0, es, ccs);
    if constexpr (S::EPB_ALT != S::EPB) {
        if (tu.tile_alt)
            return launch_tile<N1, GEO, true, false, S::EPB_ALT, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st,
                                                                    nullptr, 0, es, ccs);
    }
    return launch_tile<N1, GEO, true, false, S::EPB, T>(E, nrhs, geo, Gs, X, Y, bs, tu.grid_mult, st, nullptr, 0, es, ccs);
}

template <int GEO, typename T>
static int dispatch(int N, int64_t E, int nrhs, const double* geo, const T* Gs, const T* X, T* Y,
                    const double* D, const double* xi, const double* w, hipStream_t st,
                    const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs, FusedOut* fo)
{
    if (fo && (!l2g || nrhs != 1)) return fail(AX_ERR_ARG, "internal: the fused operator takes one gathered column");
    switch (N + 1) {
#define AX_CASE(n1) \
    case n1: return launch_n1<n1, GEO, T>(E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
        AX_CASE(2) AX_CASE(3) AX_CASE(4) AX_CASE(5) AX_CASE(6) AX_CASE(7) AX_CASE(8) AX_CASE(9)
        AX_CASE(10) AX_CASE(11) AX_CASE(12) AX_CASE(13) AX_CASE(14) AX_CASE(15) AX_CASE(16)
#undef AX_CASE
    default:
        return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    }
}
}  // namespace ax
