// Element-level building blocks shared by the AxLocal kernels (internal header): work-group
// shapes per order and the one-dimensional D-contractions.
#pragma once

#include "ax_internal.h"

namespace ax {

// GEO_TRIL: trilinear with the per-node scale lam = 0.125 w / det(8J) read from memory (the
// partial recomputation of Sec. 4.2.2): no determinant and no division in the kernel.
// GEO_HELM: the trilinear Helmholtz operator with merged scalar factors (Sec. 4.2.1): per node
// Lambda2 = lam * lambda0 scales adj(K) and Lambda3 = gwj * lambda1 the mass term.
enum { GEO_TRI = 0, GEO_PARA = 1, GEO_STORED = 2, GEO_TRIL = 3, GEO_HELM = 4 };

constexpr bool is_trilinear(int geo) { return geo == GEO_TRI || geo == GEO_TRIL || geo == GEO_HELM; }

// ---- Launch variants chosen at run time (the tuning table, ax_tune_set) ----
//
// Tuning kinds: one table entry per (order, kind, precision).
enum { TUNE_TRI = 0, TUNE_PARA = 1, TUNE_STORED = 2, TUNE_PARTIAL = 3, TUNE_HELM = 4, TUNE_BATCHED = 5,
       TUNE_KINDS = 6 };
constexpr int tune_kind_of(int geo)
{
    return geo == GEO_TRI ? TUNE_TRI : geo == GEO_PARA ? TUNE_PARA : geo == GEO_STORED ? TUNE_STORED
         : geo == GEO_TRIL ? TUNE_PARTIAL : TUNE_HELM;
}

// Shape of the per-item kernels (one element per N1^2 lanes, several elements per work-group):
// variant 0 is a 256-lane work-group holding floor(256 / N1^2) elements (at most 64); variant 1
// is the alternative the tuner may pick: half the work-group for N1 <= 8 (smaller groups, cheaper
// barriers), a larger group for N1 = 9, 10 and a tighter one for N1 = 11..13 (fewer idle lanes:
// at N1 = 12 the 256-lane group leaves 112 lanes idle, a 192-lane group 48).  N1 >= 14 has no
// alternative.
struct ItemShape {
    int epb, block;
};
constexpr ItemShape item_shape(int N1, int v)
{
    if (v == 1) {
        switch (N1) {
        case 2: return {32, 128};
        case 3: return {14, 128};
        case 4: return {8, 128};
        case 5: return {5, 128};
        case 6: return {5, 192};
        case 7: return {2, 128};
        case 8: return {2, 128};
        case 9: return {4, 384};
        case 10: return {3, 320};
        case 11: return {1, 128};
        case 12: return {1, 192};
        case 13: return {1, 192};
        default: break;
        }
    }
    return {256 / (N1 * N1) > 64 ? 64 : (256 / (N1 * N1) < 1 ? 1 : 256 / (N1 * N1)), 256};
}
constexpr bool item_has_alt(int N1) { return N1 >= 2 && N1 <= 13; }

// Register budget of the single-mesh per-item kernel, as waves per SIMD: the default (FP32 full
// form five waves except at N1 = 13, otherwise no limit beyond two) and the alternative (one wave
// more where the default is two, one fewer where it is five).
constexpr int item_waves(int N1, bool fp32, bool partial, int alt)
{
    const int d = (fp32 && !partial && N1 != 13) ? 5 : 2;
    return alt ? (d == 2 ? 3 : 4) : d;
}

// Which kernel runs when the tuning table says "auto" (measured on gfx950, interleaved runs).
// FP64 full form: the per-item kernel for N1 = 6, 7 and 9..15 (faster than the prefetching
// kernel there, about even at N1 = 5, slower at N1 <= 4, 8 and 16).  FP64 partial form: the
// per-item kernel from N1 = 9 (the prefetching kernel, with fewer live registers in this form,
// was faster at N1 = 6).  FP32 full form: the per-item kernel from N1 = 9 (at five waves per SIMD:
// +7-8 % at N1 = 9 and 10, +13-15 % at N1 = 12, 15, where the prefetching kernel runs at two).
// FP32 partial form: from N1 = 13 (+18 % at 13, +7 % at 14, +2 % at 15; even at 10 and 8-10 %
// behind at 11, 12).
#ifndef AX_ITEM_LO
#define AX_ITEM_LO 6
#endif
#ifndef AX_ITEM_LO_F32
#define AX_ITEM_LO_F32 9
#endif
#ifndef AX_ITEM_PL_LO_F32
#define AX_ITEM_PL_LO_F32 13
#endif
constexpr bool item_default(int N1, int geo, bool fp32)
{
    if (N1 > 15) return false;
    if (fp32)
        return (geo == GEO_TRI && N1 >= AX_ITEM_LO_F32 && N1 >= 9) ||
               (geo == GEO_TRIL && N1 >= AX_ITEM_PL_LO_F32 && N1 >= 13);
    return (geo == GEO_TRI && N1 >= AX_ITEM_LO && N1 != 8) || (geo == GEO_TRIL && N1 >= 9);
}

// Orders with a batched tile kernel (the single-mesh tile body walking the batch's work list):
// FP64 up to N1 = 7, FP32 up to N1 = 10.  At FP64 N1 >= 8 the kernel spills (N1 = 8: 464-496
// bytes of scratch with the tables resident, read through the constant address space or reloaded
// per row, whether or not the item descriptors are re-read at each use; 45 against 214 GDOF/s for
// the per-item kernel on sixteen order-7 meshes of 512 to 32768 elements, 8 columns).
constexpr bool batched_tile_available(int N1, bool fp32) { return fp32 ? N1 <= 10 : N1 <= 7; }

// Register budget of the batched per-order kernels: FP32 fits five waves per SIMD.
#ifndef AX_BATCH_MINW_F32
#define AX_BATCH_MINW_F32 5
#endif
constexpr int batch_waves(bool fp32) { return fp32 ? AX_BATCH_MINW_F32 : 2; }

// Orders with a per-item kernel: the full trilinear form for every order, the partial form from
// N1 = 9.
constexpr bool item_available(int N1, int geo)
{
    return (geo == GEO_TRI && N1 >= 2 && N1 <= 16) || (geo == GEO_TRIL && N1 >= 9 && N1 <= 16);
}

// Tuning knobs (compile-time): waves per SIMD the register allocation targets for N1 <= 8, and
// how many times the resident capacity the persistent grid is.
#ifndef AX_MINW_SMALL
#define AX_MINW_SMALL 4
#endif
#ifndef AX_MINW_OTHER
#define AX_MINW_OTHER 2
#endif
#ifndef AX_PERSIST_MULT
#define AX_PERSIST_MULT 2
#endif
// XOR-swizzled LDS layout for N1 = 8 (no padding; conflict-free for the home, r-pencil and
// s-pencil access patterns) instead of the padded row stride.
#ifndef AX_LDS_SWIZZLE
#define AX_LDS_SWIZZLE 0
#endif
// LDS layout for N1 = 8: 0 = word i + 9 j + 72 k (row stride padded to 9); 1 = word
// i + 8 j + 65 k with the r-pencils assigned to lanes k-fastest; 2 (8-byte words only) = word
// i + 8 j + 66 k, r-pencils k-fastest and moved as 16-byte accesses, s-pencils assigned so that
// each group of 16 lanes takes the slices k and k + 4 (4-byte words: i + 8 j + 68 k, each group
// of 32 lanes takes the slices k = 0, 2, 4, 6 or 1, 3, 5, 7, so i + 4 k covers the 32 banks; a
// 16-byte r-pencil access starts at bank 8 j + 4 k, 8 lanes k = 0..7 cover them).  With 64-bit
// accesses served 16 lanes per
// clock over 32 four-byte banks, layout 0 is conflict-free for the r- and s-pencils and 2-way
// conflicted for the home columns; layout 1 is conflict-free for the home columns and the
// r-pencils and 2-way conflicted for the s-pencils (no additive layout is conflict-free for all
// three patterns with lanes taking pencils in order); layout 2 is conflict-free for all three:
// home columns i + 8 j (two rows j per 16 lanes) cover the 16 double-word banks, each 16-byte
// r-pencil access starts at bank 2 k (8 lanes k = 0..7 cover the 16 banks), and s-pencil lanes
// i + 2 k with k and k + 4 cover them too.
#ifndef AX_LDS_LAYOUT
#define AX_LDS_LAYOUT 2
#endif

// Element shape of order N1 - 1 and its LDS layout; WB = bytes per stored value.
template <int N1, int WB = 8>
struct Shape {
    static constexpr int NN = N1;                             // points per direction
    static constexpr int NT = N1 * N1;                        // lanes per element
    static constexpr bool SWZ = AX_LDS_SWIZZLE && N1 == 8;
    static constexpr bool L2 = !SWZ && AX_LDS_LAYOUT == 2 && N1 == 8 && (WB == 8 || WB == 4);
    static constexpr bool L1 = !SWZ && AX_LDS_LAYOUT == 1 && N1 == 8;
    static constexpr int SJ = (L1 || L2) ? 8 : (N1 % 2 == 0) ? N1 + 1 : N1;   // LDS row stride
    static constexpr int SK = L2 ? (WB == 8 ? 66 : 68) : L1 ? 65 : N1 * SJ;    // LDS slice stride
    static constexpr int FS = SWZ ? 512 : (L1 || L2) ? 8 * SK : N1 * SK;       // LDS words per field
    // LDS word of node (i, j, k) within one field
    __device__ static __forceinline__ int pos(int i, int j, int k)
    {
        if constexpr (SWZ)
            return 64 * k + 8 * (j ^ (k & 1)) + (i ^ ((j >> 1) << 1));
        else
            return k * SK + j * SJ + i;
    }
    // pencil lanes: the r-pencil (j, k) and the s-pencil (i, k) a lane owns
    __device__ static __forceinline__ int rpa(int lane) { return (L1 || L2) ? lane / N1 : lane % N1; }
    __device__ static __forceinline__ int rpb(int lane) { return (L1 || L2) ? lane % N1 : lane / N1; }
    __device__ static __forceinline__ int spa(int lane) { return lane % N1; }
    __device__ static __forceinline__ int spb(int lane)
    {
        if constexpr (L2 && WB == 8) return ((lane >> 3) & 1) * 4 + (lane >> 4);
        if constexpr (L2 && WB == 4) return 2 * ((lane >> 3) & 3) + (lane >> 5);
        return lane / N1;
    }
    static constexpr int NP = N1 * N1 * N1;                   // nodes per element
    // elements per work-group: fill (nearly) whole waves while keeping LDS modest
    static constexpr int EPB = N1 == 2 ? 16 : N1 == 3 ? 7 : N1 == 4 ? 4 : N1 == 5 ? 5
                             : N1 == 6 ? 7 : N1 == 7 ? 5 : N1 == 9 ? 3 : N1 == 10 ? 3
                             : N1 == 11 ? 2 : 1;
    // the alternative elements-per-group the tuner may pick (same as EPB where there is none)
    static constexpr int EPB_ALT = N1 == 2 ? 32 : N1 == 3 ? 14 : N1 == 4 ? 8 : N1 == 5 ? 10
                                 : N1 == 6 ? 14 : N1 == 7 ? 10 : N1 == 8 ? 2 : N1 <= 11 ? 1 : EPB;
    static constexpr int BLOCK = ((EPB * NT + 63) / 64) * 64;
    static constexpr int SLOTS = (BLOCK + NT - 1) / NT;
    // waves per SIMD the register allocation must allow (latency hiding for the X/Y streams)
    static constexpr int MINW = N1 == 8 ? AX_MINW_SMALL : AX_MINW_OTHER;
};

// Waves per SIMD the register allocation of the prefetching (tile) kernel targets: four at
// N1 = 8 and two elsewhere (AX_MINW_SMALL / AX_MINW_OTHER), except that the FP64 Helmholtz kernel
// at N1 = 8 also carries the mass-term operands through the last phases, which does not fit the
// four-wave budget without spills, and FP32 at N1 = 8, measured interleaved at N = 7, 32^3 with
// LDS layout 2: the trilinear kernel is fastest at four (49.3 us; five spill 6 registers,
// 52.0 us; six 58.2 us), partial recomputation at five (47.0 vs 48.6 us at four),
// parallelepipeds and stored factors within 1 % of each other from four to six.
#ifndef AX_HELM_MINW
#define AX_HELM_MINW 3
#endif
#ifndef AX_MINW_F32
#define AX_MINW_F32 5
#endif
#ifndef AX_MINW_F32_TRI
#define AX_MINW_F32_TRI 4
#endif
#ifndef AX_MINW_TINY
#define AX_MINW_TINY AX_MINW_OTHER
#endif
#ifndef AX_MINW_MID
#define AX_MINW_MID AX_MINW_OTHER
#endif
constexpr int tile_waves(int N1, int geo, bool fp32)
{
    return (geo == GEO_HELM && N1 == 8 && !fp32) ? AX_HELM_MINW
           : (N1 == 8 && fp32)                  ? (geo == GEO_TRI ? AX_MINW_F32_TRI : AX_MINW_F32)
           : N1 == 8                            ? AX_MINW_SMALL
           : N1 <= 4                            ? AX_MINW_TINY
           : N1 <= 7                            ? AX_MINW_MID
                                                : AX_MINW_OTHER;
}

// Coefficient sources of the contractions.  CoefResident reads the basis tables as they are
// (kernel arguments: the compiler keeps every coefficient it needs in scalar registers).
// CoefReload reads them through a pointer into the kernel-argument segment that is made opaque
// before each output row, so only one row of coefficients is live in scalar registers at a time
// (scalar loads from the scalar cache): for orders whose tables do not fit the scalar register
// file, where keeping them resident would spill them into vector-register lanes.
template <typename T>
struct CoefResident {
    const Basis<T>& b;
    __device__ __forceinline__ CoefResident row() const { return *this; }
    __device__ __forceinline__ T D(int q) const { return b.D[q]; }
    __device__ __forceinline__ T P(int q) const { return b.P[q]; }
    __device__ __forceinline__ T M(int q) const { return b.M[q]; }
    __device__ __forceinline__ T Cm(int q) const { return b.Cm[q]; }
    __device__ __forceinline__ T Rm(int q) const { return b.Rm[q]; }
    __device__ __forceinline__ double xi(int q) const { return b.xi[q]; }
    __device__ __forceinline__ double w(int q) const { return b.w[q]; }
};

template <typename KA>
using KargPtr = const __attribute__((address_space(4))) KA*;

// The tables behind a constant-address-space pointer (the kernel-argument segment, or a device
// table that the kernel only reads), which keeps the loads on the scalar unit.
template <typename T>
struct CoefReload {
    KargPtr<Basis<T>> k;
    __device__ __forceinline__ CoefReload row() const
    {
        KargPtr<Basis<T>> q = k;
        asm volatile("" : "+s"(q));
        return CoefReload{q};
    }
    __device__ __forceinline__ T D(int q) const { return k->D[q]; }
    __device__ __forceinline__ T P(int q) const { return k->P[q]; }
    __device__ __forceinline__ T M(int q) const { return k->M[q]; }
    __device__ __forceinline__ T Cm(int q) const { return k->Cm[q]; }
    __device__ __forceinline__ T Rm(int q) const { return k->Rm[q]; }
    __device__ __forceinline__ double xi(int q) const { return k->xi[q]; }
    __device__ __forceinline__ double w(int q) const { return k->w[q]; }
};

// Basis tables in device memory read through the constant address space and left to the
// compiler to keep in scalar registers or reload (loads there are invariant, so it can
// rematerialise them under register pressure instead of spilling): the resident tables of a
// kernel that receives them by pointer.
template <typename T>
struct CoefConst {
    KargPtr<Basis<T>> k;
    __device__ __forceinline__ CoefConst row() const { return *this; }
    __device__ __forceinline__ T D(int q) const { return k->D[q]; }
    __device__ __forceinline__ T P(int q) const { return k->P[q]; }
    __device__ __forceinline__ T M(int q) const { return k->M[q]; }
    __device__ __forceinline__ T Cm(int q) const { return k->Cm[q]; }
    __device__ __forceinline__ T Rm(int q) const { return k->Rm[q]; }
    __device__ __forceinline__ double xi(int q) const { return k->xi[q]; }
    __device__ __forceinline__ double w(int q) const { return k->w[q]; }
};

// Basis member `bs` of the kernel's single by-value argument struct KA.
template <typename T, typename KA>
__device__ __forceinline__ CoefReload<T> karg_coefs()
{
    const KargPtr<KA> ka = (KargPtr<KA>)__builtin_amdgcn_kernarg_segment_ptr();
    return CoefReload<T>{&ka->bs};
}

// A device pointer that every lane shares (moved to scalar registers), viewed in the constant
// address space.
template <typename T>
__device__ __forceinline__ KargPtr<T> as_constant(const T* p)
{
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (KargPtr<T>)(uintptr_t)(lo | (hi << 32));
}

// out[a] = sum_n D[a][n] in[n]   (TRANS: out[a] = sum_n D[n][a] in[n])
template <int N1, bool TRANS, typename T, typename C>
__device__ __forceinline__ void contract_full(const C& src, const T* in, T* out)
{
#pragma unroll
    for (int a = 0; a < N1; ++a) {
        const C c = src.row();
        T acc = T(0);
#pragma unroll
        for (int n = 0; n < N1; ++n) acc = fma(c.D(TRANS ? n * N1 + a : a * N1 + n), in[n], acc);
        out[a] = acc;
    }
}

// The same contraction for a centro-antisymmetric D by its even-odd split (H = N1/2 squared
// blocks P and M, see Basis): with ue[n] = in[n] + in[N-n], uo[n] = in[n] - in[N-n],
//   e[a] = sum_n P[a][n] ue[n],  o[a] = sum_n M[a][n] uo[n],  out[a] = e + o,  out[N-a] = o - e.
// D^T is centro-antisymmetric too, with blocks M^T and P^T.  2 H^2 FMAs instead of N1^2, and
// half as many distinct coefficients.
template <int N1, bool TRANS, typename T, typename C>
__device__ __forceinline__ void contract_eo(const C& src, const T* in, T* out)
{
    constexpr int H = N1 / 2, N = N1 - 1;
    T ue[H], uo[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
        ue[n] = in[n] + in[N - n];
        uo[n] = in[n] - in[N - n];
    }
#pragma unroll
    for (int a = 0; a < H; ++a) {
        const C c = src.row();
        T e = T(0), o = T(0);
#pragma unroll
        for (int n = 0; n < H; ++n) {
            e = fma(TRANS ? c.M(n * H + a) : c.P(a * H + n), ue[n], e);
            o = fma(TRANS ? c.P(n * H + a) : c.M(a * H + n), uo[n], o);
        }
        if constexpr (N1 % 2 == 1) e = fma(TRANS ? c.Rm(a) : c.Cm(a), in[H], e);
        out[a] = e + o;
        out[N - a] = o - e;
    }
    if constexpr (N1 % 2 == 1) {
        const C c = src.row();
        T m = T(0);
#pragma unroll
        for (int n = 0; n < H; ++n) m = fma(TRANS ? c.Cm(n) : c.Rm(n), uo[n], m);
        out[H] = m;
    }
}

// ---- FP32 contractions on the matrix cores ----
//
// v_mfma_f32_4x4x1f32 runs 16 independent 4x4 outer products per wave: block b = lane / 4 forms
// acc_b[i][j] += a(lane 4b + i) * b(lane 4b + j) and lane 4b + j receives acc_b[i][j] in its
// register i.  With b = a lane's own pencil value in[n] and a = C[4g + (lane % 4)][n] (a per-lane
// coefficient register), N1 such instructions leave out[4g + i] of the lane's OWN pencil in
// register i: the pencil contraction of the vector-unit code, in the same lane layout, with no
// re-layout and no vector-ALU work.  A centro-antisymmetric C (C[N-a][N-n] = -C[a][n], which D
// and D^T of GLL points are) gives the rows a >= N1/2 from the rows below through the reversed
// pencil: sum_m C[a][m] in[N-m] = -out[N-a], so one set of coefficient registers (rows
// 0..N1/2-1) serves all rows.  Even N1 only (an odd order's middle row would need its own set).
typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int N1>
struct MfmaCoef {
    static constexpr int H = N1 / 2;
    static constexpr int G = (H + 3) / 4;  // groups of four output rows
    float c[G][N1];                        // C[4g + lane % 4][n] (0 past row H-1)
};

// Coefficient registers of this lane for C = D (TRANS = false) or C = D^T, from the basis table.
template <int N1, bool TRANS, typename B>
__device__ __forceinline__ void mfma_coef_init(const B& bs, int lane, MfmaCoef<N1>& k)
{
    const int r = lane & 3;
#pragma unroll
    for (int g = 0; g < MfmaCoef<N1>::G; ++g)
#pragma unroll
        for (int n = 0; n < N1; ++n) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int a = 4 * g + q;
                v[q] = a < MfmaCoef<N1>::H ? float(TRANS ? bs.D[n * N1 + a] : bs.D[a * N1 + n]) : 0.0f;
            }
            k.c[g][n] = r == 0 ? v[0] : r == 1 ? v[1] : r == 2 ? v[2] : v[3];
        }
}

// out = C in for this lane's pencil (every lane of the wave must execute it: the matrix-core
// instruction works on whole waves).
template <int N1>
__device__ __forceinline__ void contract_mfma(const MfmaCoef<N1>& k, const float* in, float* out)
{
    static_assert(N1 % 2 == 0, "matrix-core contraction: even N1");
    constexpr int H = N1 / 2, N = N1 - 1;
#pragma unroll
    for (int g = 0; g < MfmaCoef<N1>::G; ++g) {
        mfma_f4 acc = {0.f, 0.f, 0.f, 0.f}, rev = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < N1; ++n) {
            acc = __builtin_amdgcn_mfma_f32_4x4x1f32(k.c[g][n], in[n], acc, 0, 0, 0);
            rev = __builtin_amdgcn_mfma_f32_4x4x1f32(k.c[g][n], in[N - n], rev, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = 4 * g + q;
            if (a < H) {
                out[a] = acc[q];
                out[N - a] = -rev[q];
            }
        }
    }
}

template <int N1, bool TRANS, bool EO, typename T, typename C>
__device__ __forceinline__ void contract(const C& src, const T* in, T* out)
{
    if constexpr (EO)
        contract_eo<N1, TRANS>(src, in, out);
    else
        contract_full<N1, TRANS>(src, in, out);
}

template <int N1, bool TRANS, bool EO, typename T>
__device__ __forceinline__ void contract(const Basis<T>& bs, const T* in, T* out)
{
    contract<N1, TRANS, EO>(CoefResident<T>{bs}, in, out);
}

}  // namespace ax
