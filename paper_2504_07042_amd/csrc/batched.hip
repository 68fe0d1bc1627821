// Batched AxLocal: many independent trilinear meshes of uneven size and order (each with nrhs
// columns).  The host groups the (mesh, element group) work items by order, largest meshes
// first; the launch runs one persistent 256-thread kernel per order present, each specialised for
// its order (register allocation and elements per work-group) and walking its own item list, all
// enqueued on one stream (one graph node each when captured).  Per-order specialisation, rather
// than one kernel switching over the order per item, keeps each order's register footprint its
// own (measured on gfx950: 167 vs 137 GDOF/s in FP64 and 258 vs 207 in FP32 on the 64-mesh
// batch).  No atomics: the launches read everything from the caller's workspace, so they can be
// captured in a HIP graph and replayed.
//
// Per item the work is the trilinear on-the-fly operator of ax_local (geometric factors of
// Sec. 3.3 / Algorithm 2, contractions of Algorithm 1) with the basis tables read per output row
// (scalar loads from the workspace).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "ax_internal.h"
#include "ax_kernels.h"
#include "geom.h"

namespace ax {

constexpr int kBBlock = 256;
constexpr int kBMaxN1 = 10;

// One mesh of a batch (device descriptor) and one work item (element group eb of mesh `mesh`).
struct BMesh {
    int64_t E;
    int64_t ld;  // stride between columns of X and Y (values)
    const double* verts;
    const void* X;
    void* Y;
    int N1;
    int pad;
    int64_t es;  // stride between elements of X and Y (values): N1^3, or ncol N1^3 interleaved
};

struct BItem {
    int mesh;
    int eb;  // element group within the mesh
};

template <int N1>
struct BShape {
    static constexpr int NT = N1 * N1;
    static constexpr int EPB = kBBlock / NT > 64 ? 64 : kBBlock / NT;
    static constexpr int NP = Shape<N1>::NP;
    template <typename T>
    static constexpr int FS = Shape<N1, sizeof(T)>::FS;
    template <typename T>
    static constexpr size_t lds_bytes() { return (size_t)EPB * 2 * FS<T> * sizeof(T) + (size_t)EPB * 24 * 8; }
};

template <typename T>
constexpr size_t bmax_lds()
{
    size_t m = 0;
    m = std::max(m, BShape<2>::lds_bytes<T>());
    m = std::max(m, BShape<3>::lds_bytes<T>());
    m = std::max(m, BShape<4>::lds_bytes<T>());
    m = std::max(m, BShape<5>::lds_bytes<T>());
    m = std::max(m, BShape<6>::lds_bytes<T>());
    m = std::max(m, BShape<7>::lds_bytes<T>());
    m = std::max(m, BShape<8>::lds_bytes<T>());
    m = std::max(m, BShape<9>::lds_bytes<T>());
    m = std::max(m, BShape<10>::lds_bytes<T>());
    return m;
}


struct BHeader {
    int n_mesh, n_items, nrhs, prec;
    int64_t off_mesh, off_items, off_basis;
    int64_t bytes;
    int ready;
    int pad;
};

// cs: source of the basis tables (CoefResident or CoefReload)
// PL: partial recomputation (Sec. 4.2.2), the per-node scale read from lam [E][N1^3].
template <int N1, typename T, bool PL = false, typename C>
__device__ __forceinline__ void batched_item(const BMesh& m, int64_t eb, int nrhs, const C& cs, char* lds,
                                             const T* __restrict__ lamp = nullptr)
{
    using S = BShape<N1>;
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

    for (int q = tid; q < EPB * 24; q += kBBlock) {
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
#pragma unroll
        for (int k = 0; k < N1; ++k) xr[k] = active ? X[base + i + j * N1 + k * NT] : T(0);
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

// Per-order persistent kernel over the items [0, n) of one order.
// Waves per SIMD the register allocation targets (FP32 per-order kernels fit five)
#ifndef AX_BATCH_MINW_F32
#define AX_BATCH_MINW_F32 5
#endif
template <int N1, typename T>
__global__ void __launch_bounds__(kBBlock, (sizeof(T) == 4 ? AX_BATCH_MINW_F32 : 2))
order_item_kernel(const BItem* __restrict__ items, const BMesh* __restrict__ meshes, int64_t n, int nrhs,
                  const Basis<T>* __restrict__ bsp)
{
    __shared__ __attribute__((aligned(16))) char lds[BShape<N1>::template lds_bytes<T>()];
    lds_poison(lds, sizeof(lds));
    const CoefReload<T> cs{as_constant(bsp)};
    for (int64_t it = blockIdx.x; it < n; it += gridDim.x) {
        const BItem q = items[it];
        batched_item<N1, T>(meshes[q.mesh], q.eb, nrhs, cs, lds);
    }
}

// Elements per item of order N1.
static int order_epb(int N1)
{
    switch (N1) {
    case 2: return BShape<2>::EPB;
    case 3: return BShape<3>::EPB;
    case 4: return BShape<4>::EPB;
    case 5: return BShape<5>::EPB;
    case 6: return BShape<6>::EPB;
    case 7: return BShape<7>::EPB;
    case 8: return BShape<8>::EPB;
    case 9: return BShape<9>::EPB;
    default: return BShape<10>::EPB;
    }
}

template <int N1, typename T>
static int order_launch(const char* ws, const BHeader& h, int64_t first, int64_t count, hipStream_t st)
{
    const BItem* items = reinterpret_cast<const BItem*>(ws + h.off_items) + first;
    const BMesh* meshes = reinterpret_cast<const BMesh*>(ws + h.off_mesh);
    const Basis<T>* bsp = reinterpret_cast<const Basis<T>*>(ws + h.off_basis) + (N1 - 2);
    const TuneEntry tu = tune_get(N1, GEO_TRI, sizeof(T) == 8 ? AX_FP64 : AX_FP32);
    static int per = 0, cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, order_item_kernel<N1, T>, kBBlock, 0) != hipSuccess || q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t cap = (int64_t)cus * per * (tu.grid_mult > 0 ? tu.grid_mult : 1);
    const unsigned grid = (unsigned)std::min<int64_t>(count, cap);
    hipLaunchKernelGGL((order_item_kernel<N1, T>), dim3(grid), dim3(kBBlock), 0, st, items, meshes, count, h.nrhs, bsp);
    return hip_check(hipGetLastError(), "batched launch");
}

template <typename T>
static int order_dispatch(int N1, const char* ws, const BHeader& h, int64_t first, int64_t count, hipStream_t st)
{
    switch (N1) {
    case 2: return order_launch<2, T>(ws, h, first, count, st);
    case 3: return order_launch<3, T>(ws, h, first, count, st);
    case 4: return order_launch<4, T>(ws, h, first, count, st);
    case 5: return order_launch<5, T>(ws, h, first, count, st);
    case 6: return order_launch<6, T>(ws, h, first, count, st);
    case 7: return order_launch<7, T>(ws, h, first, count, st);
    case 8: return order_launch<8, T>(ws, h, first, count, st);
    case 9: return order_launch<9, T>(ws, h, first, count, st);
    default: return order_launch<10, T>(ws, h, first, count, st);
    }
}

// The per-item path above as a single-mesh persistent kernel (no work list): work-group g takes
// element groups g, g + grid, ...  Used by ax_local (and its partial-recomputation form) for the
// trilinear FP64 orders whose register footprint the prefetching kernel exceeds (N1 = 9..15:
// 118-162 VGPRs here against 256 plus spills there; measured 1.4-3.2x faster) or fills only at
// two waves per SIMD (N1 = 6, 7), with the tables reloaded per output row.
template <typename T>
struct ItemArgs {
    BMesh m;
    int nrhs;
    Basis<T> bs;
    const T* lam;  // per-node scale of the partial recomputation (PL), else unused
};

// Waves per SIMD the register allocation of the single-mesh kernel targets: the FP32 full form
// fits five (88-96 VGPRs; measured 3-8% faster than four at N1 = 10, 11, 12, 14, 15, 2% slower
// at 13); the FP32 partial form spills at five and keeps the default budget (measured 12% faster
// at N1 = 14, even at 13 and 15).
template <int N1, typename T, bool PL>
constexpr int item_minw() { return sizeof(T) == 4 && !PL && N1 != 13 ? 5 : 2; }

template <int N1, typename T, bool PL>
__global__ void __launch_bounds__(kBBlock, (item_minw<N1, T, PL>()))
tri_item_kernel(const ItemArgs<T> a)
{
    __shared__ __attribute__((aligned(16))) char lds[BShape<N1>::template lds_bytes<T>()];
    lds_poison(lds, sizeof(lds));
    const int64_t ng = (a.m.E + BShape<N1>::EPB - 1) / BShape<N1>::EPB;
    const CoefReload<T> cs = karg_coefs<T, ItemArgs<T>>();
    for (int64_t eb = blockIdx.x; eb < ng; eb += gridDim.x)
        batched_item<N1, T, PL>(a.m, eb, a.nrhs, cs, lds, a.lam);
}

template <int N1, typename T, bool PL>
static int tri_item_launch(int64_t E, int nrhs, const double* verts, const T* X, T* Y, const Basis<T>& bs,
                           const T* lam, int grid_mult, hipStream_t st, int64_t es, int64_t ccs)
{
    static int per = 0, cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, tri_item_kernel<N1, T, PL>, kBBlock, 0) != hipSuccess ||
            q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t ng = (E + BShape<N1>::EPB - 1) / BShape<N1>::EPB;
    const int64_t cap = (int64_t)cus * per * (grid_mult > 0 ? grid_mult : 1);
    const int64_t blocks = ng < cap ? ng : cap;
    if (blocks <= 0) return AX_OK;
    const ItemArgs<T> a{BMesh{E, ccs, verts, X, Y, N1, 0, es}, nrhs, bs, lam};
    hipLaunchKernelGGL((tri_item_kernel<N1, T, PL>), dim3((unsigned)blocks), dim3(kBBlock), 0, st, a);
    return hip_check(hipGetLastError(), "ax_local (item kernel) launch");
}

// lam != nullptr: the partial-recomputation form (orders 9..15).
int tri_item_dispatch_f64(int N1, int64_t E, int nrhs, const double* verts, const double* X, double* Y,
                          const Basis<double>& bs, int grid_mult, hipStream_t st, const double* lam, int64_t es,
                          int64_t ccs)
{
    if (lam) {
        switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_launch<n, double, true>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs);
            AX_ITEM_CASE(9) AX_ITEM_CASE(10) AX_ITEM_CASE(11) AX_ITEM_CASE(12) AX_ITEM_CASE(13) AX_ITEM_CASE(14)
            AX_ITEM_CASE(15)
#undef AX_ITEM_CASE
        default: return fail(AX_ERR_UNSUPPORTED, "partial item kernel for N1=%d", N1);
        }
    }
    switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_launch<n, double, false>(E, nrhs, verts, X, Y, bs, nullptr, grid_mult, st, es, ccs);
        AX_ITEM_CASE(2) AX_ITEM_CASE(3) AX_ITEM_CASE(4) AX_ITEM_CASE(5) AX_ITEM_CASE(6) AX_ITEM_CASE(7)
        AX_ITEM_CASE(8) AX_ITEM_CASE(9) AX_ITEM_CASE(10) AX_ITEM_CASE(11) AX_ITEM_CASE(12) AX_ITEM_CASE(13)
        AX_ITEM_CASE(14) AX_ITEM_CASE(15) AX_ITEM_CASE(16)
#undef AX_ITEM_CASE
    default: return fail(AX_ERR_UNSUPPORTED, "item kernel for N1=%d", N1);
    }
}

// FP32 orders served by the per-item kernel (see use_item_kernel in ax_local_impl.h);
// lam != nullptr: the partial-recomputation form.
int tri_item_dispatch_f32(int N1, int64_t E, int nrhs, const double* verts, const float* X, float* Y,
                          const Basis<float>& bs, int grid_mult, hipStream_t st, const float* lam, int64_t es,
                          int64_t ccs)
{
    if (lam) {
        switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_launch<n, float, true>(E, nrhs, verts, X, Y, bs, lam, grid_mult, st, es, ccs);
            AX_ITEM_CASE(13) AX_ITEM_CASE(14) AX_ITEM_CASE(15)
#undef AX_ITEM_CASE
        default: return fail(AX_ERR_UNSUPPORTED, "FP32 partial item kernel for N1=%d", N1);
        }
    }
    switch (N1) {
#define AX_ITEM_CASE(n) \
    case n: return tri_item_launch<n, float, false>(E, nrhs, verts, X, Y, bs, nullptr, grid_mult, st, es, ccs);
        AX_ITEM_CASE(9) AX_ITEM_CASE(10) AX_ITEM_CASE(11) AX_ITEM_CASE(12) AX_ITEM_CASE(13) AX_ITEM_CASE(14)
        AX_ITEM_CASE(15)
#undef AX_ITEM_CASE
    default: return fail(AX_ERR_UNSUPPORTED, "FP32 item kernel for N1=%d", N1);
    }
}

static int64_t n_items_of(int n_mesh, const ax_problem* meshes)
{
    int64_t n = 0;
    for (int q = 0; q < n_mesh; ++q) {
        const int e = order_epb(meshes[q].N + 1);
        n += (meshes[q].E + e - 1) / e;
    }
    return n;
}

static void layout(int n_mesh, int64_t n_items, BHeader& h)
{
    auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    h.off_mesh = up(sizeof(BHeader));
    h.off_items = up(h.off_mesh + (int64_t)n_mesh * sizeof(BMesh));
    h.off_basis = up(h.off_items + n_items * (int64_t)sizeof(BItem));
    h.bytes = h.off_basis + 9 * (int64_t)std::max(sizeof(Basis<double>), sizeof(Basis<float>));
}

static int check_meshes(int n_mesh, const ax_problem* meshes)
{
    if (n_mesh < 0) return fail(AX_ERR_ARG, "n_mesh < 0");
    if (n_mesh > 0 && !meshes) return fail(AX_ERR_ARG, "meshes is NULL");
    for (int q = 0; q < n_mesh; ++q) {
        const ax_problem& p = meshes[q];
        if (p.E < 0) return fail(AX_ERR_ARG, "mesh %d: E < 0", q);
        if (p.N < 1 || p.N > 9) return fail(AX_ERR_UNSUPPORTED, "mesh %d: batched orders are 1..9 (N=%d)", q, p.N);
        if (p.geom != AX_TRILINEAR) return fail(AX_ERR_UNSUPPORTED, "mesh %d: batched path is trilinear", q);
        if (p.E > 0 && (!p.geo || !p.D || !p.xi || !p.w)) return fail(AX_ERR_ARG, "mesh %d: NULL array", q);
        if (p.E > 0 && !centro_antisymmetric(p.N + 1, p.D))
            return fail(AX_ERR_UNSUPPORTED, "mesh %d: D must be a GLL differentiation matrix", q);
        if (p.E > 0x7fffffffLL) return fail(AX_ERR_UNSUPPORTED, "mesh %d too large", q);
    }
    return AX_OK;
}

// Per-mesh input/output pointers and column strides of a batch.
static int check_io(int n_mesh, const ax_problem* meshes, const void* const* X, void* const* Y,
                    const int64_t* col_stride)
{
    if (n_mesh > 0 && (!X || !Y)) return fail(AX_ERR_ARG, "X or Y is NULL");
    for (int q = 0; q < n_mesh; ++q) {
        if (meshes[q].E > 0 && (!X[q] || !Y[q])) return fail(AX_ERR_ARG, "mesh %d: X or Y is NULL", q);
        if (meshes[q].E > 0 && X[q] == Y[q]) return fail(AX_ERR_ARG, "mesh %d: X and Y alias", q);
        const int64_t np = (int64_t)(meshes[q].N + 1) * (meshes[q].N + 1) * (meshes[q].N + 1);
        if (col_stride && col_stride[q] < meshes[q].E * np)
            return fail(AX_ERR_ARG, "mesh %d: column stride below E*N1^3", q);
    }
    return AX_OK;
}

// ---- The batched launch without allocation (ax_local_batched_noalloc) ----
//
// The work list, the mesh descriptors and the basis tables live in one file-scope device array
// instead of a caller's workspace.  Host code never uses the array's name as an address: its
// device address comes from hipGetSymbolAddress, once per device, on the first call on that
// device.  The array is written only by the fill kernels below, from data passed as kernel
// arguments, so a call makes no allocation of any kind (no hipMalloc, no host heap, no staging
// copy) and enqueues only kernels.  All calls on one device share the array.
constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr int kScratchMaxMeshes = 4096;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices];

// Device address of this device's `scratch` (resolved once per device).
static int scratch_address(char** out)
{
    int dev = 0;
    AX_TRY(hip_check(hipGetDevice(&dev), "hipGetDevice"));
    if (dev < 0 || dev >= kMaxDevices) return fail(AX_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        AX_TRY(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)"));
        if (!p) return fail(AX_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = g_scratch_ptr[dev];
    return AX_OK;
}

// Up to kFillChunk meshes of one launch: their descriptors and the ranges of work items they own
// (passed by value, about 2.3 KB of kernel arguments).
constexpr int kFillChunk = 32;
struct MeshFill {
    BMesh m[kFillChunk];
    int64_t item_base[kFillChunk];
    int64_t groups[kFillChunk];
    int id[kFillChunk];
    int count;
};

// blockIdx.y = mesh of the chunk: its descriptor, and items (id, g) for its element groups g.
__global__ void __launch_bounds__(256)
fill_meshes_kernel(const MeshFill f, BMesh* __restrict__ meshes, BItem* __restrict__ items)
{
    const int c = blockIdx.y;
    if (c >= f.count) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) meshes[f.id[c]] = f.m[c];
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < f.groups[c]; g += (int64_t)gridDim.x * 256)
        items[f.item_base[c] + g] = BItem{f.id[c], (int)g};
}

// dst = the basis tables passed by value (the kernel's first argument), copied word by word from
// the kernel-argument segment.
template <typename T>
__global__ void __launch_bounds__(256) fill_basis_kernel(const Basis<T> b, Basis<T>* __restrict__ dst)
{
    (void)b;
    constexpr int nw = (int)(sizeof(Basis<T>) / sizeof(uint64_t));
    static_assert(sizeof(Basis<T>) % sizeof(uint64_t) == 0, "basis tables are whole 8-byte words");
    const __attribute__((address_space(4))) uint64_t* src =
        (const __attribute__((address_space(4))) uint64_t*)__builtin_amdgcn_kernarg_segment_ptr();
    uint64_t* d = reinterpret_cast<uint64_t*>(dst);
    for (int q = threadIdx.x; q < nw; q += 256) d[q] = src[q];
}

static int batched_noalloc(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const void* const* X,
                           void* const* Y, const int64_t* col_stride, hipStream_t st)
{
    AX_TRY(check_meshes(n_mesh, meshes));
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs < 1");
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "batched precision must be FP64 or FP32");
    if (n_mesh > kScratchMaxMeshes)
        return fail(AX_ERR_ARG, "%d meshes: the allocation-free batched launch takes at most %d", n_mesh,
                    kScratchMaxMeshes);
    AX_TRY(check_io(n_mesh, meshes, X, Y, col_stride));
    const int64_t n_items = n_items_of(n_mesh, meshes);
    BHeader h{};
    layout(n_mesh, n_items, h);
    if ((size_t)h.bytes > kScratchBytes)
        return fail(AX_ERR_ARG, "the batch needs %lld bytes of work list (%lld items); the allocation-free "
                    "batched launch holds at most %zu bytes", (long long)h.bytes, (long long)n_items, kScratchBytes);
    if (n_items == 0) return AX_OK;
    char* base = nullptr;
    AX_TRY(scratch_address(&base));
    BMesh* dmesh = reinterpret_cast<BMesh*>(base + h.off_mesh);
    BItem* ditem = reinterpret_cast<BItem*>(base + h.off_items);
    // work list: orders ascending, the meshes of an order largest first (ties by index), as
    // ax_batched_prepare orders it
    ax_batch_plan plan{};
    int idx[kScratchMaxMeshes];
    int64_t next = 0;
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) {
        int cnt = 0;
        for (int q = 0; q < n_mesh; ++q)
            if (meshes[q].N + 1 == N1 && meshes[q].E > 0) idx[cnt++] = q;
        std::sort(idx, idx + cnt, [&](int a, int b) {
            return meshes[a].E != meshes[b].E ? meshes[a].E > meshes[b].E : a < b;
        });
        plan.order_first[N1] = next;
        const int e = order_epb(N1);
        for (int c0 = 0; c0 < cnt; c0 += kFillChunk) {
            MeshFill f{};
            int64_t gmax = 1;
            f.count = std::min(kFillChunk, cnt - c0);
            for (int c = 0; c < f.count; ++c) {
                const ax_problem& p = meshes[idx[c0 + c]];
                const int64_t np = (int64_t)N1 * N1 * N1;
                f.id[c] = idx[c0 + c];
                f.m[c] = BMesh{p.E, col_stride ? col_stride[f.id[c]] : p.E * np, p.geo, X[f.id[c]], Y[f.id[c]], N1, 0,
                               np};
                f.groups[c] = (p.E + e - 1) / e;
                f.item_base[c] = next;
                next += f.groups[c];
                gmax = std::max(gmax, f.groups[c]);
            }
            const unsigned gx = (unsigned)std::min<int64_t>((gmax + 255) / 256, 64);
            hipLaunchKernelGGL(fill_meshes_kernel, dim3(gx, f.count), dim3(256), 0, st, f, dmesh, ditem);
            AX_TRY(hip_check(hipGetLastError(), "batched work-list fill"));
        }
        plan.order_count[N1] = next - plan.order_first[N1];
        if (cnt == 0) continue;
        // one basis per order, taken from the last mesh of that order (as ax_batched_prepare does)
        const ax_problem& p0 = meshes[*std::max_element(idx, idx + cnt)];
        if (prec == AX_FP64) {
            Basis<double> b;
            fill_basis(b, N1, p0.D, p0.xi, p0.w);
            hipLaunchKernelGGL(fill_basis_kernel<double>, dim3(1), dim3(256), 0, st, b,
                               reinterpret_cast<Basis<double>*>(base + h.off_basis) + (N1 - 2));
        } else {
            Basis<float> b;
            fill_basis(b, N1, p0.D, p0.xi, p0.w);
            hipLaunchKernelGGL(fill_basis_kernel<float>, dim3(1), dim3(256), 0, st, b,
                               reinterpret_cast<Basis<float>*>(base + h.off_basis) + (N1 - 2));
        }
        AX_TRY(hip_check(hipGetLastError(), "batched basis fill"));
    }
    h.nrhs = nrhs;
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) {
        if (plan.order_count[N1] == 0) continue;
        if (prec == AX_FP64)
            AX_TRY(order_dispatch<double>(N1, base, h, plan.order_first[N1], plan.order_count[N1], st));
        else
            AX_TRY(order_dispatch<float>(N1, base, h, plan.order_first[N1], plan.order_count[N1], st));
    }
    return AX_OK;
}

}  // namespace ax

using namespace ax;

extern "C" int ax_local_batched_noalloc(int n_mesh, const ax_problem* meshes, int nrhs, int prec,
                                        const void* const* X, void* const* Y, const int64_t* col_stride,
                                        void* stream)
{
    clear_error();
    return batched_noalloc(n_mesh, meshes, nrhs, prec, X, Y, col_stride, as_stream(stream));
}

extern "C" int ax_batched_workspace_bytes(int n_mesh, const ax_problem* meshes, size_t* bytes)
{
    clear_error();
    AX_TRY(check_meshes(n_mesh, meshes));
    if (!bytes) return fail(AX_ERR_ARG, "bytes is NULL");
    BHeader h{};
    layout(n_mesh, n_items_of(n_mesh, meshes), h);
    *bytes = (size_t)h.bytes;
    return AX_OK;
}

extern "C" int ax_batched_prepare(int n_mesh, const ax_problem* meshes, int nrhs, int prec,
                                  const void* const* X, void* const* Y, const int64_t* col_stride,
                                  void* workspace, size_t workspace_bytes, ax_batch_plan* plan)
{
    clear_error();
    if (!plan) return fail(AX_ERR_ARG, "plan is NULL");
    std::memset(plan, 0, sizeof(*plan));
    AX_TRY(check_meshes(n_mesh, meshes));
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs < 1");
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "batched precision must be FP64 or FP32");
    if (!workspace) return fail(AX_ERR_ARG, "workspace is NULL");
    AX_TRY(check_io(n_mesh, meshes, X, Y, col_stride));
    const int64_t n_items = n_items_of(n_mesh, meshes);
    BHeader h{};
    layout(n_mesh, n_items, h);
    if ((size_t)h.bytes > workspace_bytes) return fail(AX_ERR_NOMEM, "workspace of %lld bytes needed", (long long)h.bytes);
    h.n_mesh = n_mesh;
    h.n_items = (int)n_items;
    h.nrhs = nrhs;
    h.prec = prec;
    h.ready = 1;
    std::vector<char> host((size_t)h.bytes, 0);
    std::vector<BMesh> bm(n_mesh);
    for (int q = 0; q < n_mesh; ++q) {
        const int64_t np = (int64_t)(meshes[q].N + 1) * (meshes[q].N + 1) * (meshes[q].N + 1);
        const int64_t ld = col_stride ? col_stride[q] : meshes[q].E * np;
        if (ld < meshes[q].E * np) return fail(AX_ERR_ARG, "mesh %d: column stride below E*N1^3", q);
        bm[q] = BMesh{meshes[q].E, ld, meshes[q].geo, X[q], Y[q], meshes[q].N + 1, 0, np};
    }
    // items grouped by order (one persistent kernel each), meshes of an order largest first
    std::vector<BItem> items;
    items.reserve((size_t)n_items);
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) {
        std::vector<std::pair<int64_t, int>> order;
        for (int q = 0; q < n_mesh; ++q)
            if (meshes[q].N + 1 == N1 && meshes[q].E > 0) order.push_back({-meshes[q].E, q});
        std::stable_sort(order.begin(), order.end());
        plan->order_first[N1] = (int64_t)items.size();
        const int e = order_epb(N1);
        for (auto& o : order) {
            const int64_t groups = (meshes[o.second].E + e - 1) / e;
            for (int64_t g = 0; g < groups; ++g) items.push_back(BItem{o.second, (int)g});
        }
        plan->order_count[N1] = (int64_t)items.size() - plan->order_first[N1];
    }
    std::memcpy(host.data(), &h, sizeof(h));
    if (n_mesh) std::memcpy(host.data() + h.off_mesh, bm.data(), sizeof(BMesh) * n_mesh);
    if (n_items) std::memcpy(host.data() + h.off_items, items.data(), sizeof(BItem) * n_items);
    // GLL tables of every order used, indexed by N1 - 2
    for (int q = 0; q < n_mesh; ++q) {
        const int N1 = meshes[q].N + 1;
        if (prec == AX_FP64) {
            Basis<double> b;
            fill_basis(b, N1, meshes[q].D, meshes[q].xi, meshes[q].w);
            std::memcpy(host.data() + h.off_basis + (N1 - 2) * sizeof(Basis<double>), &b, sizeof(b));
        } else {
            Basis<float> b;
            fill_basis(b, N1, meshes[q].D, meshes[q].xi, meshes[q].w);
            std::memcpy(host.data() + h.off_basis + (N1 - 2) * sizeof(Basis<float>), &b, sizeof(b));
        }
    }
    AX_TRY(hip_check(hipMemcpy(workspace, host.data(), (size_t)h.bytes, hipMemcpyHostToDevice),
                     "batched workspace upload"));
    plan->n_items = n_items;
    plan->n_mesh = n_mesh;
    plan->nrhs = nrhs;
    plan->prec = prec;
    plan->bytes = (size_t)h.bytes;
    return AX_OK;
}

extern "C" int ax_local_batched(const ax_batch_plan* plan, const void* workspace, void* stream)
{
    clear_error();
    if (!plan || !workspace) return fail(AX_ERR_ARG, "plan or workspace is NULL");
    if (plan->prec != AX_FP64 && plan->prec != AX_FP32) return fail(AX_ERR_ARG, "plan was not filled by ax_batched_prepare");
    if (plan->n_items == 0) return AX_OK;
    BHeader h{};
    h.off_mesh = h.off_items = h.off_basis = 0;
    {
        // offsets are a pure function of the plan: recompute them as ax_batched_prepare did
        auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
        h.off_mesh = up(sizeof(BHeader));
        h.off_items = up(h.off_mesh + (int64_t)plan->n_mesh * sizeof(BMesh));
        h.off_basis = up(h.off_items + plan->n_items * (int64_t)sizeof(BItem));
        h.nrhs = plan->nrhs;
    }
    hipStream_t st = as_stream(stream);
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) {
        if (plan->order_count[N1] == 0) continue;
        if (plan->prec == AX_FP64)
            AX_TRY(order_dispatch<double>(N1, (const char*)workspace, h, plan->order_first[N1], plan->order_count[N1], st));
        else
            AX_TRY(order_dispatch<float>(N1, (const char*)workspace, h, plan->order_first[N1], plan->order_count[N1], st));
    }
    return AX_OK;
}
