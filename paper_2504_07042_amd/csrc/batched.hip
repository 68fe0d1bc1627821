// Batched AxLocal: many independent trilinear meshes of uneven size and order (each with nrhs
// columns).  The host groups the (mesh, element group) work items by order, largest meshes
// first; the launch runs one persistent kernel per order present, each specialised for its order
// (register allocation, and the work-group shape the tuning table selects for it when the work
// list is built) and walking its own item list, all
// enqueued on one stream (one graph node each when captured).  Per-order specialisation, rather
// than one kernel switching over the order per item, keeps each order's register footprint its
// own (measured on gfx950: 167 vs 137 GDOF/s in FP64 and 258 vs 207 in FP32 on the 64-mesh
// batch).  No atomics: the launches read everything from the caller's workspace, so they can be
// captured in a HIP graph and replayed.
//
// Per item the work is that of item.h with the basis tables read per output row (scalar loads
// from the workspace).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

#include "ax_local_impl.h"
#include "item.h"

namespace ax {

struct BHeader {
    int n_mesh, n_items, nrhs, prec;
    int64_t off_mesh, off_items, off_basis;
    int64_t bytes;
    int ready;
    int pad;
};

// Per-order persistent kernel over the items [0, n) of one order, in shape variant V.
template <int N1, typename T, int V, bool G>
__global__ void __launch_bounds__((BShape<N1, V>::BLOCK), (batch_waves(sizeof(T) == 4)))
order_item_kernel(const BItem* __restrict__ items, const BMesh* __restrict__ meshes, int64_t n, int nrhs,
                  const Basis<T>* __restrict__ bsp)
{
    __shared__ __attribute__((aligned(16))) char lds[BShape<N1, V>::template lds_bytes<T>()];
    lds_poison(lds, sizeof(lds));
    const CoefReload<T> cs{as_constant(bsp)};
    // the gathering form: runs of consecutive items (neighbouring elements, which read the same
    // cache lines of the global vector) on the work-groups of one XCD
    const int64_t it0 = (G && AX_GATHER_XCD) ? xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    for (int64_t it = it0; it < n; it += gridDim.x) {
        const BItem q = items[it];
        batched_item<N1, V, T, false, G>(meshes[q.mesh], q.eb, nrhs, cs, lds);
    }
}

// The work list walked by the tile kernel (shape variant kTileVariant): group g is item
// items[g], an element group of EPB elements of one mesh; every mesh of the list has the order
// of the launch and es = N1^3.  Each lookup re-reads the item's descriptor (scalar loads; the
// group index is laundered so that the compiler does not keep descriptors live across the
// item's phases: FP32 N1 = 8 then fits 127 VGPRs without scratch).
template <int EPB, int NP>
struct MeshListWalk {
    static constexpr bool kList = true;
    static constexpr bool kSlice = false;
    const BItem* __restrict__ items;
    const BMesh* __restrict__ meshes;
    int64_t n;
    __device__ __forceinline__ int64_t groups() const { return n; }
    __device__ __forceinline__ bool has(int64_t g, int slot) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        return (int64_t)it.eb * EPB + slot < meshes[it.mesh].E;
    }
    __device__ __forceinline__ int64_t left(int64_t g) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        return meshes[it.mesh].E - (int64_t)it.eb * EPB;
    }
    __device__ __forceinline__ const double* verts(int64_t g) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        return meshes[it.mesh].verts + (int64_t)it.eb * EPB * 24;
    }
    template <typename T>
    __device__ __forceinline__ const T* xsrc(int64_t g, int c) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        const BMesh& m = meshes[it.mesh];
        return static_cast<const T*>(m.X) + (int64_t)c * m.ld + (int64_t)it.eb * EPB * NP;
    }
    __device__ __forceinline__ const int32_t* map(int64_t g) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        return meshes[it.mesh].l2g + (int64_t)it.eb * EPB * NP;
    }
    template <typename T>
    __device__ __forceinline__ const T* xglob(int64_t g, int c) const
    {
        asm volatile("" : "+s"(g));
        const BMesh& m = meshes[items[g].mesh];
        return static_cast<const T*>(m.X) + (int64_t)c * m.ldg;
    }
    template <typename T>
    __device__ __forceinline__ T* ydst(int64_t g, int c) const
    {
        asm volatile("" : "+s"(g));
        const BItem it = items[g];
        const BMesh& m = meshes[it.mesh];
        return static_cast<T*>(m.Y) + (int64_t)c * m.ld + (int64_t)it.eb * EPB * NP;
    }
};

// Per-order persistent kernel over the items [0, n) of one order with the prefetching tile body
// of the single-mesh launches (one item ahead, across meshes), for the orders whose batched
// tuning entry asks for it (kernel = TILE).
template <int N1, typename T, bool G>
__global__ void __launch_bounds__((Tile<N1, Shape<N1>::EPB>::BLOCK), (min_waves<N1, GEO_TRI, T>()))
order_tile_kernel(const BItem* __restrict__ items, const BMesh* __restrict__ meshes, int64_t n, int nrhs,
                  const Basis<T>* __restrict__ bsp)
{
    constexpr int EPB = Shape<N1>::EPB, NP = N1 * N1 * N1;
    static_assert(batched_tile_available(N1, sizeof(T) == 4), "no batched tile kernel at this order");
    const MeshListWalk<EPB, NP> wl{items, meshes, n};
    const Basis<T>& bs = *bsp;
    ax_local_body<N1, GEO_TRI, true, G ? 1 : 0, EPB, T>(0, nrhs, nullptr, nullptr, nullptr, nullptr, bs, nullptr, 0,
                                                         NP, 0, nullptr, CoefConst<T>{as_constant(bsp)}, wl);
}

// One mesh's share of a slice launch: groups first, first + stride, ... of the mesh.
struct MeshSliceWalk {
    static constexpr bool kList = false;
    static constexpr bool kSlice = true;
    int64_t first, stride;
};

// The slice form: each work-group is given one mesh of the order (items[blockIdx.x] = (mesh, w),
// the mesh's work-groups numbered w = 0 .. wgs - 1) and walks that mesh's element groups exactly
// as the single-mesh tile kernel does, the mesh's descriptor read once.  Nothing of the work list
// stays live over an item, so the kernel has the single-mesh kernel's register footprint at every
// order (the list form spills at FP64 N1 >= 8).
template <int N1, typename T, bool G>
__global__ void __launch_bounds__((Tile<N1, Shape<N1>::EPB>::BLOCK), (min_waves<N1, GEO_TRI, T>()))
order_slice_kernel(const BItem* __restrict__ items, const BMesh* __restrict__ meshes, int nrhs,
                   const Basis<T>* __restrict__ bsp)
{
    constexpr int EPB = Shape<N1>::EPB, NP = N1 * N1 * N1;
    const BItem sl = items[blockIdx.x];
    const BMesh m = meshes[sl.mesh];
    const MeshSliceWalk wl{sl.eb, m.wgs};
    const Basis<T>& bs = *bsp;
    ax_local_body<N1, GEO_TRI, true, G ? 1 : 0, EPB, T>(m.E, nrhs, m.verts, nullptr, static_cast<const T*>(m.X),
                                                         static_cast<T*>(m.Y), bs, G ? m.l2g : nullptr, m.ldg, NP, m.ld,
                                                         nullptr, CoefConst<T>{as_constant(bsp)}, wl);
}

// Shape variants of the batched launches: 0 and 1 the per-item shapes of item_shape, 2 the tile
// kernel over the work list, 3 the tile kernel over mesh slices.
constexpr int kTileVariant = 2;
constexpr int kSliceVariant = 3;

// Resident work-groups per CU of the slice kernel of order N1 (once per instantiation).
template <int N1, typename T, bool G>
static int slice_per_cu()
{
    static int per = 0;
    if (per == 0) {
        int q = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, order_slice_kernel<N1, T, G>,
                                                         Tile<N1, Shape<N1>::EPB>::BLOCK, 0) != hipSuccess ||
            q < 1)
            q = 1;
        per = q;
    }
    return per;
}

template <typename T, bool G>
static int slice_per_cu_of(int N1)
{
    switch (N1) {
    case 2: return slice_per_cu<2, T, G>();
    case 3: return slice_per_cu<3, T, G>();
    case 4: return slice_per_cu<4, T, G>();
    case 5: return slice_per_cu<5, T, G>();
    case 6: return slice_per_cu<6, T, G>();
    case 7: return slice_per_cu<7, T, G>();
    case 8: return slice_per_cu<8, T, G>();
    case 9: return slice_per_cu<9, T, G>();
    default: return slice_per_cu<10, T, G>();
    }
}

// Work-groups of a slice launch of order N1: the tuned multiple of the resident capacity, at
// most one per element group; split over the meshes in proportion to their element groups (at
// least one each, at most one per group).  groups[q] in, wgs[q] out (n meshes; no allocation);
// returns the total.
static int64_t slice_split(int N1, int prec, bool gather, const int64_t* groups, int64_t* wgs, int n)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 256;
    (void)hipGetLastError();
    const int per = prec == AX_FP64 ? (gather ? slice_per_cu_of<double, true>(N1) : slice_per_cu_of<double, false>(N1))
                                    : (gather ? slice_per_cu_of<float, true>(N1) : slice_per_cu_of<float, false>(N1));
    const int gm = tune_get(N1, TUNE_BATCHED, prec).grid_mult;
    int64_t total = 0;
    for (int q = 0; q < n; ++q) total += groups[q];
    const int64_t cap = std::min<int64_t>(total, (int64_t)cus * per * (gm > 0 ? gm : 1));
    int64_t sum = 0;
    for (int q = 0; q < n; ++q) {
        const double share = total > 0 ? (double)cap * (double)groups[q] / (double)total : 0.0;
        wgs[q] = std::max<int64_t>(1, std::min<int64_t>(groups[q], (int64_t)std::llround(share)));
        sum += wgs[q];
    }
    return sum;
}

static int tile_items_epb(int N1)
{
    switch (N1) {
    case 2: return Shape<2>::EPB;
    case 3: return Shape<3>::EPB;
    case 4: return Shape<4>::EPB;
    case 5: return Shape<5>::EPB;
    case 6: return Shape<6>::EPB;
    case 7: return Shape<7>::EPB;
    case 8: return Shape<8>::EPB;
    case 9: return Shape<9>::EPB;
    default: return Shape<10>::EPB;
    }
}

// Elements per item of order N1 in shape variant V.
static int order_epb(int N1, int V)
{
    return (V == kTileVariant || V == kSliceVariant) ? tile_items_epb(N1) : item_shape(N1, V).epb;
}

// The shape variant the tuning table selects for the batched kernel of order N1.
static int order_variant(int N1, int prec)
{
    const TuneEntry t = tune_get(N1, TUNE_BATCHED, prec);
    if (t.kernel == AX_KERNEL_TILE && t.tile_alt) return kSliceVariant;
    if (t.kernel == AX_KERNEL_TILE && batched_tile_available(N1, prec == AX_FP32)) return kTileVariant;
    return item_has_alt(N1) ? t.item_alt : 0;
}

template <int N1, typename T, bool G>
static int order_tile_launch(const char* ws, const BHeader& h, int64_t first, int64_t count, hipStream_t st)
{
    const BItem* items = reinterpret_cast<const BItem*>(ws + h.off_items) + first;
    const BMesh* meshes = reinterpret_cast<const BMesh*>(ws + h.off_mesh);
    const Basis<T>* bsp = reinterpret_cast<const Basis<T>*>(ws + h.off_basis) + (N1 - 2);
    const TuneEntry tu = tune_get(N1, TUNE_BATCHED, sizeof(T) == 8 ? AX_FP64 : AX_FP32);
    constexpr int BLOCK = Tile<N1, Shape<N1>::EPB>::BLOCK;
    static int per = 0, cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, order_tile_kernel<N1, T, G>, BLOCK, 0) != hipSuccess ||
            q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t cap = (int64_t)cus * per * (tu.grid_mult > 0 ? tu.grid_mult : 1);
    const unsigned grid = (unsigned)std::min<int64_t>(count, cap);
    hipLaunchKernelGGL((order_tile_kernel<N1, T, G>), dim3(grid), dim3(BLOCK), 0, st, items, meshes, count, h.nrhs,
                       bsp);
    return hip_check(hipGetLastError(), "batched tile launch");
}

template <int N1, typename T, int V, bool G>
static int order_launch(const char* ws, const BHeader& h, int64_t first, int64_t count, hipStream_t st)
{
    const BItem* items = reinterpret_cast<const BItem*>(ws + h.off_items) + first;
    const BMesh* meshes = reinterpret_cast<const BMesh*>(ws + h.off_mesh);
    const Basis<T>* bsp = reinterpret_cast<const Basis<T>*>(ws + h.off_basis) + (N1 - 2);
    const TuneEntry tu = tune_get(N1, TUNE_BATCHED, sizeof(T) == 8 ? AX_FP64 : AX_FP32);
    static int per = 0, cus = 0;
    if (per == 0) {
        int dev = 0, c = 256, q = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, order_item_kernel<N1, T, V, G>, BShape<N1, V>::BLOCK, 0) !=
                hipSuccess ||
            q < 1)
            q = 1;
        cus = c;
        per = q;
    }
    const int64_t cap = (int64_t)cus * per * (tu.grid_mult > 0 ? tu.grid_mult : 1);
    const unsigned grid = (unsigned)std::min<int64_t>(count, cap);
    hipLaunchKernelGGL((order_item_kernel<N1, T, V, G>), dim3(grid), dim3(BShape<N1, V>::BLOCK), 0, st, items, meshes,
                       count, h.nrhs, bsp);
    return hip_check(hipGetLastError(), "batched launch");
}

template <int N1, typename T, bool G>
static int order_slice_launch(const char* ws, const BHeader& h, int64_t first, int64_t count, hipStream_t st)
{
    const BItem* items = reinterpret_cast<const BItem*>(ws + h.off_items) + first;
    const BMesh* meshes = reinterpret_cast<const BMesh*>(ws + h.off_mesh);
    const Basis<T>* bsp = reinterpret_cast<const Basis<T>*>(ws + h.off_basis) + (N1 - 2);
    if (count > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many work-groups for one launch");
    hipLaunchKernelGGL((order_slice_kernel<N1, T, G>), dim3((unsigned)count), dim3(Tile<N1, Shape<N1>::EPB>::BLOCK), 0,
                       st, items, meshes, h.nrhs, bsp);
    return hip_check(hipGetLastError(), "batched slice launch");
}

template <int N1, typename T>
static int order_launch_v(int V, bool G, const char* ws, const BHeader& h, int64_t first, int64_t count,
                          hipStream_t st)
{
    if (V == kSliceVariant)
        return G ? order_slice_launch<N1, T, true>(ws, h, first, count, st)
                 : order_slice_launch<N1, T, false>(ws, h, first, count, st);
    if (V == kTileVariant) {
        if constexpr (batched_tile_available(N1, sizeof(T) == 4))
            return G ? order_tile_launch<N1, T, true>(ws, h, first, count, st)
                     : order_tile_launch<N1, T, false>(ws, h, first, count, st);
        return fail(AX_ERR_ARG, "no batched tile kernel at N1 = %d in this precision", N1);
    }
    if (G)
        return V ? order_launch<N1, T, 1, true>(ws, h, first, count, st)
                 : order_launch<N1, T, 0, true>(ws, h, first, count, st);
    return V ? order_launch<N1, T, 1, false>(ws, h, first, count, st)
             : order_launch<N1, T, 0, false>(ws, h, first, count, st);
}

// V: the shape variant the work list of this order was built with; G: the gathering form.
template <typename T>
static int order_dispatch(int N1, int V, bool G, const char* ws, const BHeader& h, int64_t first, int64_t count,
                          hipStream_t st)
{
    switch (N1) {
    case 2: return order_launch_v<2, T>(V, G, ws, h, first, count, st);
    case 3: return order_launch_v<3, T>(V, G, ws, h, first, count, st);
    case 4: return order_launch_v<4, T>(V, G, ws, h, first, count, st);
    case 5: return order_launch_v<5, T>(V, G, ws, h, first, count, st);
    case 6: return order_launch_v<6, T>(V, G, ws, h, first, count, st);
    case 7: return order_launch_v<7, T>(V, G, ws, h, first, count, st);
    case 8: return order_launch_v<8, T>(V, G, ws, h, first, count, st);
    case 9: return order_launch_v<9, T>(V, G, ws, h, first, count, st);
    default: return order_launch_v<10, T>(V, G, ws, h, first, count, st);
    }
}

// Work items of a batch: with the variants of `prec` (prec < 0: an upper bound over every
// variant, for sizing a workspace before the precision is known).
static int64_t n_items_of(int n_mesh, const ax_problem* meshes, int prec)
{
    int64_t n = 0;
    for (int q = 0; q < n_mesh; ++q) {
        const int N1 = meshes[q].N + 1;
        const int e = prec < 0 ? std::min({order_epb(N1, 0), order_epb(N1, 1), order_epb(N1, kTileVariant)})
                               : order_epb(N1, order_variant(N1, prec));
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
    int var[kBMaxN1 + 1] = {};
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) var[N1] = order_variant(N1, prec);
    const int64_t n_items = n_items_of(n_mesh, meshes, prec);
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
        const int e = order_epb(N1, var[N1]);
        // slice form: each mesh's work-group count (stack arrays: this path allocates nothing)
        int64_t sgroups[kScratchMaxMeshes], swgs[kScratchMaxMeshes];
        const bool slices = var[N1] == kSliceVariant && cnt > 0;
        if (slices) {
            for (int c = 0; c < cnt; ++c) sgroups[c] = (meshes[idx[c]].E + e - 1) / e;
            slice_split(N1, prec, false, sgroups, swgs, cnt);
        }
        for (int c0 = 0; c0 < cnt; c0 += kFillChunk) {
            MeshFill f{};
            int64_t gmax = 1;
            f.count = std::min(kFillChunk, cnt - c0);
            for (int c = 0; c < f.count; ++c) {
                const ax_problem& p = meshes[idx[c0 + c]];
                const int64_t np = (int64_t)N1 * N1 * N1;
                f.id[c] = idx[c0 + c];
                f.m[c] = BMesh{p.E, col_stride ? col_stride[f.id[c]] : p.E * np, p.geo, X[f.id[c]], Y[f.id[c]], N1,
                               slices ? (int)swgs[c0 + c] : 0, np};
                // items: the mesh's element groups, or its work-groups in the slice form
                f.groups[c] = slices ? swgs[c0 + c] : (p.E + e - 1) / e;
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
            AX_TRY(order_dispatch<double>(N1, var[N1], false, base, h, plan.order_first[N1], plan.order_count[N1],
                                          st));
        else
            AX_TRY(order_dispatch<float>(N1, var[N1], false, base, h, plan.order_first[N1], plan.order_count[N1],
                                         st));
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
    layout(n_mesh, n_items_of(n_mesh, meshes, -1), h);
    *bytes = (size_t)h.bytes;
    return AX_OK;
}

// Workspace offsets of a prepared plan (a pure function of it, as batched_prepare laid them out).
static BHeader plan_header(const ax_batch_plan* plan)
{
    BHeader h{};
    auto up = [](int64_t v) { return (v + 255) & ~int64_t(255); };
    h.off_mesh = up(sizeof(BHeader));
    h.off_items = up(h.off_mesh + (int64_t)plan->n_mesh * sizeof(BMesh));
    h.off_basis = up(h.off_items + plan->n_items * (int64_t)sizeof(BItem));
    h.nrhs = plan->nrhs;
    return h;
}

__global__ void __launch_bounds__(256) set_source_kernel(BMesh* __restrict__ meshes, int n_mesh, const void* xg)
{
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q < n_mesh) meshes[q].X = xg;
}

// l2g == nullptr: X[q] local vectors as Y.  Otherwise the gathering form: mesh q reads a global
// vector (its address set by batched_set_source, X unused) through l2g + lbase[q], columns ldg
// values apart.
static int batched_prepare(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const void* const* X,
                           void* const* Y, const int64_t* col_stride, const int32_t* l2g, const int64_t* lbase,
                           int64_t ldg, void* workspace, size_t workspace_bytes, ax_batch_plan* plan)
{
    if (!plan) return fail(AX_ERR_ARG, "plan is NULL");
    std::memset(plan, 0, sizeof(*plan));
    AX_TRY(check_meshes(n_mesh, meshes));
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs < 1");
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "batched precision must be FP64 or FP32");
    if (!workspace) return fail(AX_ERR_ARG, "workspace is NULL");
    if (!l2g) AX_TRY(check_io(n_mesh, meshes, X, Y, col_stride));
    for (int N1 = 2; N1 <= kBMaxN1; ++N1) plan->order_variant[N1] = order_variant(N1, prec);
    const int64_t n_items = n_items_of(n_mesh, meshes, prec);
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
        bm[q] = BMesh{meshes[q].E, ld, meshes[q].geo, l2g ? nullptr : X[q], Y[q], meshes[q].N + 1, 0, np,
                      l2g ? l2g + lbase[q] : nullptr, ldg};
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
        const int e = order_epb(N1, plan->order_variant[N1]);
        if (plan->order_variant[N1] == kSliceVariant && !order.empty()) {
            // slices: work-group w of mesh q is item (q, w); the mesh records its work-group count
            std::vector<int64_t> groups, wgs(order.size());
            for (auto& o : order) groups.push_back((meshes[o.second].E + e - 1) / e);
            slice_split(N1, prec, l2g != nullptr, groups.data(), wgs.data(), (int)order.size());
            for (size_t k = 0; k < order.size(); ++k) {
                bm[order[k].second].wgs = (int)wgs[k];
                for (int64_t w = 0; w < wgs[k]; ++w) items.push_back(BItem{order[k].second, (int)w});
            }
        } else {
            for (auto& o : order) {
                const int64_t groups = (meshes[o.second].E + e - 1) / e;
                for (int64_t g = 0; g < groups; ++g) items.push_back(BItem{o.second, (int)g});
            }
        }
        plan->order_count[N1] = (int64_t)items.size() - plan->order_first[N1];
    }
    std::memcpy(host.data(), &h, sizeof(h));
    if (n_mesh) std::memcpy(host.data() + h.off_mesh, bm.data(), sizeof(BMesh) * n_mesh);
    // (slice orders use fewer items than the element groups the layout was sized for)
    if (!items.empty()) std::memcpy(host.data() + h.off_items, items.data(), sizeof(BItem) * items.size());
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
    plan->gather = l2g ? 1 : 0;
    plan->n_mesh = n_mesh;
    plan->nrhs = nrhs;
    plan->prec = prec;
    plan->bytes = (size_t)h.bytes;
    return AX_OK;
}

namespace ax {

// Internal (the batched CG): a plan in the gathering form, every mesh reading the global vector
// set by batched_set_source through l2g + lbase[q] (columns n_global apart) and writing its local
// result to Y[q] (columns ldy[q] apart).
int batched_prepare_gather(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const int32_t* l2g,
                           const int64_t* lbase, int64_t n_global, void* const* Y, const int64_t* ldy, void* ws,
                           size_t bytes, ax_batch_plan* plan)
{
    if (!l2g || !lbase || !Y || !ldy) return fail(AX_ERR_ARG, "internal: NULL gather arguments");
    return batched_prepare(n_mesh, meshes, nrhs, prec, nullptr, Y, ldy, l2g, lbase, n_global, ws, bytes, plan);
}

// Point every mesh of a gathering plan at the global vector xg (one small kernel: capturable).
int batched_set_source(const ax_batch_plan* plan, void* ws, const void* xg, hipStream_t st)
{
    if (plan->n_mesh == 0) return AX_OK;
    const BHeader h = plan_header(plan);
    BMesh* m = reinterpret_cast<BMesh*>(static_cast<char*>(ws) + h.off_mesh);
    hipLaunchKernelGGL(set_source_kernel, dim3((unsigned)((plan->n_mesh + 255) / 256)), dim3(256), 0, st, m,
                       plan->n_mesh, xg);
    return hip_check(hipGetLastError(), "batched source");
}

}  // namespace ax

extern "C" int ax_batched_prepare(int n_mesh, const ax_problem* meshes, int nrhs, int prec,
                                  const void* const* X, void* const* Y, const int64_t* col_stride,
                                  void* workspace, size_t workspace_bytes, ax_batch_plan* plan)
{
    clear_error();
    return batched_prepare(n_mesh, meshes, nrhs, prec, X, Y, col_stride, nullptr, nullptr, 0, workspace,
                           workspace_bytes, plan);
}

extern "C" int ax_local_batched(const ax_batch_plan* plan, const void* workspace, void* stream)
{
    clear_error();
    if (!plan || !workspace) return fail(AX_ERR_ARG, "plan or workspace is NULL");
    if (plan->prec != AX_FP64 && plan->prec != AX_FP32) return fail(AX_ERR_ARG, "plan was not filled by ax_batched_prepare");
    for (int N1 = 2; N1 <= kBMaxN1; ++N1)
        if (plan->order_variant[N1] < 0 || plan->order_variant[N1] > kSliceVariant)
            return fail(AX_ERR_ARG, "plan was not filled by ax_batched_prepare (shape variant %d)", plan->order_variant[N1]);
    if (plan->gather != 0 && plan->gather != 1) return fail(AX_ERR_ARG, "plan was not filled by ax_batched_prepare");
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
            AX_TRY(order_dispatch<double>(N1, plan->order_variant[N1], plan->gather != 0, (const char*)workspace,
                                          h, plan->order_first[N1], plan->order_count[N1], st));
        else
            AX_TRY(order_dispatch<float>(N1, plan->order_variant[N1], plan->gather != 0, (const char*)workspace,
                                         h, plan->order_first[N1], plan->order_count[N1], st));
    }
    return AX_OK;
}
