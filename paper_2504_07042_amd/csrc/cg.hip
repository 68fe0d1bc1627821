// Conjugate gradients on the assembled operator A = mask o Q^T AxLocal(Q .) (Eq. 1), the
// iterative solve whose dominant kernel is AxLocal (Sec. 1), plus mixed-precision iterative
// refinement: FP64 outer residual, norm and update; inner CG with a reduced-precision AxLocal,
// float vectors and FP64-accumulated dot products.
//
// Every scalar of the iteration (alpha, beta, |r|^2) lives on the device; the host only polls
// the convergence flags every few iterations.  Dot products are two-stage reductions with a
// fixed grid and a fixed combination order, so a solve is bitwise reproducible.
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "ax_internal.h"
#include "gs_impl.h"

namespace ax {

int gs_apply(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
             const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, int dtype, const void* in,
             void* out, hipStream_t st);
int ax_local_gather(const ax_problem& p, int nrhs, int prec, const void* xg, int64_t ldg, void* Y, hipStream_t st);
int ax_local_gather_fused(const ax_problem& p, const float* xg, int64_t ldg, float* yl, FusedOut* fo,
                          hipStream_t st);
int batched_prepare_gather(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const int32_t* l2g,
                           const int64_t* lbase, int64_t n_global, void* const* Y, const int64_t* ldy, void* ws,
                           size_t bytes, ax_batch_plan* plan);
int batched_set_source(const ax_batch_plan* plan, void* ws, const void* xg, hipStream_t st);

// The single-column FP32 operator of cg_solve with p^T A p summed inside the gathering AxLocal
// (fused_operator); 0 = off.
#ifndef AX_CG_FUSED
#define AX_CG_FUSED 1
#endif

constexpr int kRedBlocks = 4096;  // partial sums per dot product and column (fixed grid)
constexpr int kRedThreads = 256;
constexpr int kPoll = 8;         // iterations between host convergence checks
constexpr int kReliableCheck = 256;  // longest run of reduced-precision iterations between FP64 checks

// Per-column scalar state of one CG (device).
struct CgScal {
    double rr;      // r . r (convergence test on the residual norm)
    double rz;      // r . z, z = M^-1 r (= r . r without a preconditioner)
    double alpha;
    double beta;
    double tol2;    // (rtol * |b|)^2 target on r . r
    int converged;  // 1 once r . r <= tol2
    int breakdown;  // 1 on p^T A p <= 0 or a non-finite scalar
    int iters;
    int pad;
};

// Partial sums of the fixed-grid reductions: [2][nrhs][kRedBlocks], the second half for r . z.
__device__ __forceinline__ double* rz_partials(double* partials, int nrhs) { return partials + (size_t)nrhs * kRedBlocks; }

template <typename TA, typename TB>
__global__ void __launch_bounds__(kRedThreads)
dot_partial_kernel(const TA* __restrict__ a, const TB* __restrict__ b, int64_t n,
                   double* __restrict__ partials)
{
    const int c = blockIdx.y;
    a += (int64_t)c * n;
    b += (int64_t)c * n;
    double s = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kRedThreads)
        s = fma((double)a[q], (double)b[q], s);
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[c * kRedBlocks + blockIdx.x] = red[0];
}

__device__ double block_sum_partials(const double* partials)
{
    __shared__ double red[kRedThreads];
    double s = 0.0;
    for (int q = threadIdx.x; q < kRedBlocks; q += kRedThreads) s += partials[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

// mode 0: rr = sum (initial), converged if rr <= tol2.   mode 1: alpha = rr / sum (= p.Ap).
// mode 2: rr_new = sum; beta = rr_new / rr; rr = rr_new; converged test.
// mode 3: rr = sum after a reliable update (alpha, beta and the iteration count are kept).
// mode 4: sum = d . d of the iterate about to be folded; flags a non-finite one (breakdown 2).
// With `pre` the partials hold r . r in the first and r . z in the second half (modes 0, 2, 3);
// without, r . z = r . r.
__global__ void __launch_bounds__(kRedThreads)
cg_scalar_kernel(const double* __restrict__ partials, CgScal* __restrict__ sc, int mode, int pre)
{
    const int c = blockIdx.x, nrhs = gridDim.x;
    const double s = block_sum_partials(partials + c * kRedBlocks);
    __syncthreads();
    const double s2 = (pre && mode != 1 && mode != 4)
                          ? block_sum_partials(partials + (size_t)nrhs * kRedBlocks + c * kRedBlocks)
                          : s;
    if (threadIdx.x != 0) return;
    CgScal& q = sc[c];
    if (mode == 0) {
        q.rr = s;
        q.rz = s2;
        q.converged = (s <= q.tol2) ? 1 : 0;
        q.breakdown = isfinite(s) && isfinite(s2) ? 0 : 1;
        q.iters = 0;
        q.alpha = q.beta = 0.0;
    } else if (mode == 1) {
        if (q.converged || q.breakdown) {
            q.alpha = 0.0;
        } else if (!(s > 0.0) || !isfinite(s)) {
            q.breakdown = 1;
            q.alpha = 0.0;
        } else {
            q.alpha = q.rz / s;
        }
    } else if (mode == 4) {
        // s = d . d of the reduced-precision iterate: a non-finite one must not reach x
        if (!isfinite(s)) q.breakdown = 2;
    } else if (mode == 3) {
        // the iterated residual was replaced by the true one: new r . r, keep the iteration count
        q.rr = s;
        q.rz = s2;
        q.converged = (s <= q.tol2) ? 1 : 0;
        q.breakdown = isfinite(s) && isfinite(s2) ? 0 : 1;
    } else {
        if (q.converged || q.breakdown) {
            q.beta = 0.0;
        } else {
            q.beta = s2 / q.rz;
            q.rz = s2;
            q.rr = s;
            q.iters += 1;
            if (!isfinite(s) || !isfinite(s2)) q.breakdown = 1;
            else if (s <= q.tol2) q.converged = 1;
        }
    }
}

// The solver's view of Q^T: per global node the first two local copies (ascending local id),
// built once per solve from the CSR inverse and the Dirichlet mask.  first < 0: the node is
// masked or has no copy (its sum is 0); second >= 0: the second copy; second == -1: a single
// copy; second == -2: more than two copies, the rest read through the CSR.  Most nodes of a hex
// mesh have one or two copies, so their gather is one 8-byte index load and one or two value
// loads, against three dependent loads (offsets, index, value) through the CSR.
struct alignas(8) CopyPair {
    int32_t first, second;
};

__global__ void __launch_bounds__(256)
copy_pairs_kernel(CopyPair* __restrict__ cp, const int64_t* __restrict__ gptr, const int32_t* __restrict__ gidx,
                  const uint8_t* __restrict__ mask, int64_t n_global)
{
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < n_global; g += (int64_t)gridDim.x * 256) {
        const int64_t q0 = gptr[g], n = gptr[g + 1] - q0;
        CopyPair c{-1, -1};
        if (n > 0 && !(mask && mask[g])) {
            c.first = gidx[q0];
            c.second = n == 1 ? -1 : n == 2 ? gidx[q0 + 1] : -2;
        }
        cp[g] = c;
    }
}

// Ap[g] = mask ? 0 : sum of the local copies (ascending local id, the order of the plain loop)
// and, fused, the partial sums of p . Ap over the same fixed grid as dot_partial_kernel.  Each
// thread takes kQtUnroll nodes per tile so that their loads are in flight together.
// FOLD (after the fused operator): p . Ap comes from AxLocal's per-work-group energies
// epart[0, nparts), folded onto this fixed grid (block b takes b, b + gridDim.x, ...), so p is
// not read.
#ifndef AX_QT_UNROLL
#define AX_QT_UNROLL 4
#endif
constexpr int kQtUnroll = AX_QT_UNROLL;
template <typename T, bool FOLD>
__global__ void __launch_bounds__(kRedThreads)
qt_dot_kernel(int64_t n_global, const CopyPair* __restrict__ cp, const int64_t* __restrict__ gptr,
              const int32_t* __restrict__ gidx, int64_t n_local, const T* __restrict__ in,
              const T* __restrict__ pdir, T* __restrict__ out, double* __restrict__ partials,
              const double* __restrict__ epart, int64_t nparts)
{
    const int c = blockIdx.y;
    const T* x = in + (int64_t)c * n_local;
    const T* pd = pdir + (int64_t)c * n_global;
    T* o = out + (int64_t)c * n_global;
    double acc = 0.0;
    // Tile order: plain (the XCD-aware order of the other gather kernels measured 0.5-1 % slower
    // per CG solve here, although it cuts the re-read traffic).
#ifndef AX_QT_XCD
#define AX_QT_XCD 0
#endif
    const int64_t tile0 = AX_QT_XCD ? xcd_tile(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    for (int64_t g0 = tile0 * kRedThreads * kQtUnroll + threadIdx.x; g0 < n_global;
         g0 += (int64_t)gridDim.x * kRedThreads * kQtUnroll) {
        CopyPair q[kQtUnroll];
#pragma unroll
        for (int u = 0; u < kQtUnroll; ++u) {
            const int64_t g = g0 + u * kRedThreads;
            q[u] = g < n_global ? cp[g] : CopyPair{-1, -1};
        }
        T v0[kQtUnroll], v1[kQtUnroll];
        int64_t b[kQtUnroll], e[kQtUnroll];
#pragma unroll
        for (int u = 0; u < kQtUnroll; ++u) {
            v0[u] = q[u].first >= 0 ? x[q[u].first] : T(0);
            v1[u] = q[u].second >= 0 ? x[q[u].second] : T(0);
            const bool many = q[u].second == -2;
            b[u] = many ? gptr[g0 + u * kRedThreads] + 1 : 0;
            e[u] = many ? gptr[g0 + u * kRedThreads + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < kQtUnroll; ++u) {
            const int64_t g = g0 + u * kRedThreads;
            if (g < n_global) {
                T s = T(0) + v0[u];
                if (q[u].second >= 0) {
                    s += v1[u];
                } else if (q[u].second == -2) {
                    // the further copies (at most 7 more on a hexahedral mesh) fetched with
                    // independent loads, summed in ascending local id
                    constexpr int kMore = 7;
                    int32_t id[kMore];
#pragma unroll
                    for (int m = 0; m < kMore; ++m) id[m] = b[u] + m < e[u] ? gidx[b[u] + m] : -1;
                    T v[kMore];
#pragma unroll
                    for (int m = 0; m < kMore; ++m) v[m] = id[m] >= 0 ? x[id[m]] : T(0);
#pragma unroll
                    for (int m = 0; m < kMore; ++m)
                        if (id[m] >= 0) s += v[m];
                    for (int64_t k = b[u] + kMore; k < e[u]; ++k) s += x[gidx[k]];
                }
                o[g] = s;
                if constexpr (!FOLD) acc = fma((double)pd[g], (double)s, acc);
            }
        }
    }
    if constexpr (FOLD) {
        if (threadIdx.x == 0) {
            for (int64_t q = blockIdx.x; q < nparts; q += gridDim.x) acc += epart[q];
            partials[c * kRedBlocks + blockIdx.x] = acc;
        }
        return;
    }
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[c * kRedBlocks + blockIdx.x] = red[0];
}

// Block sum of `acc` into partials[slot] (fixed combination order).
__device__ __forceinline__ void block_partial(double acc, double* __restrict__ dst)
{
    __shared__ double red[kRedThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kRedThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = red[0];
    __syncthreads();
}

// r -= alpha Ap and, with XUPD, x += alpha p; partial sums of r . r and, with the Jacobi
// preconditioner (dinv != NULL), of r . z with z = dinv o r (fixed grid).  Without XUPD the x
// update is left to cg_dir_kernel, which reads p anyway (see merged_x_update).
template <typename TX, typename T, bool XUPD>
__global__ void __launch_bounds__(kRedThreads)
update_dot_kernel(TX* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ Ap,
                  const CgScal* __restrict__ sc, int64_t n, const T* __restrict__ dinv, double* __restrict__ partials)
{
    const int c = blockIdx.y;
    const double al = sc[c].alpha;
    const int64_t o = (int64_t)c * n;
    double acc = 0.0, acz = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kRedThreads) {
        T rv = r[o + q];
        if (al != 0.0) {
            if constexpr (XUPD) x[o + q] = (TX)((double)x[o + q] + al * (double)p[o + q]);
            rv = (T)((double)rv - al * (double)Ap[o + q]);
            r[o + q] = rv;
        }
        acc = fma((double)rv, (double)rv, acc);
        if (dinv) acz = fma((double)rv * (double)dinv[q], (double)rv, acz);
    }
    block_partial(acc, partials + c * kRedBlocks + blockIdx.x);
    if (dinv) block_partial(acz, partials + ((size_t)gridDim.y + c) * kRedBlocks + blockIdx.x);
}

// Partial sums of r . r and (dinv != NULL) r . (dinv o r), for modes 0 and 3 of the scalar kernel.
template <typename T>
__global__ void __launch_bounds__(kRedThreads)
rr_rz_kernel(const T* __restrict__ r, const T* __restrict__ dinv, int64_t n, double* __restrict__ partials)
{
    const int c = blockIdx.y;
    const T* rc = r + (int64_t)c * n;
    double acc = 0.0, acz = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; q < n; q += (int64_t)gridDim.x * kRedThreads) {
        const double v = (double)rc[q];
        acc = fma(v, v, acc);
        if (dinv) acz = fma(v * (double)dinv[q], v, acz);
    }
    block_partial(acc, partials + c * kRedBlocks + blockIdx.x);
    if (dinv) block_partial(acz, partials + ((size_t)gridDim.y + c) * kRedBlocks + blockIdx.x);
}

// dst = dinv o src (dinv != NULL) or dst = src: the preconditioned residual z
template <typename T>
__global__ void __launch_bounds__(256)
precond_kernel(T* __restrict__ dst, const T* __restrict__ src, const T* __restrict__ dinv, int64_t n)
{
    const int64_t o = (int64_t)blockIdx.y * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[o + q] = dinv ? T((double)dinv[q] * (double)src[o + q]) : src[o + q];
}

// dinv = 1 / diag on the free nodes, 0 on the masked (Dirichlet) ones; also the float copy
__global__ void __launch_bounds__(256)
invert_diag_kernel(double* __restrict__ dinv, float* __restrict__ dinv32, const double* __restrict__ diag,
                   const uint8_t* __restrict__ mask, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        const double v = (mask && mask[q]) ? 0.0 : 1.0 / diag[q];
        dinv[q] = v;
        if (dinv32) dinv32[q] = (float)v;
    }
}

// With XUPD, x += alpha p with this iteration's p (whenever alpha != 0, as the r update pairs
// it); then p = z + beta p, z = dinv o r (dinv != NULL) or r, unless the column has converged or
// broken down
template <typename TX, typename T, bool XUPD>
__global__ void __launch_bounds__(256)
cg_dir_kernel(TX* __restrict__ x, T* __restrict__ p, const T* __restrict__ r, const CgScal* __restrict__ sc,
              int64_t n, const T* __restrict__ dinv)
{
    const int c = blockIdx.y;
    const bool dir = !(sc[c].converged || sc[c].breakdown);
    const double be = sc[c].beta;
    const int64_t o = (int64_t)c * n;
    if constexpr (!XUPD) {
        if (!dir) return;
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
            const double z = dinv ? (double)dinv[q] * (double)r[o + q] : (double)r[o + q];
            p[o + q] = (T)(z + be * (double)p[o + q]);
        }
    } else {
        const double al = sc[c].alpha;
        if (al == 0.0 && !dir) return;
        for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
            const double pv = (double)p[o + q];
            if (al != 0.0) x[o + q] = (TX)((double)x[o + q] + al * pv);
            if (dir) {
                const double z = dinv ? (double)dinv[q] * (double)r[o + q] : (double)r[o + q];
                p[o + q] = (T)(z + be * pv);
            }
        }
    }
}

// r = b - Ax (FP64).  Entries under the Dirichlet mask come out 0 because Ax is 0 there and the
// solver has checked that b is 0 there (masked_rhs_kernel).
__global__ void __launch_bounds__(256)
residual_kernel(double* __restrict__ r, const double* __restrict__ b, const double* __restrict__ Ax,
                int64_t n)
{
    const int64_t o = (int64_t)blockIdx.y * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        r[o + q] = b[o + q] - Ax[o + q];
}

// dst(float) = src(double) * scale[c]; scale = 1 / |r| from the scalar state
__global__ void __launch_bounds__(256)
scale_to_f32_kernel(float* __restrict__ dst, const double* __restrict__ src,
                    const CgScal* __restrict__ sc, int64_t n)
{
    const int c = blockIdx.y;
    const double nr = sqrt(sc[c].rr);
    const double s = nr > 0.0 ? 1.0 / nr : 0.0;
    const int64_t o = (int64_t)c * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[o + q] = (float)(src[o + q] * s);
}

// x += |r| d (FP64 update with the float correction)
__global__ void __launch_bounds__(256)
ir_update_kernel(double* __restrict__ x, const float* __restrict__ d, const CgScal* __restrict__ sc,
                 int64_t n)
{
    const int c = blockIdx.y;
    const double nr = sqrt(sc[c].rr);
    const int64_t o = (int64_t)c * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        x[o + q] += nr * (double)d[o + q];
}

// dst(float) = src(double)
__global__ void __launch_bounds__(256)
to_f32_kernel(float* __restrict__ dst, const double* __restrict__ src, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[q] = (float)src[q];
}

// x += sgn d (FP64 accumulation of the reduced-precision iterate) unless the column's iterate
// was flagged non-finite; d = 0 if `clear`
__global__ void __launch_bounds__(256)
fold_kernel(double* __restrict__ x, float* __restrict__ d, const CgScal* __restrict__ sc, int64_t n,
            double sgn, int clear)
{
    const int c = blockIdx.y;
    const bool keep = sc[c].breakdown != 2;
    const int64_t o = (int64_t)c * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
        if (keep) x[o + q] += sgn * (double)d[o + q];
        if (clear) d[o + q] = 0.0f;
    }
}

template <typename T>
__global__ void __launch_bounds__(256)
copy_kernel(T* __restrict__ dst, const T* __restrict__ src, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[q] = src[q];
}

template <typename T>
__global__ void __launch_bounds__(256) zero_kernel(T* __restrict__ dst, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        dst[q] = T(0);
}

// flag = 1 if some column of b is nonzero (or not a number) on a masked (Dirichlet) node
__global__ void __launch_bounds__(256)
masked_rhs_kernel(const double* __restrict__ b, const uint8_t* __restrict__ mask, int64_t n, int* __restrict__ flag)
{
    const int64_t o = (int64_t)blockIdx.y * n;
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256)
        if (mask[q] && !(b[o + q] == 0.0)) *flag = 1;
}

__global__ void set_tol_kernel(CgScal* sc, const double* __restrict__ partials, double rtol)
{
    const int c = blockIdx.x;
    const double bb = block_sum_partials(partials + c * kRedBlocks);
    if (threadIdx.x == 0) {
        sc[c].tol2 = rtol * rtol * bb;
        sc[c].converged = 0;
        sc[c].breakdown = 0;
    }
}

static unsigned vgrid(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

// Device workspace carve-up (256-byte aligned pieces).
struct Carver {
    char* p;
    size_t used = 0, cap;
    template <typename T>
    T* take(size_t count)
    {
        size_t off = (used + 255) & ~size_t(255);
        used = off + count * sizeof(T);
        return (p && used <= cap) ? reinterpret_cast<T*>(p + off) : nullptr;
    }
};

struct CgWork {
    double *r, *p, *Ap;            // FP64 global vectors [nrhs][ng]
    double *pl, *wl;               // FP64 local vectors [nrhs][nl]
    float *b32, *r32, *p32, *Ap32, *d32; // inner global vectors
    float *pl32, *wl32;            // inner local vectors
    double* partials;              // [2][nrhs][kRedBlocks]
    double* dinv;                  // Jacobi preconditioner [n_global] (or NULL)
    float* dinv32;                 // its float copy for the reduced-precision recurrences
    CopyPair* pairs;               // [n_global]
    CgScal *sc, *sc_in;            // outer / inner scalar state [nrhs]
    int* flag;                     // masked right-hand-side check
    double* epart;                 // fused operator: per-work-group energies [fused_e] (or NULL)
};

// fused_e > 0: room for the fused single-column operator of a mesh of fused_e elements
static void carve(Carver& cv, int64_t nl, int64_t ng, int nrhs, bool mixed, bool pre, CgWork& w,
                  int64_t fused_e = 0)
{
    w.r = cv.take<double>(ng * nrhs);
    w.p = cv.take<double>(ng * nrhs);
    w.Ap = cv.take<double>(ng * nrhs);
    w.pl = cv.take<double>(nl * nrhs);
    w.wl = cv.take<double>(nl * nrhs);
    if (mixed) {
        w.b32 = cv.take<float>(ng * nrhs);
        w.r32 = cv.take<float>(ng * nrhs);
        w.p32 = cv.take<float>(ng * nrhs);
        w.Ap32 = cv.take<float>(ng * nrhs);
        w.d32 = cv.take<float>(ng * nrhs);
        w.pl32 = cv.take<float>(nl * nrhs);
        w.wl32 = cv.take<float>(nl * nrhs);
    } else {
        w.b32 = w.r32 = w.p32 = w.Ap32 = w.d32 = w.pl32 = w.wl32 = nullptr;
    }
    w.partials = cv.take<double>((size_t)2 * kRedBlocks * nrhs);
    w.dinv = pre ? cv.take<double>(ng) : nullptr;
    w.dinv32 = (pre && mixed) ? cv.take<float>(ng) : nullptr;
    w.pairs = cv.take<CopyPair>(ng);
    w.sc = cv.take<CgScal>(nrhs);
    w.sc_in = cv.take<CgScal>(nrhs);
    w.flag = cv.take<int>(1);
    w.epart = fused_e > 0 ? cv.take<double>(fused_e) : nullptr;
}

// The assembled operator y = mask o Q^T AxLocal(Q x) over one mesh (ax_local) or over the
// union of many meshes (one batched persistent launch whose X/Y pointers are the local work
// vectors; the union gather-scatter then assembles every mesh at once).
struct Operator {
    int64_t n_local = 0, n_global = 0;
    const int32_t* l2g = nullptr;
    const int64_t* gptr = nullptr;
    const CopyPair* pairs = nullptr;  // first two copies per global node, mask applied
    const int32_t* gidx = nullptr;
    const uint8_t* mask = nullptr;
    const ax_problem* p = nullptr;  // single mesh
    const ax_batch_plan* plan64 = nullptr;
    const void* ws64 = nullptr;
    const ax_batch_plan* plan32 = nullptr;
    const void* ws32 = nullptr;
    bool batched_gather = false;    // the batched plans read the global vector through l2g
    const double* dinv64 = nullptr;  // Jacobi preconditioner (NULL: none)
    const float* dinv32 = nullptr;
    double* epart = nullptr;           // fused single-column operator (NULL: not used)
    int64_t epart_cap = 0;
};

template <typename T>
static const T* op_dinv(const Operator& op)
{
    if constexpr (sizeof(T) == 8) return op.dinv64;
    else return op.dinv32;
}

// Local result yl = AxLocal(Q x).  With AX_CG_GATHER the gather Q x of one mesh is fused into
// the AxLocal load (FP64/FP32, GLL D): the prefetching kernel reads each node column through the
// local-to-global map one element ahead, so the local copy of x is never written or read back.
// Measured on one MI355X, N = 7, 32^3, CG to 1e-10 (interleaved, same iterations): FP64
// 0.665 -> 0.565 s, FP32-inner reliable 0.454 -> 0.403 s, Jacobi mixed 0.403 -> 0.360 s against
// the separate gather kernel + streaming AxLocal (an earlier form of the kernel measured the
// other way round).  The batched operator keeps the separate gather.
#ifndef AX_CG_GATHER
#define AX_CG_GATHER 1
#endif
// The same for the batched operator of cg_solve_batched: every mesh's per-item kernel reads the
// global vector through its part of the union's local-to-global map.
#ifndef AX_CG_GATHER_BATCHED
#define AX_CG_GATHER_BATCHED 1
#endif
template <typename T>
static int apply_local(const Operator& op, int nrhs, int prec, const T* x, T* xl, T* yl, hipStream_t st)
{
    const int dt = sizeof(T) == 8 ? AX_FP64 : AX_FP32;
    if (AX_CG_GATHER && op.p && prec != AX_FP16_ACC32 && centro_antisymmetric(op.p->N + 1, op.p->D))
        return ax_local_gather(*op.p, nrhs, prec, x, op.n_global, yl, st);
    if (!op.batched_gather)
        AX_TRY(gs_apply(op.n_local, op.n_global, op.l2g, op.gptr, op.gidx, nullptr, GS_Q, nrhs, dt, x, xl, st));
    if (op.p) {
        const ax_problem& pb = *op.p;
        return ax_local(pb.E, pb.N, pb.geom, pb.geo, pb.D, pb.xi, pb.w, nrhs, prec, xl, yl, st);
    }
    const ax_batch_plan* plan = sizeof(T) == 8 ? op.plan64 : op.plan32;
    void* ws = const_cast<void*>(sizeof(T) == 8 ? op.ws64 : op.ws32);
    if (op.batched_gather) {
        AX_TRY(batched_set_source(plan, ws, x, st));
        return ax_local_batched(plan, ws, st);
    }
    return ax_local_batched(plan, ws, st);
}

template <typename T>
static int apply_op(const Operator& op, int nrhs, int prec, const T* x, T* y, T* xl, T* yl, hipStream_t st)
{
    const int dt = sizeof(T) == 8 ? AX_FP64 : AX_FP32;
    AX_TRY(apply_local<T>(op, nrhs, prec, x, xl, yl, st));
    AX_TRY(gs_apply(op.n_local, op.n_global, op.l2g, op.gptr, op.gidx, op.mask, GS_QT, nrhs, dt, yl, y, st));
    return AX_OK;
}

template <typename TA, typename TB>
static int dot(const TA* a, const TB* b, int64_t n, int nrhs, double* partials, hipStream_t st)
{
    hipLaunchKernelGGL((dot_partial_kernel<TA, TB>), dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0, st, a,
                       b, n, partials);
    return hip_check(hipGetLastError(), "dot");
}

static int scal(const double* partials, CgScal* sc, int mode, int nrhs, hipStream_t st, bool pre = false)
{
    hipLaunchKernelGGL(cg_scalar_kernel, dim3(nrhs), dim3(kRedThreads), 0, st, partials, sc, mode, pre ? 1 : 0);
    return hip_check(hipGetLastError(), "cg scalar");
}

// r . r and r . z partials (z = dinv o r), then scalar mode 0 or 3
template <typename T>
static int rr_rz(const T* r, const T* dinv, int64_t n, int nrhs, double* partials, CgScal* sc, int mode, hipStream_t st)
{
    hipLaunchKernelGGL(rr_rz_kernel<T>, dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0, st, r, dinv, n, partials);
    AX_TRY(hip_check(hipGetLastError(), "r.r / r.z"));
    return scal(partials, sc, mode, nrhs, st, dinv != nullptr);
}

// Host view of the scalar state (synchronises the stream).
static int poll(const CgScal* sc, int nrhs, std::vector<CgScal>& h, hipStream_t st)
{
    h.resize(nrhs);
    AX_TRY(hip_check(hipMemcpyAsync(h.data(), sc, sizeof(CgScal) * nrhs, hipMemcpyDeviceToHost, st),
                     "poll copy"));
    return hip_check(hipStreamSynchronize(st), "poll sync");
}

// Where x += alpha p goes.  Folded into cg_dir_kernel it saves one pass over p per iteration,
// which pays once a vector no longer stays in the 256 MB last-level cache between update_dot and
// cg_dir (N=7, 32^3: FP64 vectors of 91 MB, 4% less time per iteration).  For smaller vectors the
// second read of p hits that cache and the x stream moved into cg_dir is the colder one (FP32
// vectors of 46 MB: 8% more time merged), so there x stays in update_dot.
static bool merged_x_update(int64_t vector_bytes) { return vector_bytes > (int64_t)64 << 20; }

// The fused operator (one column, single mesh, FP32 gathering AxLocal): AxLocal also sums
// p^T A p as the elements' energies (D X_e)^T G_e (D X_e), so Q^T does not read p.  Measured at
// N = 7, 32^3: FP32 AxLocal 63.8 -> 64.1 us, Q^T 70.2 -> 65.1 us per application (FP32-inner CG
// 0.400 -> 0.393 s).  In FP64 the energies pushed the kernel's register use into spills (90 ->
// 102 us, the same again saved in Q^T), so FP64 keeps the dot in Q^T.  Writing the nodes with a
// single unmasked copy (the element interiors) straight from AxLocal to the global vector, so
// that Q^T visits only the shared nodes, measured slower still (FP64 CG 0.551 -> 0.638 s): the
// reload of the map before the stores serialises the item's memory traffic and the stores
// diverge per node.
static bool fused_operator(const Operator& op, int prec)
{
    return AX_CG_FUSED && op.epart && op.p && prec == AX_FP32 && centro_antisymmetric(op.p->N + 1, op.p->D);
}

// One block of kPoll CG iterations (device scalars only: capturable).
template <typename TX, typename T>
static int cg_block(const Operator& op, int nrhs, int prec, TX* x, T* r, T* p, T* Ap, T* pl, T* wl,
                    double* partials, CgScal* sc, int count, hipStream_t st)
{
    const int64_t ng = op.n_global;
    const dim3 g(vgrid(ng), nrhs);
    const T* dinv = op_dinv<T>(op);
    const bool merged = merged_x_update(ng * nrhs * (int64_t)sizeof(T));
    const bool fused = nrhs == 1 && fused_operator(op, prec);
    for (int q = 0; q < count; ++q) {
        if (fused) {
            if constexpr (sizeof(T) == 4) {
                // AxLocal also leaves the energies whose sum is p^T A p
                FusedOut fo{op.epart, op.epart_cap, 0};
                AX_TRY(ax_local_gather_fused(*op.p, p, ng, wl, &fo, st));
                hipLaunchKernelGGL((qt_dot_kernel<T, true>), dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0, st, ng,
                                   op.pairs, op.gptr, op.gidx, op.n_local, wl, p, Ap, partials, op.epart,
                                   fo.nparts);
            } else {
                return fail(AX_ERR_ARG, "internal: the fused operator is FP32");
            }
        } else {
            AX_TRY(apply_local<T>(op, nrhs, prec, p, pl, wl, st));
            hipLaunchKernelGGL((qt_dot_kernel<T, false>), dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0, st, ng,
                               op.pairs, op.gptr, op.gidx, op.n_local, wl, p, Ap, partials, nullptr, 0);
        }
        AX_TRY(scal(partials, sc, 1, nrhs, st));
        if (merged)
            hipLaunchKernelGGL((update_dot_kernel<TX, T, false>), dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0,
                               st, x, r, p, Ap, sc, ng, dinv, partials);
        else
            hipLaunchKernelGGL((update_dot_kernel<TX, T, true>), dim3(kRedBlocks, nrhs), dim3(kRedThreads), 0,
                               st, x, r, p, Ap, sc, ng, dinv, partials);
        AX_TRY(scal(partials, sc, 2, nrhs, st, dinv != nullptr));
        if (merged)
            hipLaunchKernelGGL((cg_dir_kernel<TX, T, true>), g, dim3(256), 0, st, x, p, r, sc, ng, dinv);
        else
            hipLaunchKernelGGL((cg_dir_kernel<TX, T, false>), g, dim3(256), 0, st, x, p, r, sc, ng, dinv);
    }
    return hip_check(hipGetLastError(), "cg iteration");
}

// A captured kPoll-iteration block, reused while the buffers stay the same.
struct GraphCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    ~GraphCache()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// `count` iterations: replays the captured kPoll-iteration graph when count == kPoll (capturing
// it on first use), otherwise enqueues the kernels directly.
template <typename TX, typename T>
static int run_block(const Operator& op, int nrhs, int prec, TX* x, T* r, T* p, T* Ap, T* pl, T* wl,
                     double* partials, CgScal* sc, int count, GraphCache* gc, hipStream_t st)
{
    if (gc && count == kPoll) {
        if (!gc->exec) {
            AX_TRY(hip_check(hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed), "begin capture"));
            const int s = cg_block<TX, T>(op, nrhs, prec, x, r, p, Ap, pl, wl, partials, sc, kPoll, st);
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(st, &graph);
            if (s != AX_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return s;
            }
            AX_TRY(hip_check(ec, "end capture"));
            gc->graph = graph;
            AX_TRY(hip_check(hipGraphInstantiate(&gc->exec, graph, nullptr, nullptr, 0), "graph instantiate"));
        }
        return hip_check(hipGraphLaunch(gc->exec, st), "graph launch");
    }
    return cg_block<TX, T>(op, nrhs, prec, x, r, p, Ap, pl, wl, partials, sc, count, st);
}

// Plain CG in precision T on A_T x = b (x holds the initial guess unless x_zero).  `iters` gets
// the largest iteration count over the columns.  Returns AX_OK (all converged),
// AX_ERR_NOT_CONVERGED or AX_ERR_BREAKDOWN.
template <typename TX, typename T>
static int cg_core(const Operator& op, int nrhs, int prec, const T* b, TX* x, T* r, T* p, T* Ap,
                   T* pl, T* wl, double* partials, CgScal* sc, double rtol, int max_it, bool x_zero,
                   GraphCache* gc, int& iters, hipStream_t st)
{
    const int64_t ng = op.n_global;
    const dim3 g(vgrid(ng), nrhs);
    AX_TRY(dot(b, b, ng, nrhs, partials, st));
    hipLaunchKernelGGL(set_tol_kernel, dim3(nrhs), dim3(kRedThreads), 0, st, sc, partials, rtol);
    if (x_zero) {
        hipLaunchKernelGGL(copy_kernel<T>, dim3(vgrid(ng * nrhs)), dim3(256), 0, st, r, b, ng * nrhs);
    } else {
        if constexpr (std::is_same<T, double>::value && std::is_same<TX, double>::value) {
            AX_TRY(apply_op<T>(op, nrhs, prec, (const T*)x, Ap, pl, wl, st));
            hipLaunchKernelGGL(residual_kernel, g, dim3(256), 0, st, (double*)r, (const double*)b,
                               (const double*)Ap, ng);
        } else {
            return fail(AX_ERR_ARG, "internal: warm start needs FP64 vectors");
        }
    }
    hipLaunchKernelGGL(precond_kernel<T>, g, dim3(256), 0, st, p, r, op_dinv<T>(op), ng);
    AX_TRY(rr_rz<T>(r, op_dinv<T>(op), ng, nrhs, partials, sc, 0, st));
    std::vector<CgScal> h;
    int it = 0;
    for (;;) {
        AX_TRY(poll(sc, nrhs, h, st));
        bool all = true, brk = false;
        iters = 0;
        for (int c = 0; c < nrhs; ++c) {
            all = all && h[c].converged;
            brk = brk || h[c].breakdown;
            iters = iters > h[c].iters ? iters : h[c].iters;
        }
        if (brk) return fail(AX_ERR_BREAKDOWN, "CG breakdown (p^T A p <= 0 or non-finite)");
        if (all) return AX_OK;
        if (it >= max_it) return fail(AX_ERR_NOT_CONVERGED, "CG reached %d iterations", max_it);
        const int count = (max_it - it) < kPoll ? (max_it - it) : kPoll;
        AX_TRY((run_block<TX, T>(op, nrhs, prec, x, r, p, Ap, pl, wl, partials, sc, count, gc, st)));
        it += count;
    }
}

static int validate(const ax_problem* p, int nrhs, const ax_cg_opts* o)
{
    if (!p || !o) return fail(AX_ERR_ARG, "NULL problem or options");
    if (nrhs < 1) return fail(AX_ERR_ARG, "nrhs < 1");
    if (p->E < 0 || p->n_global < 0) return fail(AX_ERR_ARG, "negative size");
    if (p->N < 1 || p->N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", p->N);
    if (p->geom != AX_TRILINEAR && p->geom != AX_PARALLELEPIPED) return fail(AX_ERR_UNSUPPORTED, "geometry");
    if (o->inner_prec != AX_FP64 && o->inner_prec != AX_FP32 && o->inner_prec != AX_FP16_ACC32)
        return fail(AX_ERR_UNSUPPORTED, "inner precision %d", o->inner_prec);
    if (!(o->rtol > 0.0)) return fail(AX_ERR_ARG, "rtol must be > 0");
    if (o->max_it < 1) return fail(AX_ERR_ARG, "max_it < 1");
    if (o->inner_prec != AX_FP64 && (!(o->inner_rtol > 0.0) || o->max_outer < 1))
        return fail(AX_ERR_ARG, "refinement needs inner_rtol > 0 and max_outer >= 1");
    if (o->refine != AX_REFINE_RESTART && o->refine != AX_REFINE_RELIABLE)
        return fail(AX_ERR_ARG, "refine must be AX_REFINE_RESTART or AX_REFINE_RELIABLE");
    if (o->precond != AX_PRECOND_NONE && o->precond != AX_PRECOND_JACOBI)
        return fail(AX_ERR_ARG, "precond must be AX_PRECOND_NONE or AX_PRECOND_JACOBI");
    if (o->inner_prec != AX_FP64 && o->refine == AX_REFINE_RELIABLE && !(o->inner_rtol < 1.0))
        return fail(AX_ERR_ARG, "reliable updates need inner_rtol < 1");
    if (p->E > 0 && (!p->geo || !p->D || !p->w || !p->l2g || !p->gptr || !p->gidx))
        return fail(AX_ERR_ARG, "NULL problem array");
    if (p->geom == AX_TRILINEAR && !p->xi) return fail(AX_ERR_ARG, "xi is NULL");
    const int64_t N1 = p->N + 1;
    if (p->E > 0x7fffffffLL / (N1 * N1 * N1))
        return fail(AX_ERR_UNSUPPORTED, "more than 2^31 - 1 local nodes (local ids are int32)");
    return AX_OK;
}

// Jacobi preconditioner of the assembled operator: the element diagonals (recomputed factors)
// in the local work vector, assembled by Q^T, inverted on the free nodes (0 on the masked ones).
static int jacobi_setup(Operator& op, const CgWork& w, hipStream_t st)
{
    if (!w.dinv) return AX_OK;
    AX_TRY(gs_apply(op.n_local, op.n_global, op.l2g, op.gptr, op.gidx, op.mask, GS_QT, 1, AX_FP64, w.wl, w.Ap, st));
    hipLaunchKernelGGL(invert_diag_kernel, dim3(vgrid(op.n_global)), dim3(256), 0, st, w.dinv, w.dinv32, w.Ap,
                       op.mask, op.n_global);
    AX_TRY(hip_check(hipGetLastError(), "jacobi inverse"));
    op.dinv64 = w.dinv;
    op.dinv32 = w.dinv32;
    return AX_OK;
}

// The right-hand side must vanish on the Dirichlet nodes (the assembled operator's rows there
// are zero, so a nonzero entry could never be matched and the solve would only stall).
// Synchronises the stream; AX_ERR_ARG if b violates it.
static int check_masked_rhs(const double* b, const uint8_t* mask, int64_t ng, int nrhs, int* flag, hipStream_t st)
{
    if (!mask || ng == 0) return AX_OK;
    hipLaunchKernelGGL(zero_kernel<int>, dim3(1), dim3(256), 0, st, flag, (int64_t)1);
    hipLaunchKernelGGL(masked_rhs_kernel, dim3(vgrid(ng), nrhs), dim3(256), 0, st, b, mask, ng, flag);
    int h = 0;
    AX_TRY(hip_check(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "mask check copy"));
    AX_TRY(hip_check(hipStreamSynchronize(st), "mask check sync"));
    if (h) return fail(AX_ERR_ARG, "b is nonzero (or not a number) on a masked (Dirichlet) node");
    return AX_OK;
}

// Shared driver of cg_solve and cg_solve_batched.
static int solve(const Operator& op, int64_t nl, int nrhs, const double* b, double* x, const ax_cg_opts* o,
                 ax_cg_report* rep, CgWork& w, hipStream_t st)
{
    const int64_t ng = op.n_global;
    const dim3 g(vgrid(ng), nrhs);
    const bool mixed = o->inner_prec != AX_FP64;
    int status = AX_OK;
    std::vector<CgScal> h;
    GraphCache gc64, gc32;
    const bool graphs = o->use_graph != 0;

    auto true_residual = [&](double& worst) -> int {
        AX_TRY(apply_op<double>(op, nrhs, AX_FP64, x, w.Ap, w.pl, w.wl, st));
        hipLaunchKernelGGL(residual_kernel, g, dim3(256), 0, st, w.r, b, w.Ap, ng);
        AX_TRY(dot(b, b, ng, nrhs, w.partials, st));
        hipLaunchKernelGGL(set_tol_kernel, dim3(nrhs), dim3(kRedThreads), 0, st, w.sc, w.partials, 1.0);
        AX_TRY(dot(w.r, w.r, ng, nrhs, w.partials, st));
        AX_TRY(scal(w.partials, w.sc, 0, nrhs, st));
        AX_TRY(poll(w.sc, nrhs, h, st));
        worst = 0.0;
        bool bad = false;
        for (int c = 0; c < nrhs; ++c) {
            const double rel = h[c].tol2 > 0 ? std::sqrt(h[c].rr / h[c].tol2) : std::sqrt(h[c].rr);
            if (!std::isfinite(rel)) bad = true;
            else worst = worst > rel ? worst : rel;
        }
        if (bad) worst = std::nan("");
        return AX_OK;
    };

    if (!mixed) {
        int total = 0;
        double worst = 0.0;
        for (int restart = 0; restart < 4; ++restart) {
            int it = 0;
            status = cg_core<double, double>(op, nrhs, AX_FP64, b, x, w.r, w.p, w.Ap, w.pl, w.wl, w.partials, w.sc,
                                             o->rtol, o->max_it - total, false, graphs ? &gc64 : nullptr, it, st);
            total += it;
            if (status == AX_ERR_BREAKDOWN) break;
            if (status != AX_OK && status != AX_ERR_NOT_CONVERGED) return status;
            AX_TRY(true_residual(worst));
            if (worst <= o->rtol || total >= o->max_it) break;
        }
        rep->outer_it = 1;
        rep->inner_it_total = total;
        rep->rel_res_true = worst;
        if (status == AX_OK && !(worst <= o->rtol)) status = AX_ERR_NOT_CONVERGED;
    } else if (o->refine == AX_REFINE_RELIABLE) {
        // One reduced-precision CG recurrence (float vectors, inner_prec AxLocal, FP64-accumulated
        // dot products) whose iterate d is folded into the FP64 solution, and whose residual is
        // replaced by the FP64 true residual b - A x, every time its own residual has dropped by
        // inner_rtol since the last replacement (reliable updates); the search direction is kept,
        // so the Krylov space is not thrown away as in restarted refinement.
        const int64_t n = ng * nrhs;
        const dim3 gv(vgrid(n));
        int total = 0, updates = 0;
        double worst = 0.0;
        std::vector<CgScal> hi;
        AX_TRY(true_residual(worst));
        if (worst > o->rtol) {
            hipLaunchKernelGGL(to_f32_kernel, gv, dim3(256), 0, st, w.r32, w.r, n);
            hipLaunchKernelGGL(precond_kernel<float>, g, dim3(256), 0, st, w.p32, w.r32, op.dinv32, ng);
            hipLaunchKernelGGL(zero_kernel<float>, gv, dim3(256), 0, st, w.d32, n);
            AX_TRY(dot(b, b, ng, nrhs, w.partials, st));
            hipLaunchKernelGGL(set_tol_kernel, dim3(nrhs), dim3(kRedThreads), 0, st, w.sc_in, w.partials, o->rtol);
            AX_TRY(rr_rz<float>(w.r32, op.dinv32, ng, nrhs, w.partials, w.sc_in, 0, st));
            AX_TRY(poll(w.sc_in, nrhs, hi, st));
            std::vector<double> rref(nrhs);
            for (int c = 0; c < nrhs; ++c) rref[c] = hi[c].rr;
            const double d2 = o->inner_rtol * o->inner_rtol;
            int since = 0;
            for (;;) {
                const int count = (o->max_it - total) < kPoll ? (o->max_it - total) : kPoll;
                AX_TRY((run_block<float, float>(op, nrhs, o->inner_prec, w.d32, w.r32, w.p32, w.Ap32, w.pl32,
                                                w.wl32, w.partials, w.sc_in, count, graphs ? &gc32 : nullptr, st)));
                total += count;
                since += count;
                AX_TRY(poll(w.sc_in, nrhs, hi, st));
                bool all = true, brk = false, drop = false;
                for (int c = 0; c < nrhs; ++c) {
                    all = all && hi[c].converged;
                    brk = brk || hi[c].breakdown;
                    drop = drop || (!hi[c].converged && hi[c].rr <= d2 * rref[c]);
                }
                // besides the residual drop, the true residual is checked at least every
                // kReliableCheck iterations: a recurrence that drifts away from the FP64 operator
                // (e.g. with a half-precision AxLocal) is caught and discarded
                if (!(all || brk || drop || since >= kReliableCheck || total >= o->max_it)) continue;
                since = 0;
                if (brk) {
                    AX_TRY(dot(w.d32, w.d32, ng, nrhs, w.partials, st));
                    AX_TRY(scal(w.partials, w.sc_in, 4, nrhs, st));
                }
                const double prev = worst;
                hipLaunchKernelGGL(fold_kernel, g, dim3(256), 0, st, x, w.d32, w.sc_in, ng, 1.0, 0);
                AX_TRY(true_residual(worst));
                ++updates;
                bool restart_dir = brk;
                if (!(worst < prev)) {
                    // the recurrence has drifted from the FP64 operator (its own residual fell,
                    // the true one did not): take the update back and restart the direction
                    hipLaunchKernelGGL(fold_kernel, g, dim3(256), 0, st, x, w.d32, w.sc_in, ng, -1.0, 0);
                    AX_TRY(true_residual(worst));
                    restart_dir = true;
                }
                hipLaunchKernelGGL(zero_kernel<float>, gv, dim3(256), 0, st, w.d32, n);
                if (!std::isfinite(worst)) {
                    status = fail(AX_ERR_BREAKDOWN, "non-finite true residual");
                    break;
                }
                if (worst <= o->rtol || total >= o->max_it || updates >= o->max_outer) break;
                hipLaunchKernelGGL(to_f32_kernel, gv, dim3(256), 0, st, w.r32, w.r, n);
                if (restart_dir) hipLaunchKernelGGL(precond_kernel<float>, g, dim3(256), 0, st, w.p32, w.r32, op.dinv32, ng);
                AX_TRY(rr_rz<float>(w.r32, op.dinv32, ng, nrhs, w.partials, w.sc_in, 3, st));
                AX_TRY(poll(w.sc_in, nrhs, hi, st));
                for (int c = 0; c < nrhs; ++c) rref[c] = hi[c].rr;
            }
            int its = 0;
            for (int c = 0; c < nrhs; ++c) its = its > hi[c].iters ? its : hi[c].iters;
            total = its;
        }
        rep->outer_it = updates;
        rep->inner_it_total = total;
        rep->rel_res_true = worst;
        if (status == AX_OK) status = worst <= o->rtol ? AX_OK : AX_ERR_NOT_CONVERGED;
    } else {
        int total = 0, outer = 0;
        double worst = 0.0;
        for (outer = 0; outer < o->max_outer; ++outer) {
            AX_TRY(true_residual(worst));
            if (worst <= o->rtol) break;
            hipLaunchKernelGGL(scale_to_f32_kernel, g, dim3(256), 0, st, w.b32, w.r, w.sc, ng);
            hipLaunchKernelGGL(zero_kernel<float>, dim3(vgrid(ng * nrhs)), dim3(256), 0, st, w.d32, ng * nrhs);
            int it = 0;
            // the inner solve needs to reduce the residual by at most rtol / |r| (with a safety
            // factor of 2): the last refinement step is then only as long as it has to be
            const double need = 0.5 * o->rtol / (worst > 0.0 ? worst : 1.0);
            const double itol = need > o->inner_rtol ? need : o->inner_rtol;
            const int s = cg_core<float, float>(op, nrhs, o->inner_prec, w.b32, w.d32, w.r32, w.p32, w.Ap32,
                                                w.pl32, w.wl32, w.partials, w.sc_in, itol, o->max_it,
                                                true, graphs ? &gc32 : nullptr, it, st);
            // an inner solve that stops on its iteration limit or breaks down still yields a
            // useful correction; only launch errors abort
            if (s != AX_OK && s != AX_ERR_NOT_CONVERGED && s != AX_ERR_BREAKDOWN) return s;
            clear_error();
            total += it;
            hipLaunchKernelGGL(ir_update_kernel, g, dim3(256), 0, st, x, w.d32, w.sc, ng);
            AX_TRY(hip_check(hipGetLastError(), "refinement update"));
        }
        if (outer == o->max_outer) AX_TRY(true_residual(worst));
        rep->outer_it = outer;
        rep->inner_it_total = total;
        rep->rel_res_true = worst;
        status = worst <= o->rtol ? AX_OK : AX_ERR_NOT_CONVERGED;
    }
    (void)nl;
    return status;
}

// The solver runs on a private non-blocking stream of the calling thread (a HIP graph cannot be
// captured on the null stream); the caller's stream is synchronised before and after.
static int private_stream(hipStream_t& s)
{
    static thread_local hipStream_t ps = nullptr;
    if (!ps) AX_TRY(hip_check(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking), "stream create"));
    s = ps;
    return AX_OK;
}

static int finish(int status, ax_cg_report* rep, const std::chrono::steady_clock::time_point& t0,
                  hipStream_t st, hipStream_t caller)
{
    AX_TRY(hip_check(hipStreamSynchronize(st), "cg sync"));
    AX_TRY(hip_check(hipStreamSynchronize(caller), "cg sync"));
    rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep->status = status;
    if (status != AX_OK && ax_last_error()[0] == '\0')
        set_error("cg_solve: relative residual %.3e above the target", rep->rel_res_true);
    return status;
}

// Elements of room for the fused single-column operator (0: the solve does not use it)
static int64_t fused_elements(const ax_problem* p, int nrhs, const ax_cg_opts* o)
{
    return (AX_CG_FUSED && nrhs == 1 && p->E > 0 && o->inner_prec == AX_FP32) ? p->E : 0;
}

}  // namespace ax

using namespace ax;

extern "C" int cg_workspace_bytes(const ax_problem* p, int nrhs, const ax_cg_opts* o, size_t* bytes)
{
    clear_error();
    AX_TRY(validate(p, nrhs, o));
    if (!bytes) return fail(AX_ERR_ARG, "bytes is NULL");
    const int N1 = p->N + 1;
    Carver cv{nullptr, 0, 0};
    CgWork w;
    carve(cv, p->E * N1 * N1 * N1, p->n_global, nrhs, o->inner_prec != AX_FP64, o->precond == AX_PRECOND_JACOBI, w,
          fused_elements(p, nrhs, o));
    *bytes = cv.used + 256;
    return AX_OK;
}

extern "C" int cg_solve(const ax_problem* p, int nrhs, const double* b, double* x, const ax_cg_opts* o,
                        ax_cg_report* rep, void* stream)
{
    clear_error();
    AX_TRY(validate(p, nrhs, o));
    if (!rep) return fail(AX_ERR_ARG, "report is NULL");
    std::memset(rep, 0, sizeof(*rep));
    if (p->n_global == 0) return AX_OK;
    if (!b || !x) return fail(AX_ERR_ARG, "b or x is NULL");
    size_t need = 0;
    AX_TRY(cg_workspace_bytes(p, nrhs, o, &need));
    if (!o->workspace || o->workspace_bytes < need)
        return fail(AX_ERR_NOMEM, "workspace of %zu bytes needed", need);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t caller = as_stream(stream), st = nullptr;
    AX_TRY(private_stream(st));
    AX_TRY(hip_check(hipStreamSynchronize(caller), "cg sync"));
    const int N1 = p->N + 1;
    const int64_t nl = p->E * N1 * N1 * N1;
    Carver cv{(char*)(((uintptr_t)o->workspace + 255) & ~uintptr_t(255)), 0, o->workspace_bytes - 256};
    CgWork w;
    carve(cv, nl, p->n_global, nrhs, o->inner_prec != AX_FP64, o->precond == AX_PRECOND_JACOBI, w,
          fused_elements(p, nrhs, o));
    Operator op;
    op.n_local = nl;
    op.n_global = p->n_global;
    op.l2g = p->l2g;
    op.gptr = p->gptr;
    op.gidx = p->gidx;
    op.mask = p->mask;
    op.p = p;
    hipLaunchKernelGGL(copy_pairs_kernel, dim3(vgrid(p->n_global)), dim3(256), 0, st, w.pairs, p->gptr, p->gidx,
                       p->mask, p->n_global);
    op.pairs = w.pairs;
    if (w.epart) {
        op.epart = w.epart;
        op.epart_cap = p->E;
    }
    AX_TRY(check_masked_rhs(b, op.mask, op.n_global, nrhs, w.flag, st));
    if (w.dinv) {
        AX_TRY(ax_local_diag(p->E, p->N, p->geom, p->geo, p->D, p->xi, p->w, w.wl, st));
        AX_TRY(jacobi_setup(op, w, st));
    }
    const int status = solve(op, nl, nrhs, b, x, o, rep, w, st);
    if (status != AX_OK && status != AX_ERR_NOT_CONVERGED && status != AX_ERR_BREAKDOWN) {
        (void)hipStreamSynchronize(st);
        return status;
    }
    return finish(status, rep, t0, st, caller);
}

static int batched_sizes(int n_mesh, const ax_problem* meshes, int64_t& nl, std::vector<int64_t>& lbase)
{
    nl = 0;
    lbase.resize(n_mesh);
    for (int q = 0; q < n_mesh; ++q) {
        const int64_t N1 = meshes[q].N + 1;
        lbase[q] = nl;
        nl += meshes[q].E * N1 * N1 * N1;
    }
    return AX_OK;
}

static int validate_batched(int n_mesh, const ax_problem* meshes, int64_t n_global, int nrhs, const ax_cg_opts* o)
{
    if (n_mesh < 1 || !meshes) return fail(AX_ERR_ARG, "no meshes");
    if (!o) return fail(AX_ERR_ARG, "NULL options");
    if (o->inner_prec == AX_FP16_ACC32) return fail(AX_ERR_UNSUPPORTED, "batched refinement supports FP32 inner solves");
    ax_problem u = meshes[0];
    u.n_global = n_global;
    u.l2g = reinterpret_cast<const int32_t*>(1);
    u.gptr = reinterpret_cast<const int64_t*>(1);
    u.gidx = reinterpret_cast<const int32_t*>(1);
    AX_TRY(validate(&u, nrhs, o));
    size_t bytes = 0;
    AX_TRY(ax_batched_workspace_bytes(n_mesh, meshes, &bytes));
    int64_t nl;
    std::vector<int64_t> lbase;
    batched_sizes(n_mesh, meshes, nl, lbase);
    if (nl > 0x7fffffffLL) return fail(AX_ERR_UNSUPPORTED, "more than 2^31 - 1 local nodes (local ids are int32)");
    return AX_OK;
}

extern "C" int cg_batched_workspace_bytes(int n_mesh, const ax_problem* meshes, int64_t n_global, int nrhs,
                                          const ax_cg_opts* o, size_t* bytes)
{
    clear_error();
    AX_TRY(validate_batched(n_mesh, meshes, n_global, nrhs, o));
    if (!bytes) return fail(AX_ERR_ARG, "bytes is NULL");
    int64_t nl;
    std::vector<int64_t> lbase;
    batched_sizes(n_mesh, meshes, nl, lbase);
    Carver cv{nullptr, 0, 0};
    CgWork w;
    carve(cv, nl, n_global, nrhs, o->inner_prec != AX_FP64, o->precond == AX_PRECOND_JACOBI, w);
    size_t bw = 0;
    AX_TRY(ax_batched_workspace_bytes(n_mesh, meshes, &bw));
    *bytes = cv.used + 2 * ((bw + 255) & ~size_t(255)) + 512;
    return AX_OK;
}

extern "C" int cg_solve_batched(int n_mesh, const ax_problem* meshes, int64_t n_global, const int32_t* l2g,
                                const int64_t* gptr, const int32_t* gidx, const uint8_t* mask, int nrhs,
                                const double* b, double* x, const ax_cg_opts* o, ax_cg_report* rep, void* stream)
{
    clear_error();
    AX_TRY(validate_batched(n_mesh, meshes, n_global, nrhs, o));
    if (!rep) return fail(AX_ERR_ARG, "report is NULL");
    std::memset(rep, 0, sizeof(*rep));
    if (!l2g || !gptr || !gidx || !b || !x) return fail(AX_ERR_ARG, "NULL array");
    size_t need = 0;
    AX_TRY(cg_batched_workspace_bytes(n_mesh, meshes, n_global, nrhs, o, &need));
    if (!o->workspace || o->workspace_bytes < need)
        return fail(AX_ERR_NOMEM, "workspace of %zu bytes needed", need);
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t caller = as_stream(stream), st = nullptr;
    AX_TRY(private_stream(st));
    AX_TRY(hip_check(hipStreamSynchronize(caller), "cg sync"));
    int64_t nl;
    std::vector<int64_t> lbase;
    batched_sizes(n_mesh, meshes, nl, lbase);
    Carver cv{(char*)(((uintptr_t)o->workspace + 255) & ~uintptr_t(255)), 0, o->workspace_bytes - 256};
    CgWork w;
    const bool mixed = o->inner_prec != AX_FP64;
    carve(cv, nl, n_global, nrhs, mixed, o->precond == AX_PRECOND_JACOBI, w);
    size_t bw = 0;
    AX_TRY(ax_batched_workspace_bytes(n_mesh, meshes, &bw));
    char* ws64 = cv.take<char>(bw);
    char* ws32 = cv.take<char>(bw);
    // the batched launches read and write the solver's local work vectors (columns n_local apart)
    std::vector<const void*> xs(n_mesh);
    std::vector<void*> ys(n_mesh);
    std::vector<int64_t> ld(n_mesh, nl);
    ax_batch_plan plan64{}, plan32{};
    for (int q = 0; q < n_mesh; ++q) {
        xs[q] = w.pl + lbase[q];
        ys[q] = w.wl + lbase[q];
    }
    if (AX_CG_GATHER_BATCHED)
        AX_TRY(batched_prepare_gather(n_mesh, meshes, nrhs, AX_FP64, l2g, lbase.data(), n_global, ys.data(),
                                      ld.data(), ws64, bw, &plan64));
    else
        AX_TRY(ax_batched_prepare(n_mesh, meshes, nrhs, AX_FP64, xs.data(), ys.data(), ld.data(), ws64, bw, &plan64));
    if (mixed) {
        for (int q = 0; q < n_mesh; ++q) {
            xs[q] = w.pl32 + lbase[q];
            ys[q] = w.wl32 + lbase[q];
        }
        if (AX_CG_GATHER_BATCHED)
            AX_TRY(batched_prepare_gather(n_mesh, meshes, nrhs, AX_FP32, l2g, lbase.data(), n_global, ys.data(),
                                          ld.data(), ws32, bw, &plan32));
        else
            AX_TRY(ax_batched_prepare(n_mesh, meshes, nrhs, AX_FP32, xs.data(), ys.data(), ld.data(), ws32, bw,
                                      &plan32));
    }
    Operator op;
    op.n_local = nl;
    op.n_global = n_global;
    op.l2g = l2g;
    op.gptr = gptr;
    op.gidx = gidx;
    op.mask = mask;
    op.plan64 = &plan64;
    op.ws64 = ws64;
    op.plan32 = &plan32;
    op.ws32 = ws32;
    op.batched_gather = AX_CG_GATHER_BATCHED != 0;
    hipLaunchKernelGGL(copy_pairs_kernel, dim3(vgrid(n_global)), dim3(256), 0, st, w.pairs, gptr, gidx, mask,
                       n_global);
    op.pairs = w.pairs;
    AX_TRY(check_masked_rhs(b, op.mask, op.n_global, nrhs, w.flag, st));
    if (w.dinv) {
        for (int q = 0; q < n_mesh; ++q) {
            const ax_problem& m = meshes[q];
            AX_TRY(ax_local_diag(m.E, m.N, m.geom, m.geo, m.D, m.xi, m.w, w.wl + lbase[q], st));
        }
        AX_TRY(jacobi_setup(op, w, st));
    }
    const int status = solve(op, nl, nrhs, b, x, o, rep, w, st);
    if (status != AX_OK && status != AX_ERR_NOT_CONVERGED && status != AX_ERR_BREAKDOWN) {
        (void)hipStreamSynchronize(st);
        return status;
    }
    return finish(status, rep, t0, st, caller);
}
