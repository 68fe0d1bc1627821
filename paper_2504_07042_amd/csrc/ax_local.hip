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
//     pencils from an LDS copy of the element (padded layouts chosen so that the home-column,
//     r-pencil and s-pencil accesses are free of bank conflicts; see ax_kernels.h) and hand
//     results back through LDS.
//   * The FP64 matrix cores are no faster here: measured on gfx950, 16x16x4 FP64 MFMA loops
//     reach about 49 TF/s against 63-68 TF/s for FP64 FMA on the vector unit, the two overlap
//     little (issued together in the same waves they take 0.87-0.91 of the summed times), and a
//     dense MFMA contraction cannot use the even-odd split that halves the vector FMAs; so the
//     FP64 contractions stay on the vector unit.
#include "ax_internal.h"
#include "ax_kernels.h"
#include "geom.h"

namespace ax {

int axl_dispatch_f64(int geo_kind, int N, int64_t E, int nrhs, const double* geo, const double* Gs,
                     const double* X, double* Y, const double* D, const double* xi, const double* w,
                     hipStream_t st, const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs,
                     FusedOut* fo = nullptr);
int axl_dispatch_f32(int geo_kind, int N, int64_t E, int nrhs, const double* geo, const float* Gs,
                     const float* X, float* Y, const double* D, const double* xi, const double* w,
                     hipStream_t st, const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs,
                     FusedOut* fo = nullptr);

// values per element and column: (N + 1)^3
static inline int64_t NPL(int N) { return (int64_t)(N + 1) * (N + 1) * (N + 1); }

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

// AxLocal reading X from a global vector through l2g (Q fused into the load); used by the CG
// solver.  FP64 / FP32, trilinear or parallelepiped, GLL differentiation matrix.
int ax_local_gather(const ax_problem& p, int nrhs, int prec, const void* xg, int64_t ldg, void* Y, hipStream_t st)
{
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "gathering AxLocal is FP64/FP32");
    if (p.E == 0) return AX_OK;
    const int gk = p.geom == AX_TRILINEAR ? GEO_TRI : GEO_PARA;
    if (prec == AX_FP64)
        return axl_dispatch_f64(gk, p.N, p.E, nrhs, p.geo, nullptr, (const double*)xg, (double*)Y, p.D, p.xi, p.w, st, p.l2g, ldg, NPL(p.N), p.E * NPL(p.N));
    return axl_dispatch_f32(gk, p.N, p.E, nrhs, p.geo, nullptr, (const float*)xg, (float*)Y, p.D, p.xi, p.w, st, p.l2g, ldg, NPL(p.N), p.E * NPL(p.N));
}

// The CG's fused operator for one column: ax_local_gather that also leaves each work-group's
// element energies X_e^T Y_e in fo->epart (their sum is p^T A p for X = Q p).  FP32.
int ax_local_gather_fused(const ax_problem& p, const float* xg, int64_t ldg, float* yl, FusedOut* fo,
                          hipStream_t st)
{
    if (p.E == 0) {
        fo->nparts = 0;
        return AX_OK;
    }
    const int gk = p.geom == AX_TRILINEAR ? GEO_TRI : GEO_PARA;
    return axl_dispatch_f32(gk, p.N, p.E, 1, p.geo, nullptr, xg, yl, p.D, p.xi, p.w, st, p.l2g, ldg, NPL(p.N),
                            p.E * NPL(p.N), fo);
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
    if (prec == AX_FP64)
        return axl_dispatch_f64(gk, N, E, nrhs, geo, nullptr, (const double*)X, (double*)Y, D, xi, w, st, nullptr, 0, NPL(N), E * NPL(N));
    if (prec == AX_FP32)
        return axl_dispatch_f32(gk, N, E, nrhs, geo, nullptr, (const float*)X, (float*)Y, D, xi, w, st, nullptr, 0, NPL(N), E * NPL(N));
    return ax_local_f16(E, N, gk, geo, nullptr, D, xi, w, nrhs, (const float*)X, (float*)Y, st);
}

// Argument checks shared by the gathering entry points; fills p (E > 0) or returns AX_OK with
// p.E == 0 for an empty mesh.
static int gathered_problem(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                            const double* w, int nrhs, int prec, const int32_t* l2g, int64_t n_global,
                            const void* Xg, void* Y, ax_problem& p)
{
    p = ax_problem{};
    AX_TRY(check_common(E, N, nrhs, prec, Xg, Y, D));
    if (prec == AX_FP16_ACC32) return fail(AX_ERR_UNSUPPORTED, "the gathering operator is FP64/FP32");
    if (geom != AX_TRILINEAR && geom != AX_PARALLELEPIPED)
        return fail(AX_ERR_UNSUPPORTED, "unknown geometry %d", geom);
    if (!w) return fail(AX_ERR_ARG, "w is NULL");
    if (geom == AX_TRILINEAR && !xi) return fail(AX_ERR_ARG, "xi is NULL (needed for trilinear)");
    if (E == 0) return AX_OK;
    if (!geo || !l2g) return fail(AX_ERR_ARG, "geo or l2g is NULL");
    if (n_global < 1) return fail(AX_ERR_ARG, "n_global < 1");
    if (!centro_antisymmetric(N + 1, D)) return fail(AX_ERR_UNSUPPORTED, "the gathering operator needs a GLL D");
    p.E = E;
    p.N = N;
    p.geom = geom;
    p.geo = geo;
    p.D = D;
    p.xi = xi;
    p.w = w;
    p.n_global = n_global;
    p.l2g = l2g;
    return AX_OK;
}

extern "C" int ax_local_gathered(int64_t E, int N, int geom, const double* geo, const double* D,
                                 const double* xi, const double* w, int nrhs, int prec, const int32_t* l2g,
                                 int64_t n_global, const void* Xg, void* Y, void* stream)
{
    clear_error();
    ax_problem p;
    AX_TRY(gathered_problem(E, N, geom, geo, D, xi, w, nrhs, prec, l2g, n_global, Xg, Y, p));
    if (p.E == 0) return AX_OK;
    return ax_local_gather(p, nrhs, prec, Xg, n_global, Y, as_stream(stream));
}

// energy = sum of parts[0, n) in a fixed order (one work-group)
__global__ void __launch_bounds__(256)
sum_parts_kernel(const double* __restrict__ parts, int64_t n, double* __restrict__ energy)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t q = threadIdx.x; q < n; q += 256) s += parts[q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *energy = red[0];
}

extern "C" int ax_local_gathered_energy(int64_t E, int N, int geom, const double* geo, const double* D,
                                        const double* xi, const double* w, const int32_t* l2g, int64_t n_global,
                                        const float* Xg, float* Y, double* work, double* energy, void* stream)
{
    clear_error();
    ax_problem p;
    AX_TRY(gathered_problem(E, N, geom, geo, D, xi, w, 1, AX_FP32, l2g, n_global, Xg, Y, p));
    if (!energy || (E > 0 && !work)) return fail(AX_ERR_ARG, "work or energy is NULL");
    hipStream_t st = as_stream(stream);
    FusedOut fo{work, E, 0};
    if (p.E > 0) AX_TRY(ax_local_gather_fused(p, Xg, n_global, Y, &fo, st));
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, st, work, fo.nparts, energy);
    return hip_check(hipGetLastError(), "energy sum");
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
        return axl_dispatch_f64(GEO_STORED, N, E, nrhs, nullptr, (const double*)G, (const double*)X, (double*)Y, D, nullptr, nullptr, st, nullptr, 0, NPL(N), E * NPL(N));
    if (prec == AX_FP32)
        return axl_dispatch_f32(GEO_STORED, N, E, nrhs, nullptr, (const float*)G, (const float*)X, (float*)Y, D, nullptr, nullptr, st, nullptr, 0, NPL(N), E * NPL(N));
    return ax_local_f16(E, N, GEO_STORED, nullptr, (const float*)G, D, nullptr, nullptr, nrhs, (const float*)X, (float*)Y, st);
}

extern "C" int ax_local_partial(int64_t E, int N, const double* verts, const void* lam, const double* D,
                                const double* xi, const double* w, int nrhs, int prec, const void* X, void* Y,
                                void* stream)
{
    clear_error();
    AX_TRY(check_common(E, N, nrhs, prec, X, Y, D));
    if (prec == AX_FP16_ACC32) return fail(AX_ERR_UNSUPPORTED, "partial recomputation is FP64 or FP32");
    if (!xi || !w) return fail(AX_ERR_ARG, "xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!verts || !lam) return fail(AX_ERR_ARG, "verts or lam is NULL");
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        return axl_dispatch_f64(GEO_TRIL, N, E, nrhs, verts, (const double*)lam, (const double*)X, (double*)Y, D,
                                xi, w, st, nullptr, 0, NPL(N), E * NPL(N));
    return axl_dispatch_f32(GEO_TRIL, N, E, nrhs, verts, (const float*)lam, (const float*)X, (float*)Y, D, xi, w,
                            st, nullptr, 0, NPL(N), E * NPL(N));
}

extern "C" int ax_local_helmholtz(int64_t E, int N, const double* verts, const void* L23, const double* D,
                                  const double* xi, const double* w, int nrhs, int prec, const void* X, void* Y,
                                  void* stream)
{
    clear_error();
    AX_TRY(check_common(E, N, nrhs, prec, X, Y, D));
    if (prec == AX_FP16_ACC32) return fail(AX_ERR_UNSUPPORTED, "the Helmholtz operator is FP64 or FP32");
    if (!xi || !w) return fail(AX_ERR_ARG, "xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!verts || !L23) return fail(AX_ERR_ARG, "verts or L23 is NULL");
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        return axl_dispatch_f64(GEO_HELM, N, E, nrhs, verts, (const double*)L23, (const double*)X, (double*)Y, D,
                                xi, w, st, nullptr, 0, NPL(N), E * NPL(N));
    return axl_dispatch_f32(GEO_HELM, N, E, nrhs, verts, (const float*)L23, (const float*)X, (float*)Y, D, xi, w,
                            st, nullptr, 0, NPL(N), E * NPL(N));
}

extern "C" int ax_local_vector(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                               const double* w, int prec, const void* X, void* Y, void* stream)
{
    clear_error();
    AX_TRY(check_common(E, N, 3, prec, X, Y, D));
    if (prec == AX_FP16_ACC32) return fail(AX_ERR_UNSUPPORTED, "the vector-field operator is FP64 or FP32");
    if (geom != AX_TRILINEAR && geom != AX_PARALLELEPIPED)
        return fail(AX_ERR_UNSUPPORTED, "unknown geometry %d", geom);
    if (!w) return fail(AX_ERR_ARG, "w is NULL");
    if (geom == AX_TRILINEAR && !xi) return fail(AX_ERR_ARG, "xi is NULL (needed for trilinear)");
    if (E == 0) return AX_OK;
    if (!geo) return fail(AX_ERR_ARG, "geo is NULL");
    hipStream_t st = as_stream(stream);
    const int gk = geom == AX_TRILINEAR ? GEO_TRI : GEO_PARA;
    const int64_t np = NPL(N);
    // three components per element, contiguous: element stride 3 N1^3, component stride N1^3
    if (prec == AX_FP64)
        return axl_dispatch_f64(gk, N, E, 3, geo, nullptr, (const double*)X, (double*)Y, D, xi, w, st, nullptr, 0,
                                3 * np, np);
    return axl_dispatch_f32(gk, N, E, 3, geo, nullptr, (const float*)X, (float*)Y, D, xi, w, st, nullptr, 0, 3 * np,
                            np);
}
