// Set-up kernels: stored geometric factors (Eq. 7) of trilinear elements, the constant factors h
// of parallelepipeds (input of Algorithm 3), physical node coordinates (Eq. 8), element diagonals
// and the mesh validity check (det J > 0 at every GLL node).
#include <cstring>

#include "ax_internal.h"
#include "geom.h"

namespace ax {

struct Nodes {
    double xi[kMaxN1];
    double w[kMaxN1];
};

// One thread per node.  Same per-column invariants as the fused kernel (geom.h).
template <typename T>
__global__ void __launch_bounds__(256)
geom_factors_kernel(int64_t E, int N1, const double* __restrict__ verts, T* __restrict__ G,
                    double* __restrict__ gwj, const Nodes nd)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * NP) return;
    const int64_t e = idx / NP;
    const int l = (int)(idx - e * NP);
    const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
    const double* Ve = verts + e * 24;
    TriCoef tc;
    tri_prelude([&](int v, int q) { return Ve[v * 3 + q]; }, nd.xi[i], nd.xi[j], nd.w[i], nd.w[j], tc);
    double g[6], lam;
    tri_adj<double>(tc, nd.xi[k], nd.w[k], g, lam);
    if (G) {
        T* ge = G + e * 6 * NP + l;
        for (int q = 0; q < 6; ++q) ge[q * NP] = T(lam * g[q]);
    }
    if (gwj) gwj[idx] = nd.w[i] * nd.w[j] * nd.w[k] * tri_det(tc, nd.xi[k]) * (1.0 / 512.0);
}

// The per-node scale of the partial recomputation (Sec. 4.2.2): lam = 0.125 w_i w_j w_k / det(8J),
// the factor that turns adj(K) into the geometric factors (Eq. 12).  One thread per node.
template <typename T>
__global__ void __launch_bounds__(256)
geom_lambda_kernel(int64_t E, int N1, const double* __restrict__ verts, T* __restrict__ lam, const Nodes nd)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * NP) return;
    const int64_t e = idx / NP;
    const int l = (int)(idx - e * NP);
    const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
    const double* Ve = verts + e * 24;
    TriCoef tc;
    tri_prelude([&](int v, int q) { return Ve[v * 3 + q]; }, nd.xi[i], nd.xi[j], nd.w[i], nd.w[j], tc);
    double g[6], lm;
    tri_adj<double>(tc, nd.xi[k], nd.w[k], g, lm);
    lam[idx] = T(lm);
}

// Merged scalar factors of the Helmholtz operator (Sec. 4.2.1): L23[e][0][node] = lam lambda0,
// L23[e][1][node] = gwj lambda1 with lam = 0.125 w_i w_j w_k / det(8J) and gwj = w_i w_j w_k det J.
template <typename T>
__global__ void __launch_bounds__(256)
helmholtz_factors_kernel(int64_t E, int N1, const double* __restrict__ verts, const double* __restrict__ lambda0,
                         const double* __restrict__ lambda1, T* __restrict__ L23, const Nodes nd)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * NP) return;
    const int64_t e = idx / NP;
    const int l = (int)(idx - e * NP);
    const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
    const double* Ve = verts + e * 24;
    TriCoef tc;
    tri_prelude([&](int v, int q) { return Ve[v * 3 + q]; }, nd.xi[i], nd.xi[j], nd.w[i], nd.w[j], tc);
    double g[6], lm;
    tri_adj<double>(tc, nd.xi[k], nd.w[k], g, lm);
    const double gwj = nd.w[i] * nd.w[j] * nd.w[k] * tri_det(tc, nd.xi[k]) * (1.0 / 512.0);
    L23[(e * 2) * NP + l] = T(lm * lambda0[idx]);
    L23[(e * 2 + 1) * NP + l] = T(gwj * lambda1[idx]);
}

// h = det J J^-1 J^-T = adj(J^T J) / det J with J = 1/2 [v1 - v0, v2 - v0, v4 - v0] (columns).
__global__ void __launch_bounds__(256)
parallelepiped_kernel(int64_t E, const double* __restrict__ verts, double* __restrict__ h)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    const double* V = verts + e * 24;
    double c0[3], c1[3], c2[3];
    for (int q = 0; q < 3; ++q) {
        c0[q] = 0.5 * (V[3 + q] - V[q]);
        c1[q] = 0.5 * (V[6 + q] - V[q]);
        c2[q] = 0.5 * (V[12 + q] - V[q]);
    }
    const double K00 = dot3(c0, c0), K11 = dot3(c1, c1), K22 = dot3(c2, c2);
    const double K01 = dot3(c0, c1), K02 = dot3(c0, c2), K12 = dot3(c1, c2);
    double x12[3];
    cross3(c1, c2, x12);
    const double det = dot3(c0, x12);
    const double id = 1.0 / det;
    double* he = h + e * 6;
    he[0] = (K11 * K22 - K12 * K12) * id;
    he[1] = (K02 * K12 - K01 * K22) * id;
    he[2] = (K01 * K12 - K02 * K11) * id;
    he[3] = (K00 * K22 - K02 * K02) * id;
    he[4] = (K01 * K02 - K00 * K12) * id;
    he[5] = (K00 * K11 - K01 * K01) * id;
}

// x = sum_v sigma_v(xi_i, xi_j, xi_k) V_v, one thread per node, output [E][3][N1^3].
__global__ void __launch_bounds__(256)
node_coords_kernel(int64_t E, int N1, const double* __restrict__ verts, double* __restrict__ XYZ,
                   const Nodes nd)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * NP) return;
    const int64_t e = idx / NP;
    const int l = (int)(idx - e * NP);
    const double r = nd.xi[l % N1], s = nd.xi[(l / N1) % N1], t = nd.xi[l / (N1 * N1)];
    const double* V = verts + e * 24;
    const double fr[2] = {0.5 * (1.0 - r), 0.5 * (1.0 + r)};
    const double fs[2] = {0.5 * (1.0 - s), 0.5 * (1.0 + s)};
    const double ft[2] = {0.5 * (1.0 - t), 0.5 * (1.0 + t)};
    for (int q = 0; q < 3; ++q) {
        double x = 0.0;
        for (int v = 0; v < 8; ++v) x += fr[v & 1] * fs[(v >> 1) & 1] * ft[v >> 2] * V[v * 3 + q];
        XYZ[(e * 3 + q) * NP + l] = x;
    }
}

// Tables of the diagonal kernel: the differentiation matrix and the nodes.
struct DiagTables {
    double D[kMaxN1 * kMaxN1];
    Nodes nd;
};

// Diagonal of the element matrix D^T G D of Eq. (3) at node q = (i, j, k), one thread per node.
// With the gradient blocks of Table 1, (D_a e_q) is nonzero only on the GLL line through q in
// direction a, so the diagonal is
//   sum_a sum_n G_aa(q with index a set to n) D[n][q_a]^2 + sum_{a != b} G_ab(q) D[q_a][q_a] D[q_b][q_b].
// Trilinear: the factors at the 3 N1 line nodes are recomputed from the vertices (Eq. 12 via the
// per-column polynomials); parallelepiped: G = w_i w_j w_k h.
template <bool TRI>
__global__ void __launch_bounds__(256)
local_diag_kernel(int64_t E, int N1, const double* __restrict__ geo, double* __restrict__ out, const DiagTables tb)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= E * NP) return;
    const int64_t e = idx / NP;
    const int l = (int)(idx - e * NP);
    const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
    const int q[3] = {i, j, k};
    const Nodes& nd = tb.nd;
    auto Dm = [&](int a, int b) { return tb.D[a * N1 + b]; };
    // factors at node (a, b, c): g[6] in order 00, 01, 02, 11, 12, 22
    auto factors = [&](int a, int b, int c, double* g) {
        if constexpr (TRI) {
            const double* Ve = geo + e * 24;
            TriCoef tc;
            tri_prelude([&](int v, int qq) { return Ve[v * 3 + qq]; }, nd.xi[a], nd.xi[b], nd.w[a], nd.w[b], tc);
            double lam;
            tri_adj<double>(tc, nd.xi[c], nd.w[c], g, lam);
            for (int m = 0; m < 6; ++m) g[m] *= lam;
        } else {
            const double W = nd.w[a] * nd.w[b] * nd.w[c];
            for (int m = 0; m < 6; ++m) g[m] = W * geo[e * 6 + m];
        }
    };
    double acc = 0.0, g[6];
    for (int n = 0; n < N1; ++n) {
        factors(n, j, k, g);
        acc += g[0] * Dm(n, i) * Dm(n, i);
        factors(i, n, k, g);
        acc += g[3] * Dm(n, j) * Dm(n, j);
        factors(i, j, n, g);
        acc += g[5] * Dm(n, k) * Dm(n, k);
    }
    factors(i, j, k, g);
    const double di = Dm(q[0], q[0]), dj = Dm(q[1], q[1]), dk = Dm(q[2], q[2]);
    acc += 2.0 * (g[1] * di * dj + g[2] * di * dk + g[4] * dj * dk);
    out[idx] = acc;
}

// Mesh validity (Eq. 8-9): det J of the trilinear map at every GLL node of every element.  The
// factors of Eq. (7) divide by det J, so an element with det J <= 0 at a node is inverted or
// collapsed there and the operator is undefined.  One thread per node; each wave reduces the
// smallest det and the lowest failing element index, and one lane per wave merges them into
// res[0] (min element index whose det is <= 0 or not finite, ~0 if none) and res[1] (the
// order-preserving key of the smallest finite det(8J)).
__device__ __forceinline__ unsigned long long det_key(double d)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void __launch_bounds__(256)
check_mesh_kernel(int64_t E, int N1, const double* __restrict__ verts, unsigned long long* __restrict__ res,
                  const Nodes nd)
{
    const int NP = N1 * N1 * N1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dmin = __builtin_inf();
    unsigned long long bad = ~0ull;
    if (idx < E * NP) {
        const int64_t e = idx / NP;
        const int l = (int)(idx - e * NP);
        const int i = l % N1, j = (l / N1) % N1, k = l / (N1 * N1);
        const double* Ve = verts + e * 24;
        TriCoef tc;
        tri_prelude([&](int v, int q) { return Ve[v * 3 + q]; }, nd.xi[i], nd.xi[j], 1.0, 1.0, tc);
        const double det = tri_det(tc, nd.xi[k]);
        if (!(det > 0.0) || !(det < __builtin_inf())) bad = (unsigned long long)e;
        if (det == det) dmin = det;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        dmin = fmin(dmin, __shfl_xor(dmin, off));
        const unsigned long long o = __shfl_xor(bad, off);
        bad = o < bad ? o : bad;
    }
    if ((threadIdx.x & 63) == 0) {
        if (bad != ~0ull) atomicMin(&res[0], bad);
        atomicMin(&res[1], det_key(dmin));
    }
}

static void fill_nodes(Nodes& nd, int N1, const double* xi, const double* w)
{
    for (int q = 0; q < kMaxN1; ++q) {
        nd.xi[q] = (xi && q < N1) ? xi[q] : 0.0;
        nd.w[q] = (w && q < N1) ? w[q] : 0.0;
    }
}

static unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace ax

using namespace ax;

extern "C" int ax_geom_factors(int64_t E, int N, const double* verts, const double* xi,
                               const double* w, int prec, void* G, double* gwj, void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "prec must be FP64 or FP32");
    if (!xi || !w) return fail(AX_ERR_ARG, "xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!verts) return fail(AX_ERR_ARG, "verts is NULL");
    if (!G && !gwj) return AX_OK;
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    if (grid_for(n, 256) == 0 || n / 256 > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many nodes");
    Nodes nd;
    fill_nodes(nd, N1, xi, w);
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        hipLaunchKernelGGL(geom_factors_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1,
                           verts, (double*)G, gwj, nd);
    else
        hipLaunchKernelGGL(geom_factors_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1,
                           verts, (float*)G, gwj, nd);
    return hip_check(hipGetLastError(), "ax_geom_factors launch");
}

extern "C" int ax_geom_lambda(int64_t E, int N, const double* verts, const double* xi, const double* w, int prec,
                              void* lam, void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "prec must be FP64 or FP32");
    if (!xi || !w) return fail(AX_ERR_ARG, "xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!verts || !lam) return fail(AX_ERR_ARG, "verts or lam is NULL");
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    if (n / 256 > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many nodes");
    Nodes nd;
    fill_nodes(nd, N1, xi, w);
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        hipLaunchKernelGGL(geom_lambda_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, verts,
                           (double*)lam, nd);
    else
        hipLaunchKernelGGL(geom_lambda_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, verts,
                           (float*)lam, nd);
    return hip_check(hipGetLastError(), "ax_geom_lambda launch");
}

extern "C" int ax_helmholtz_factors(int64_t E, int N, const double* verts, const double* xi, const double* w,
                                    const double* lambda0, const double* lambda1, int prec, void* L23, void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_UNSUPPORTED, "prec must be FP64 or FP32");
    if (!xi || !w) return fail(AX_ERR_ARG, "xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!verts || !lambda0 || !lambda1 || !L23) return fail(AX_ERR_ARG, "NULL array");
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    if (n / 256 > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many nodes");
    Nodes nd;
    fill_nodes(nd, N1, xi, w);
    hipStream_t st = as_stream(stream);
    if (prec == AX_FP64)
        hipLaunchKernelGGL(helmholtz_factors_kernel<double>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, verts,
                           lambda0, lambda1, (double*)L23, nd);
    else
        hipLaunchKernelGGL(helmholtz_factors_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, verts,
                           lambda0, lambda1, (float*)L23, nd);
    return hip_check(hipGetLastError(), "ax_helmholtz_factors launch");
}

extern "C" int ax_parallelepiped_factors(int64_t E, const double* verts, double* h, void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (E == 0) return AX_OK;
    if (!verts || !h) return fail(AX_ERR_ARG, "NULL pointer");
    hipLaunchKernelGGL(parallelepiped_kernel, dim3(grid_for(E, 256)), dim3(256), 0, as_stream(stream),
                       E, verts, h);
    return hip_check(hipGetLastError(), "ax_parallelepiped_factors launch");
}

extern "C" int ax_node_coords(int64_t E, int N, const double* verts, const double* xi, double* XYZ,
                              void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (!xi) return fail(AX_ERR_ARG, "xi is NULL");
    if (E == 0) return AX_OK;
    if (!verts || !XYZ) return fail(AX_ERR_ARG, "NULL pointer");
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    Nodes nd;
    fill_nodes(nd, N1, xi, nullptr);
    hipLaunchKernelGGL(node_coords_kernel, dim3(grid_for(n, 256)), dim3(256), 0, as_stream(stream), E,
                       N1, verts, XYZ, nd);
    return hip_check(hipGetLastError(), "ax_node_coords launch");
}

extern "C" int ax_local_diag(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                             const double* w, double* out, void* stream)
{
    clear_error();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (geom != AX_TRILINEAR && geom != AX_PARALLELEPIPED) return fail(AX_ERR_UNSUPPORTED, "unknown geometry %d", geom);
    if (!D || !w || (geom == AX_TRILINEAR && !xi)) return fail(AX_ERR_ARG, "D, xi or w is NULL");
    if (E == 0) return AX_OK;
    if (!geo || !out) return fail(AX_ERR_ARG, "geo or out is NULL");
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    if (n / 256 > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many nodes");
    DiagTables tb;
    for (int q = 0; q < kMaxN1 * kMaxN1; ++q) tb.D[q] = q < N1 * N1 ? D[q] : 0.0;
    fill_nodes(tb.nd, N1, xi, w);
    hipStream_t st = as_stream(stream);
    if (geom == AX_TRILINEAR)
        hipLaunchKernelGGL(local_diag_kernel<true>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, geo, out, tb);
    else
        hipLaunchKernelGGL(local_diag_kernel<false>, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, geo, out, tb);
    return hip_check(hipGetLastError(), "ax_local_diag launch");
}

extern "C" int ax_check_mesh(int64_t E, int N, const double* verts, const double* xi, int64_t* bad_element,
                             double* min_det, void* stream)
{
    clear_error();
    if (bad_element) *bad_element = -1;
    if (min_det) *min_det = __builtin_inf();
    if (E < 0) return fail(AX_ERR_ARG, "E < 0");
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (!xi) return fail(AX_ERR_ARG, "xi is NULL");
    if (E == 0) return AX_OK;
    if (!verts) return fail(AX_ERR_ARG, "verts is NULL");
    const int N1 = N + 1;
    const int64_t n = E * N1 * N1 * N1;
    if (n / 256 > 0x7fffffff) return fail(AX_ERR_UNSUPPORTED, "too many nodes");
    Nodes nd;
    fill_nodes(nd, N1, xi, nullptr);
    hipStream_t st = as_stream(stream);
    unsigned long long* res = nullptr;
    if (hipMalloc((void**)&res, 2 * sizeof(unsigned long long)) != hipSuccess)
        return fail(AX_ERR_HIP, "ax_check_mesh: hipMalloc of 16 bytes failed");
    unsigned long long h[2] = {~0ull, ~0ull};
    hipError_t err = hipMemcpyAsync(res, h, sizeof(h), hipMemcpyHostToDevice, st);
    if (err == hipSuccess) {
        hipLaunchKernelGGL(check_mesh_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, E, N1, verts, res, nd);
        err = hipGetLastError();
    }
    if (err == hipSuccess) err = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    (void)hipFree(res);
    if (err != hipSuccess) return hip_check(err, "ax_check_mesh");
    // decode the smallest finite det(8J) and scale to det J (exact: a power of two)
    double dm = __builtin_inf();
    if (h[1] != ~0ull) {
        const unsigned long long b = (h[1] >> 63) ? (h[1] & 0x7fffffffffffffffull) : ~h[1];
        std::memcpy(&dm, &b, sizeof(dm));
        dm *= 1.0 / 512.0;
    }
    if (min_det) *min_det = dm;
    if (h[0] != ~0ull) {
        if (bad_element) *bad_element = (int64_t)h[0];
        return fail(AX_ERR_ARG, "element %lld is inverted or degenerate: det J <= 0 or not finite at a GLL node "
                                "(smallest finite det J over the mesh %.6g)",
                    (long long)h[0], dm);
    }
    return AX_OK;
}
