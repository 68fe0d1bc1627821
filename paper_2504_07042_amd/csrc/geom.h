// Device-side geometry of trilinear and parallelepiped hexahedra (internal header).
//
// Trilinear map (Eq. 8): x(r,s,t) = sum_v sigma_v(r,s,t) V_v with vertex v = a + 2b + 4c at
// reference corner (2a-1, 2b-1, 2c-1).  We work with 8J, the Jacobian of Eq. (9) without its
// factor 1/8, exactly as Algorithm 2 does; its three columns are
//   col0(s,t) = (A + B) + t (B - A),  A = (1-s) d00 + (1+s) d10,  B = (1-s) d01 + (1+s) d11
//   col1(r,t) = (A' + B') + t (B' - A'), A' = (1-r) e00 + (1+r) e10, B' = (1-r) e01 + (1+r) e11
//   col2(r,s) = (1-s)((1-r) f00 + (1+r) f10) + (1+s)((1-r) f01 + (1+r) f11)
// with the element's edge vectors d (along r), e (along s), f (along t).  These are the common
// terms E0, E1, F0, F1 and the k-invariant third column of Sec. 3.3 (Eq. 10-11).
//
// Going one step further than Algorithm 2, a GPU lane that owns the node column (i, j, :) sees
// col0 and col1 as affine functions of t = xi_k and col2 as a constant, so every entry of
// K = (8J)^T (8J) and det(8J) is a polynomial of degree <= 2 in t whose coefficients depend
// on (i, j) only.  The lane forms those 17 coefficients once per element and then evaluates
// each node's K and det(8J) with 10 fused multiply-adds instead of the 30 products and sums of
// forming J, K and det J from scratch.  The factors then follow Eq. (12):
//   G = w_i w_j w_k det(J) J^{-1} J^{-T} = lambda * adj(K),  lambda = 0.125 w_i w_j w_k / det(8J).
#pragma once

#include <hip/hip_runtime.h>

namespace ax {

// Per-column coefficients, formed in double; kernels that evaluate the factors in float keep a
// float copy (TriCoefT<float>): each coefficient is rounded to float once instead of at every use,
// with the same values.
template <typename C>
struct TriCoefT {
    C q0, q1, q2;  // K00(t) = |col0|^2
    C p0, p1, p2;  // K11(t) = |col1|^2
    C k22;         // K22    = |col2|^2
    C m0, m1, m2;  // K01(t) = col0 . col1
    C n0, n1;      // K02(t) = col0 . col2
    C o0, o1;      // K12(t) = col1 . col2
    C d0, d1, d2;  // det(8J)(t) = col0 . (col1 x col2)
    C cw;          // 0.125 w_i w_j
};
using TriCoef = TriCoefT<double>;

template <typename C>
__device__ __forceinline__ void tri_narrow(const TriCoef& k, TriCoefT<C>& o)
{
    o.q0 = C(k.q0); o.q1 = C(k.q1); o.q2 = C(k.q2);
    o.p0 = C(k.p0); o.p1 = C(k.p1); o.p2 = C(k.p2);
    o.k22 = C(k.k22);
    o.m0 = C(k.m0); o.m1 = C(k.m1); o.m2 = C(k.m2);
    o.n0 = C(k.n0); o.n1 = C(k.n1);
    o.o0 = C(k.o0); o.o1 = C(k.o1);
    o.d0 = C(k.d0); o.d1 = C(k.d1); o.d2 = C(k.d2);
    o.cw = C(k.cw);
}

__device__ __forceinline__ double dot3(const double* a, const double* b)
{
    return fma(a[0], b[0], fma(a[1], b[1], a[2] * b[2]));
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c)
{
    c[0] = fma(a[1], b[2], -a[2] * b[1]);
    c[1] = fma(a[2], b[0], -a[0] * b[2]);
    c[2] = fma(a[0], b[1], -a[1] * b[0]);
}

// Columns of 8J for the node column (r, s, :): col0 = a + t b, col1 = c + t d, col2 = u.
// V(v, q) returns coordinate q of vertex v; it is called one coordinate at a time so that only
// eight vertex words need to be live at once.
template <typename VF>
__device__ __forceinline__ void tri_columns(VF V, double r, double s, double* a, double* b, double* c,
                                            double* d, double* u)
{
    const double r0 = 1.0 - r, r1 = 1.0 + r, s0 = 1.0 - s, s1 = 1.0 + s;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double v0 = V(0, q), v1 = V(1, q), v2 = V(2, q), v3 = V(3, q);
        const double v4 = V(4, q), v5 = V(5, q), v6 = V(6, q), v7 = V(7, q);
        const double d00 = v1 - v0, d10 = v3 - v2, d01 = v5 - v4, d11 = v7 - v6;   // along r
        const double A = s0 * d00 + s1 * d10, B = s0 * d01 + s1 * d11;
        a[q] = A + B;
        b[q] = B - A;
        const double e00 = v2 - v0, e10 = v3 - v1, e01 = v6 - v4, e11 = v7 - v5;   // along s
        const double A2 = r0 * e00 + r1 * e10, B2 = r0 * e01 + r1 * e11;
        c[q] = A2 + B2;
        d[q] = B2 - A2;
        const double f00 = v4 - v0, f10 = v5 - v1, f01 = v6 - v2, f11 = v7 - v3;   // along t
        u[q] = s0 * (r0 * f00 + r1 * f10) + s1 * (r0 * f01 + r1 * f11);
    }
}

template <typename VF>
__device__ __forceinline__ void tri_prelude(VF V, double r, double s, double wi, double wj, TriCoef& k)
{
    double a[3], b[3], c[3], d[3], u[3];
    tri_columns(V, r, s, a, b, c, d, u);
    k.q0 = dot3(a, a);
    k.q1 = 2.0 * dot3(a, b);
    k.q2 = dot3(b, b);
    k.p0 = dot3(c, c);
    k.p1 = 2.0 * dot3(c, d);
    k.p2 = dot3(d, d);
    k.k22 = dot3(u, u);
    k.m0 = dot3(a, c);
    k.m1 = dot3(a, d) + dot3(b, c);
    k.m2 = dot3(b, d);
    k.n0 = dot3(a, u);
    k.n1 = dot3(b, u);
    k.o0 = dot3(c, u);
    k.o1 = dot3(d, u);
    double cu[3], du[3];
    cross3(c, u, cu);
    cross3(d, u, du);
    k.d0 = dot3(a, cu);
    k.d1 = dot3(a, du) + dot3(b, cu);
    k.d2 = dot3(b, du);
    k.cw = 0.125 * wi * wj;
}

// Newton-Raphson steps applied to the hardware reciprocal estimate in FP64.
#ifndef AX_RCP_NR
#define AX_RCP_NR 1
#endif

// 1/x: the hardware reciprocal estimate refined by Newton-Raphson steps
// r <- r + r (1 - x r), each of which squares the relative error.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int q = 0; q < AX_RCP_NR; ++q) r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

__device__ __forceinline__ float recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Unscaled factors at node t = xi_k without the Jacobian determinant: g[6] = adj(K).  The
// partial-recomputation variant (Sec. 4.2.2, Table 3) reads lam per node from memory instead.
template <typename R, typename C>
__device__ __forceinline__ void tri_adj_k(const TriCoefT<C>& k, R t, R* g)
{
    const R K00 = fma(fma(R(k.q2), t, R(k.q1)), t, R(k.q0));
    const R K11 = fma(fma(R(k.p2), t, R(k.p1)), t, R(k.p0));
    const R K22 = R(k.k22);
    const R K01 = fma(fma(R(k.m2), t, R(k.m1)), t, R(k.m0));
    const R K02 = fma(R(k.n1), t, R(k.n0));
    const R K12 = fma(R(k.o1), t, R(k.o0));
    g[0] = fma(K11, K22, -K12 * K12);
    g[1] = fma(K02, K12, -K01 * K22);
    g[2] = fma(K01, K12, -K02 * K11);
    g[3] = fma(K00, K22, -K02 * K02);
    g[4] = fma(K01, K02, -K00 * K12);
    g[5] = fma(K00, K11, -K01 * K01);
}

// Unscaled factors at node t = xi_k: g[6] = adj(K) and lam = 0.125 w_i w_j w_k / det(8J), so
// that the geometric factors of Eq. (7) are lam * g (Eq. 12).
template <typename R, typename C>
__device__ __forceinline__ void tri_adj(const TriCoefT<C>& k, R t, R wk, R* g, R& lam)
{
    const R det = fma(fma(R(k.d2), t, R(k.d1)), t, R(k.d0));
    lam = R(k.cw) * wk * recip(det);
    tri_adj_k(k, t, g);
}

// det(8J) at node t (for the lumped mass w det J = w det(8J) / 512).
__device__ __forceinline__ double tri_det(const TriCoef& k, double t)
{
    return fma(fma(k.d2, t, k.d1), t, k.d0);
}

}  // namespace ax
