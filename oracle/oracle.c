/*
 * CPU reference ("oracle") for the matrix-free element-local Poisson operator of
 * "Towards a Higher Roofline for Matrix-Vector Multiplication in Matrix-Free HOSFEM"
 * (arXiv 2504.07042).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, double-precision definition that
 * the HIP kernels are checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header, table or constant
 * with the HIP library and includes nothing from it.
 *
 * Every routine evaluates a definition from the paper directly:
 *   - GLL points, weights and the differentiation matrix: Sec. 2.1, Table 1.
 *   - Trilinear map and its Jacobian: Sec. 2.3 (shape functions), Sec. 3.3 Eq. (8)-(9),
 *     Sec. 3.2 Eq. (5)-(6).
 *   - Geometric factors: Sec. 3.2 Eq. (7), by an explicit 3x3 inverse (NOT the adjugate-of-K
 *     factoring of Sec. 3.3 Eq. (12); that is what the GPU does).
 *   - AxLocal: Sec. 2.2 Eq. (3) with Lambda0 = I, Lambda1 = 0 (Poisson): the gradient blocks
 *     D_r, D_s, D_t of Table 1 applied to the whole element, the factor block, then D^T.
 *   - Gather/scatter: Sec. 2.1 (the binary matrix Q) and Eq. (1).
 *
 * Readings where the paper is silent:
 *   - Diagonal of D: Table 1 defines D[i][j] = pi_j'(xi_i).  Off the diagonal this is
 *     L_N(xi_i) / (L_N(xi_j) (xi_i - xi_j)); on the diagonal we use minus the sum of the row's
 *     other entries, which is the same number in exact arithmetic (D applied to a constant is
 *     zero) and keeps D*1 = 0 to rounding.
 *   - Q^T sums the contributions to one global node in ascending local index order.
 *
 * Layouts: local vectors [nrhs][E][N1^3], node [i,j,k] at i + j*N1 + k*N1^2 (Sec. 2.2);
 * vertices [E][8][3] in tensor order v = a + 2b + 4c (Eq. 8); stored factors
 * [E][6][N1^3] in the order G00, G01, G02, G11, G12, G22 (Algorithm 1 inputs).
 *
 * Parity status: every function here is pinned by tests against values the paper prints, closed
 * forms, brute force or invariants (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXN 32

/* Legendre polynomial L_N and its first derivative at x.  Table 1 defines L_N by Rodrigues'
 * formula; the Bonnet recurrence (n+1) L_{n+1} = (2n+1) x L_n - n L_{n-1} generates the same
 * polynomials, and L_n' follows from (1 - x^2) L_n' = n (L_{n-1} - x L_n) away from x = +-1
 * (at the endpoints L_n'(+-1) = (+-1)^{n+1} n (n+1) / 2). */
void orc_legendre(int N, double x, double* L, double* dL)
{
    double p0 = 1.0, p1 = x;
    if (N == 0) { *L = 1.0; *dL = 0.0; return; }
    for (int n = 1; n < N; ++n) {
        double p2 = ((2.0 * n + 1.0) * x * p1 - n * p0) / (n + 1.0);
        p0 = p1;
        p1 = p2;
    }
    *L = p1;
    if (fabs(1.0 - x * x) < 1e-300 || x == 1.0 || x == -1.0) {
        double s = (x > 0.0) ? 1.0 : ((N % 2 == 0) ? -1.0 : 1.0);
        *dL = s * 0.5 * N * (N + 1.0);
    } else {
        *dL = N * (p0 - x * p1) / (1.0 - x * x);
    }
}

/* GLL points (zeros of (1 - x^2) L_N'(x)), weights w_i = 2 / (N (N+1) L_N(xi_i)^2) and the
 * differentiation matrix D[i][j] = pi_j'(xi_i), Table 1.  Interior points: Newton's method on
 * L_N' with L_N'' taken from Legendre's equation, started at -cos(pi i / N).
 * Returns 0, or -1 for N outside [1, ORC_MAXN]. */
int orc_gll(int N, double* xi, double* w, double* D)
{
    if (N < 1 || N > ORC_MAXN) return -1;
    const int N1 = N + 1;
    xi[0] = -1.0;
    xi[N] = 1.0;
    for (int i = 1; i < N; ++i) {
        double x = -cos(M_PI * i / N);
        for (int it = 0; it < 200; ++it) {
            double L, dL;
            orc_legendre(N, x, &L, &dL);
            double d2L = (2.0 * x * dL - N * (N + 1.0) * L) / (1.0 - x * x);
            double dx = dL / d2L;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        xi[i] = x;
    }
    /* the point set is symmetric about 0 */
    for (int i = 0; i < N1 / 2; ++i) {
        double a = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -a;
        xi[N - i] = a;
    }
    if (N1 % 2 == 1) xi[N / 2] = 0.0;
    double Lv[ORC_MAXN + 1];
    for (int i = 0; i < N1; ++i) {
        double L, dL;
        orc_legendre(N, xi[i], &L, &dL);
        Lv[i] = L;
        w[i] = 2.0 / (N * (N + 1.0) * L * L);
    }
    for (int i = 0; i < N1; ++i) {
        double rowsum = 0.0;
        for (int j = 0; j < N1; ++j) {
            if (i == j) continue;
            D[i * N1 + j] = Lv[i] / (Lv[j] * (xi[i] - xi[j]));
            rowsum += D[i * N1 + j];
        }
        D[i * N1 + i] = -rowsum;
    }
    return 0;
}

/* Trilinear shape function sigma_v and its gradient w.r.t. (r, s, t) for v = a + 2b + 4c:
 * sigma_v = 1/8 (1 + (2a-1) r)(1 + (2b-1) s)(1 + (2c-1) t)  (Sec. 2.3, Eq. 8). */
static void shape(int v, double r, double s, double t, double* sig, double grad[3])
{
    const double sa = (v & 1) ? 1.0 : -1.0;
    const double sb = (v & 2) ? 1.0 : -1.0;
    const double sc = (v & 4) ? 1.0 : -1.0;
    const double fr = 1.0 + sa * r, fs = 1.0 + sb * s, ft = 1.0 + sc * t;
    *sig = 0.125 * fr * fs * ft;
    grad[0] = 0.125 * sa * fs * ft;
    grad[1] = 0.125 * fr * sb * ft;
    grad[2] = 0.125 * fr * fs * sc;
}

/* Jacobian of the trilinear map at (r, s, t): J[c][d] = d x_c / d r_d (Eq. 5, Eq. 9),
 * evaluated directly as the sum over the 8 vertices. */
void orc_jacobian(const double* V /* [8][3] */, double r, double s, double t, double* J /* [3][3] */)
{
    for (int q = 0; q < 9; ++q) J[q] = 0.0;
    for (int v = 0; v < 8; ++v) {
        double sig, g[3];
        shape(v, r, s, t, &sig, g);
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) J[c * 3 + d] += g[d] * V[v * 3 + c];
    }
}

/* orc_jacobian at every GLL node of every element: J[E][N1^3][3][3], node l = i + j N1 + k N1^2. */
void orc_jacobians(int64_t E, int N, const double* verts, const double* xi, double* J)
{
    const int N1 = N + 1, Np = N1 * N1 * N1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e)
        for (int k = 0; k < N1; ++k)
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i)
                    orc_jacobian(verts + e * 24, xi[i], xi[j], xi[k],
                                 J + (e * Np + i + j * N1 + k * N1 * N1) * 9);
}

static double det3(const double* J)
{
    return J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) +
           J[2] * (J[3] * J[7] - J[4] * J[6]);
}

/* Inverse of a 3x3 matrix by cofactors.  Returns the determinant. */
static double inv3(const double* J, double* Ji)
{
    const double det = det3(J);
    Ji[0] = (J[4] * J[8] - J[5] * J[7]) / det;
    Ji[1] = (J[2] * J[7] - J[1] * J[8]) / det;
    Ji[2] = (J[1] * J[5] - J[2] * J[4]) / det;
    Ji[3] = (J[5] * J[6] - J[3] * J[8]) / det;
    Ji[4] = (J[0] * J[8] - J[2] * J[6]) / det;
    Ji[5] = (J[2] * J[3] - J[0] * J[5]) / det;
    Ji[6] = (J[3] * J[7] - J[4] * J[6]) / det;
    Ji[7] = (J[1] * J[6] - J[0] * J[7]) / det;
    Ji[8] = (J[0] * J[4] - J[1] * J[3]) / det;
    return det;
}

/* Geometric factors of Eq. (7) at every node of every element:
 *   G = w_i w_j w_k det(J) J^{-1} J^{-T}  (6 entries, order 00,01,02,11,12,22) -> G[E][6][N1^3]
 *   gwj = w_i w_j w_k det(J)                                                  -> gwj[E][N1^3]
 * with J = J^Phi(xi_i, xi_j, xi_k) from Eq. (9).  Either output may be NULL.
 * min_det (may be NULL) receives the smallest det(J) over all nodes. */
void orc_geom_factors(int64_t E, int N, const double* verts, const double* xi, const double* w,
                      double* G, double* gwj, double* min_det)
{
    const int N1 = N + 1, Np = N1 * N1 * N1;
    double mind = INFINITY;
#pragma omp parallel for reduction(min : mind) schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double* V = verts + e * 24;
        for (int k = 0; k < N1; ++k)
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i) {
                    const int l = i + j * N1 + k * N1 * N1;
                    double J[9], Ji[9];
                    orc_jacobian(V, xi[i], xi[j], xi[k], J);
                    const double det = inv3(J, Ji);
                    if (det < mind) mind = det;
                    const double W = w[i] * w[j] * w[k];
                    double M[9];
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            double acc = 0.0;
                            for (int c = 0; c < 3; ++c) acc += Ji[a * 3 + c] * Ji[b * 3 + c];
                            M[a * 3 + b] = W * det * acc;
                        }
                    if (G) {
                        double* g = G + e * 6 * Np;
                        g[0 * Np + l] = M[0];
                        g[1 * Np + l] = M[1];
                        g[2 * Np + l] = M[2];
                        g[3 * Np + l] = M[4];
                        g[4 * Np + l] = M[5];
                        g[5 * Np + l] = M[8];
                    }
                    if (gwj) gwj[e * Np + l] = W * det;
                }
    }
    if (min_det) *min_det = mind;
}

/* Physical node coordinates x_e,ijk = sum_v sigma_v(xi_i, xi_j, xi_k) V_v  (Eq. 8).
 * Output [E][3][N1^3]. */
void orc_node_coords(int64_t E, int N, const double* verts, const double* xi, double* XYZ)
{
    const int N1 = N + 1, Np = N1 * N1 * N1;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double* V = verts + e * 24;
        for (int k = 0; k < N1; ++k)
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i) {
                    const int l = i + j * N1 + k * N1 * N1;
                    double x[3] = {0.0, 0.0, 0.0};
                    for (int v = 0; v < 8; ++v) {
                        double sig, g[3];
                        shape(v, xi[i], xi[j], xi[k], &sig, g);
                        for (int c = 0; c < 3; ++c) x[c] += sig * V[v * 3 + c];
                    }
                    for (int c = 0; c < 3; ++c) XYZ[(e * 3 + c) * Np + l] = x[c];
                }
    }
}

/* Parallelepiped factors without weights, h = det(J) J^{-1} J^{-T} (order 00,01,02,11,12,22)
 * from the Jacobian of Eq. (9) evaluated at the element centre (it is constant for an affine
 * element), the input of Algorithm 3.  Output h[E][6]. */
void orc_parallelepiped_h(int64_t E, const double* verts, double* h)
{
    for (int64_t e = 0; e < E; ++e) {
        double J[9], Ji[9];
        orc_jacobian(verts + e * 24, 0.0, 0.0, 0.0, J);
        const double det = inv3(J, Ji);
        double M[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += Ji[a * 3 + c] * Ji[b * 3 + c];
                M[a * 3 + b] = det * acc;
            }
        h[e * 6 + 0] = M[0];
        h[e * 6 + 1] = M[1];
        h[e * 6 + 2] = M[2];
        h[e * 6 + 3] = M[4];
        h[e * 6 + 4] = M[5];
        h[e * 6 + 5] = M[8];
    }
}

/* One block of the discrete gradient of Table 1 applied to a whole element vector:
 *   dir 0: D_r = I (x) I (x) Dh   (acts on the fastest index i of node [i,j,k]),
 *   dir 1: D_s = I (x) Dh (x) I   (acts on j),
 *   dir 2: D_t = Dh (x) I (x) I   (acts on k),
 * or its transpose (trans != 0), written out from the Kronecker definition:
 *   out[a, b, c] = sum_n M[.][n] in[...]  with M = Dh or Dh^T on the direction's index. */
static void grad_block(int N1, const double* Dh, int dir, int trans, const double* in, double* out)
{
    const int st[3] = {1, N1, N1 * N1};
    const int sd = st[dir];
    for (int k = 0; k < N1; ++k)
        for (int j = 0; j < N1; ++j)
            for (int i = 0; i < N1; ++i) {
                const int node[3] = {i, j, k};
                const int a = node[dir];
                const int base = i + j * N1 + k * N1 * N1 - a * sd;
                double acc = 0.0;
                for (int n = 0; n < N1; ++n) {
                    const double m = trans ? Dh[n * N1 + a] : Dh[a * N1 + n];
                    acc += m * in[base + n * sd];
                }
                out[i + j * N1 + k * N1 * N1] = acc;
            }
}

/* AxLocal, Poisson case of Sec. 2.2 Eq. (3) (Lambda0 = I, Lambda1 = 0):
 *   Y_e = D^T G_e D X_e,  D = [D_r; D_s; D_t] (Table 1),
 * evaluated in the order the equation is written, one column at a time:
 *   (1) the reference gradient u = D x: three whole-element vectors u_r, u_s, u_t;
 *   (2) the block of diagonal factor matrices, per node v = G u with the symmetric 3x3 matrix
 *       [[G00, G01, G02], [G01, G11, G12], [G02, G12, G22]];
 *   (3) y = D^T v = D_r^T v_r + D_s^T v_s + D_t^T v_t.
 * G [E][6][N1^3] (weights included, order 00,01,02,11,12,22), X, Y [nrhs][E][N1^3]. */
void orc_ax_local(int64_t E, int N, const double* D, const double* G, int nrhs, const double* X,
                  double* Y)
{
    const int N1 = N + 1, Np = N1 * N1 * N1;
#pragma omp parallel
    {
        double* u = (double*)malloc(sizeof(double) * 7 * Np);
        double* v = u + 3 * Np;
        double* tmp = v + 3 * Np;
#pragma omp for schedule(static)
        for (int64_t e = 0; e < E; ++e) {
            const double* g = G + e * 6 * Np;
            for (int c = 0; c < nrhs; ++c) {
                const double* x = X + ((int64_t)c * E + e) * Np;
                double* y = Y + ((int64_t)c * E + e) * Np;
                for (int d = 0; d < 3; ++d) grad_block(N1, D, d, 0, x, u + d * Np);
                for (int l = 0; l < Np; ++l) {
                    const double M[3][3] = {{g[0 * Np + l], g[1 * Np + l], g[2 * Np + l]},
                                            {g[1 * Np + l], g[3 * Np + l], g[4 * Np + l]},
                                            {g[2 * Np + l], g[4 * Np + l], g[5 * Np + l]}};
                    for (int a = 0; a < 3; ++a) {
                        double acc = 0.0;
                        for (int b = 0; b < 3; ++b) acc += M[a][b] * u[b * Np + l];
                        v[a * Np + l] = acc;
                    }
                }
                for (int l = 0; l < Np; ++l) y[l] = 0.0;
                for (int d = 0; d < 3; ++d) {
                    grad_block(N1, D, d, 1, v + d * Np, tmp);
                    for (int l = 0; l < Np; ++l) y[l] += tmp[l];
                }
            }
        }
        free(u);
    }
}

/* Diagonal of each element matrix A^(e) = D^T G D of Eq. (3) (Poisson), the Jacobi
 * preconditioner's ingredient.  With D = [D_r; D_s; D_t] (Table 1), (D_r e_q)[p] = Dh[p_i][q_i]
 * when p and q share j and k (zero otherwise), and likewise for D_s, D_t; so
 *   e_q^T D_a^T G_aa D_a e_q = sum_n G_aa[node q with its a-index set to n] Dh[n][q_a]^2,
 *   e_q^T D_a^T G_ab D_b e_q = G_ab[q] Dh[q_a][q_a] Dh[q_b][q_b]   (a != b: only p = q survives),
 * and the diagonal is the sum over a, b.  G [E][6][N1^3], out [E][N1^3]. */
void orc_ax_diag(int64_t E, int N, const double* D, const double* G, double* out)
{
    const int N1 = N + 1, Np = N1 * N1 * N1;
    const int st[3] = {1, N1, N1 * N1};
    const int gaa[3] = {0, 3, 5};                       /* G00, G11, G22 */
    const int gab[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < E; ++e) {
        const double* g = G + e * 6 * Np;
        for (int k = 0; k < N1; ++k)
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i) {
                    const int q[3] = {i, j, k};
                    const int l = i + j * N1 + k * N1 * N1;
                    double acc = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        const int base = l - q[a] * st[a];
                        for (int n = 0; n < N1; ++n) {
                            const double d = D[n * N1 + q[a]];
                            acc += g[gaa[a] * Np + base + n * st[a]] * d * d;
                        }
                        for (int b = 0; b < 3; ++b)
                            if (b != a)
                                acc += g[gab[a][b] * Np + l] * D[q[a] * N1 + q[a]] * D[q[b] * N1 + q[b]];
                    }
                    out[e * Np + l] = acc;
                }
    }
}

/* Q^T (Sec. 2.1, Eq. 1): out[g] = sum over local l with l2g[l] = g of in[l], summed in
 * ascending l.  Local [nrhs][n_local], global [nrhs][n_global]. */
void orc_gs_qt(int64_t n_local, int64_t n_global, const int32_t* l2g, int nrhs, const double* in,
               double* out)
{
    for (int c = 0; c < nrhs; ++c) {
        double* o = out + (int64_t)c * n_global;
        const double* x = in + (int64_t)c * n_local;
        for (int64_t g = 0; g < n_global; ++g) o[g] = 0.0;
        for (int64_t l = 0; l < n_local; ++l) o[l2g[l]] += x[l];
    }
}

/* Q: out[l] = in[l2g[l]]. */
void orc_gs_q(int64_t n_local, int64_t n_global, const int32_t* l2g, int nrhs, const double* in,
              double* out)
{
    for (int c = 0; c < nrhs; ++c)
        for (int64_t l = 0; l < n_local; ++l)
            out[(int64_t)c * n_local + l] = in[(int64_t)c * n_global + l2g[l]];
}

/* Assembled Poisson operator  y = mask o Q^T AxLocal(Q x)  on global vectors (Eq. 1 with
 * homogeneous Dirichlet rows zeroed).  mask may be NULL.  work: 2 * n_local doubles. */
void orc_apply_A(int64_t E, int N, const double* D, const double* G, int64_t n_global,
                 const int32_t* l2g, const uint8_t* mask, const double* x, double* y, double* work)
{
    const int N1 = N + 1;
    const int64_t n_local = E * N1 * N1 * N1;
    double* xl = work;
    double* yl = work + n_local;
    orc_gs_q(n_local, n_global, l2g, 1, x, xl);
    orc_ax_local(E, N, D, G, 1, xl, yl);
    orc_gs_qt(n_local, n_global, l2g, 1, yl, y);
    if (mask)
        for (int64_t g = 0; g < n_global; ++g)
            if (mask[g]) y[g] = 0.0;
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Unpreconditioned conjugate gradients on the assembled operator (the iterative solve of
 * Sec. 1 / Sec. 2.1; the paper does not fix the variant).  x holds x0 on entry.  Stops when
 * ||r||_2 / ||b||_2 <= rtol on the recursive residual.  Returns the iteration count, or -1 on
 * breakdown (p^T A p <= 0 or not finite).  rel_res receives the final TRUE relative residual
 * ||b - A x|| / ||b|| recomputed from x. */
int orc_cg(int64_t E, int N, const double* D, const double* G, int64_t n_global,
           const int32_t* l2g, const uint8_t* mask, const double* b, double* x, double rtol,
           int max_it, double* rel_res)
{
    const int N1 = N + 1;
    const int64_t n_local = E * N1 * N1 * N1;
    double* work = (double*)malloc(sizeof(double) * 2 * n_local);
    double* r = (double*)malloc(sizeof(double) * n_global);
    double* p = (double*)malloc(sizeof(double) * n_global);
    double* Ap = (double*)malloc(sizeof(double) * n_global);
    orc_apply_A(E, N, D, G, n_global, l2g, mask, x, Ap, work);
    for (int64_t g = 0; g < n_global; ++g) {
        r[g] = b[g] - Ap[g];
        p[g] = r[g];
    }
    const double bnorm = sqrt(dot(n_global, b, b));
    double rr = dot(n_global, r, r);
    int it = 0, status = isfinite(bnorm) ? 0 : -1;
    while (status == 0 && it < max_it && !(sqrt(rr) <= rtol * bnorm)) {
        orc_apply_A(E, N, D, G, n_global, l2g, mask, p, Ap, work);
        const double pAp = dot(n_global, p, Ap);
        if (!(pAp > 0.0) || !isfinite(pAp)) { status = -1; break; }
        const double alpha = rr / pAp;
        for (int64_t g = 0; g < n_global; ++g) {
            x[g] += alpha * p[g];
            r[g] -= alpha * Ap[g];
        }
        const double rr_new = dot(n_global, r, r);
        const double beta = rr_new / rr;
        for (int64_t g = 0; g < n_global; ++g) p[g] = r[g] + beta * p[g];
        rr = rr_new;
        ++it;
    }
    orc_apply_A(E, N, D, G, n_global, l2g, mask, x, Ap, work);
    for (int64_t g = 0; g < n_global; ++g) r[g] = b[g] - Ap[g];
    if (rel_res) *rel_res = sqrt(dot(n_global, r, r)) / bnorm;
    free(work);
    free(r);
    free(p);
    free(Ap);
    return status ? -1 : it;
}

/* Preconditioned conjugate gradients with the diagonal preconditioner M^-1 = diag(dinv) (the
 * textbook algorithm; the paper does not name the solver's preconditioner, the diagonal one is
 * the reading used for the Table 5-style runs).  Same stopping rule, return values and residual report as orc_cg. */
int orc_pcg(int64_t E, int N, const double* D, const double* G, int64_t n_global,
            const int32_t* l2g, const uint8_t* mask, const double* b, const double* dinv, double* x,
            double rtol, int max_it, double* rel_res)
{
    const int N1 = N + 1;
    const int64_t n_local = E * N1 * N1 * N1;
    double* work = (double*)malloc(sizeof(double) * 2 * n_local);
    double* r = (double*)malloc(sizeof(double) * n_global);
    double* z = (double*)malloc(sizeof(double) * n_global);
    double* p = (double*)malloc(sizeof(double) * n_global);
    double* Ap = (double*)malloc(sizeof(double) * n_global);
    orc_apply_A(E, N, D, G, n_global, l2g, mask, x, Ap, work);
    for (int64_t g = 0; g < n_global; ++g) {
        r[g] = b[g] - Ap[g];
        z[g] = dinv[g] * r[g];
        p[g] = z[g];
    }
    const double bnorm = sqrt(dot(n_global, b, b));
    double rr = dot(n_global, r, r), rz = dot(n_global, r, z);
    int it = 0, status = isfinite(bnorm) ? 0 : -1;
    while (status == 0 && it < max_it && !(sqrt(rr) <= rtol * bnorm)) {
        orc_apply_A(E, N, D, G, n_global, l2g, mask, p, Ap, work);
        const double pAp = dot(n_global, p, Ap);
        if (!(pAp > 0.0) || !isfinite(pAp)) { status = -1; break; }
        const double alpha = rz / pAp;
        for (int64_t g = 0; g < n_global; ++g) {
            x[g] += alpha * p[g];
            r[g] -= alpha * Ap[g];
            z[g] = dinv[g] * r[g];
        }
        const double rz_new = dot(n_global, r, z);
        const double beta = rz_new / rz;
        for (int64_t g = 0; g < n_global; ++g) p[g] = z[g] + beta * p[g];
        rz = rz_new;
        rr = dot(n_global, r, r);
        ++it;
    }
    orc_apply_A(E, N, D, G, n_global, l2g, mask, x, Ap, work);
    for (int64_t g = 0; g < n_global; ++g) r[g] = b[g] - Ap[g];
    if (rel_res) *rel_res = sqrt(dot(n_global, r, r)) / bnorm;
    free(work);
    free(r);
    free(z);
    free(p);
    free(Ap);
    return status ? -1 : it;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads the parallel loops use from now on (timing on one core or all of them). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
