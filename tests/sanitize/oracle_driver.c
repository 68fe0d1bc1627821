/* Calls every function of the CPU oracle on small inputs, with every buffer allocated at its
 * exact size, so that AddressSanitizer and UndefinedBehaviorSanitizer (the build in
 * test_sanitizers.py) see each access.  The mesh is a chain of E hexahedra along x with a global
 * shear (conforming, det J > 0) and homogeneous Dirichlet conditions on the whole boundary.
 * Prints "oracle-sanitize: ok" and exits 0 when every call behaved. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_legendre(int N, double x, double* L, double* dL);
int orc_gll(int N, double* xi, double* w, double* D);
void orc_jacobian(const double* V, double r, double s, double t, double* J);
void orc_jacobians(int64_t E, int N, const double* verts, const double* xi, double* J);
void orc_geom_factors(int64_t E, int N, const double* verts, const double* xi, const double* w, double* G,
                      double* gwj, double* min_det);
void orc_node_coords(int64_t E, int N, const double* verts, const double* xi, double* XYZ);
void orc_parallelepiped_h(int64_t E, const double* verts, double* h);
void orc_ax_local(int64_t E, int N, const double* D, const double* G, int nrhs, const double* X, double* Y);
void orc_ax_diag(int64_t E, int N, const double* D, const double* G, double* out);
void orc_gs_qt(int64_t n_local, int64_t n_global, const int32_t* l2g, int nrhs, const double* in, double* out);
void orc_gs_q(int64_t n_local, int64_t n_global, const int32_t* l2g, int nrhs, const double* in, double* out);
int orc_cg(int64_t E, int N, const double* D, const double* G, int64_t n_global, const int32_t* l2g,
           const uint8_t* mask, const double* b, double* x, double rtol, int max_it, double* rel_res);
int orc_pcg(int64_t E, int N, const double* D, const double* G, int64_t n_global, const int32_t* l2g,
            const uint8_t* mask, const double* b, const double* dinv, double* x, double rtol, int max_it,
            double* rel_res);
int orc_num_threads(void);
void orc_set_num_threads(int n);

static int g_fail = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            g_fail = 1;                                             \
        }                                                           \
    } while (0)

static double* dalloc(int64_t n) { return (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1)); }

static void chain(int E, int N, double* verts, int32_t* l2g, uint8_t* mask)
{
    const int N1 = N + 1, nx = E * N + 1;
    for (int e = 0; e < E; ++e)
        for (int v = 0; v < 8; ++v) {
            const double x = e + (v & 1), y = (v >> 1) & 1, z = (v >> 2) & 1;
            double* p = verts + (e * 8 + v) * 3;
            p[0] = x + 0.1 * y;
            p[1] = 0.9 * y + 0.05 * z;
            p[2] = 1.1 * z + 0.02 * x;
        }
    for (int e = 0; e < E; ++e)
        for (int k = 0; k < N1; ++k)
            for (int j = 0; j < N1; ++j)
                for (int i = 0; i < N1; ++i) {
                    const int gx = e * N + i;
                    const int32_t g = gx + nx * (j + N1 * k);
                    l2g[((int64_t)e * N1 + k) * N1 * N1 + j * N1 + i] = g;
                    mask[g] = (gx == 0 || gx == nx - 1 || j == 0 || j == N || k == 0 || k == N);
                }
}

static void run(int E, int N)
{
    const int N1 = N + 1, Np = N1 * N1 * N1, nx = E * N + 1;
    const int64_t nl = (int64_t)E * Np, ng = (int64_t)nx * N1 * N1;
    double* xi = dalloc(N1);
    double* w = dalloc(N1);
    double* D = dalloc(N1 * N1);
    CHECK(orc_gll(N, xi, w, D) == 0);
    double* verts = dalloc(E * 24);
    int32_t* l2g = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nl > 0 ? nl : 1));
    uint8_t* mask = (uint8_t*)malloc((size_t)ng);
    chain(E, N, verts, l2g, mask);
    double J1[9];
    if (E > 0) {
        orc_jacobian(verts, 0.3, -0.2, 0.7, J1);
        CHECK(isfinite(J1[0]) && isfinite(J1[8]));
    }
    double* J = dalloc(nl * 9);
    orc_jacobians(E, N, verts, xi, J);
    double* G = dalloc(nl * 6);
    double* gwj = dalloc(nl);
    double min_det = 0.0;
    orc_geom_factors(E, N, verts, xi, w, G, gwj, &min_det);
    if (E > 0) CHECK(min_det > 0.0);
    orc_geom_factors(E, N, verts, xi, w, NULL, gwj, NULL);
    double* XYZ = dalloc(nl * 3);
    orc_node_coords(E, N, verts, xi, XYZ);
    double* h = dalloc(E * 6);
    orc_parallelepiped_h(E, verts, h);
    double* X = dalloc(2 * nl);
    double* Y = dalloc(2 * nl);
    for (int64_t q = 0; q < 2 * nl; ++q) X[q] = sin(0.37 * (double)q);
    orc_ax_local(E, N, D, G, 2, X, Y);
    double* dg = dalloc(nl);
    orc_ax_diag(E, N, D, G, dg);
    double* gl = dalloc(2 * ng);
    orc_gs_qt(nl, ng, l2g, 2, Y, gl);
    orc_gs_q(nl, ng, l2g, 2, gl, X);
    /* b = Q^T of a smooth local field, zero under the mask */
    double* b = dalloc(ng);
    double* x = dalloc(ng);
    double* dinv = dalloc(ng);
    for (int64_t q = 0; q < nl; ++q) Y[q] = 1.0 + 0.5 * sin(0.11 * (double)q);
    orc_gs_qt(nl, ng, l2g, 1, Y, b);
    orc_gs_qt(nl, ng, l2g, 1, dg, dinv);
    for (int64_t g = 0; g < ng; ++g) {
        if (mask[g]) b[g] = 0.0;
        dinv[g] = mask[g] ? 0.0 : 1.0 / dinv[g];
        x[g] = 0.0;
    }
    double rr = 0.0;
    const int it = orc_cg(E, N, D, G, ng, l2g, mask, b, x, 1e-10, 2000, &rr);
    CHECK(it >= 0);
    if (N >= 2) CHECK(it > 0 && rr <= 1e-9);   /* interior nodes exist */
    for (int64_t g = 0; g < ng; ++g) x[g] = 0.0;
    const int itp = orc_pcg(E, N, D, G, ng, l2g, mask, b, dinv, x, 1e-10, 2000, &rr);
    CHECK(itp >= 0);
    if (N >= 2) CHECK(itp > 0 && rr <= 1e-9);
    printf("E=%d N=%d: cg %d it, pcg %d it, min det %.3e\n", E, N, it, itp, min_det);
    free(xi); free(w); free(D); free(verts); free(l2g); free(mask); free(J); free(G); free(gwj);
    free(XYZ); free(h); free(X); free(Y); free(dg); free(gl); free(b); free(x); free(dinv);
}

int main(void)
{
    orc_set_num_threads(1);
    CHECK(orc_num_threads() >= 1);
    for (int N = 1; N <= 32; ++N) {
        double* xi = dalloc(N + 1);
        double* w = dalloc(N + 1);
        double* D = dalloc((N + 1) * (N + 1));
        CHECK(orc_gll(N, xi, w, D) == 0);
        double L, dL;
        orc_legendre(N, 1.0, &L, &dL);
        CHECK(fabs(L - 1.0) < 1e-12);
        orc_legendre(N, -1.0, &L, &dL);
        orc_legendre(N, 0.3, &L, &dL);
        free(xi); free(w); free(D);
    }
    double t[40];
    CHECK(orc_gll(0, t, t, t) == -1);
    CHECK(orc_gll(33, t, t, t) == -1);
    run(1, 1);   /* every node on the boundary: b = 0 */
    run(3, 2);
    run(2, 5);
    run(4, 3);
    printf(g_fail ? "oracle-sanitize: FAILED\n" : "oracle-sanitize: ok\n");
    return g_fail;
}
