/*
 * axhosfem.h - C ABI of the MI355X (gfx950) matrix-free element-local Poisson operator with
 * on-the-fly geometric factors, after Cao, Sun, Zhang, Li, "Towards a Higher Roofline for
 * Matrix-Vector Multiplication in Matrix-Free HOSFEM" (arXiv 2504.07042).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - N is the polynomial order, N1 = N + 1 GLL points per direction, 1 <= N <= 15.
 *  - A local (element-wise) vector holds [nrhs][E][N1^3] values; node [i,j,k] of element e is
 *    at index i + j*N1 + k*N1^2 (the index rule stated with Algorithm 1, Sec. 2.2).
 *  - Vertex arrays are double [E][8][3] in the tensor order of the trilinear map (Eq. 8):
 *    vertex v = a + 2b + 4c sits at reference corner (2a-1, 2b-1, 2c-1).
 *  - Pointers marked [dev] are device pointers, [host] are host pointers.  Every buffer belongs to
 *    the caller; the library never frees or keeps a pointer after the call returns.  Host
 *    arrays are read during the call only (they are copied into kernel arguments).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Device work is
 *    enqueued on it and the call returns without synchronising, unless stated otherwise.
 *  - Every function returns an ax_status and never throws or aborts.  Arguments are validated
 *    on the host before anything is enqueued; on error nothing is enqueued and
 *    ax_last_error() describes the problem.  E == 0 (or an empty vector) is a valid no-op.
 *  - Device buffers must not overlap unless stated otherwise.
 */
#ifndef AXHOSFEM_H
#define AXHOSFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AX_OK = 0,
    AX_ERR_ARG = -1,           /* invalid argument (null pointer, negative size, aliasing ...) */
    AX_ERR_UNSUPPORTED = -2,   /* valid but not implemented (order, precision, geometry) */
    AX_ERR_HIP = -3,           /* a HIP runtime call failed; see ax_last_error() */
    AX_ERR_NOMEM = -4,         /* workspace too small */
    AX_ERR_NOT_CONVERGED = -5, /* iteration limit reached before the tolerance */
    AX_ERR_BREAKDOWN = -6      /* CG breakdown: p^T A p <= 0 or a non-finite scalar */
} ax_status;

/* Geometry of the elements handed to ax_local. */
enum { AX_TRILINEAR = 0, AX_PARALLELEPIPED = 1 };

/* Arithmetic of a kernel.  AX_FP64: X, Y and G are double.  AX_FP32: X, Y and G are float,
 * all arithmetic float (vertex differences and per-element geometry set-up in double).
 * AX_FP16_ACC32: X and Y are float; X and the D-contraction operands are rounded to half and
 * multiplied on the matrix cores with float accumulation; geometric factors stay float. */
enum { AX_FP64 = 0, AX_FP32 = 1, AX_FP16_ACC32 = 2 };

/* Message for the last non-OK status returned on the calling thread ("" if none). */
const char* ax_last_error(void);

/* Library version string. */
const char* ax_version(void);

/*
 * ax_gll - GLL points xi[N1], weights w[N1] and the differentiation matrix D[N1*N1] (row-major,
 * D[i*N1 + j] = pi_j'(xi_i)) of order N (Sec. 2.1, Table 1).  The diagonal of D is minus the
 * sum of the rest of its row (exactly the closed form in exact arithmetic).  [host] outputs.
 * Supports 1 <= N <= 31.
 */
int ax_gll(int N, double* xi, double* w, double* D);

/*
 * ax_local - Y = AxLocal(X): the element-local Poisson operator Y_e = D^T G_e D X_e of Eq. (3)
 * (Lambda0 = I, Lambda1 = 0), applied by sum factorisation as in Algorithm 1, with the six
 * geometric factors G_e recomputed inside the kernel instead of being read from memory:
 *   geom == AX_TRILINEAR:      geo = vertices [dev] double [E][8][3]; the factors of Eq. (7)
 *                              are rebuilt from the trilinear Jacobian (Eq. 9) with the reuse of
 *                              Sec. 3.3 (Algorithm 2, Eq. 10-12).
 *   geom == AX_PARALLELEPIPED: geo = h [dev] double [E][6], h = det(J) J^-1 J^-T of the
 *                              element's constant Jacobian without weights, order
 *                              00,01,02,11,12,22 (the input of Algorithm 3; see
 *                              ax_parallelepiped_factors).
 * D [host] double[N1*N1] (see ax_gll), xi and w [host] double[N1] (xi may be NULL for
 * AX_PARALLELEPIPED).  X [dev] read, Y [dev] fully overwritten; both [nrhs][E][N1^3] of the
 * storage type of `prec`; X and Y must not overlap.  Columns share the per-element geometric
 * set-up (Sec. 4.1): the vertices are read and the per-column polynomial coefficients of the
 * factors formed once per element for all nrhs columns; the per-node evaluation of the factors
 * from those coefficients is repeated for each column (cheaper than holding seven words per node
 * between columns).  No NaN checks are made.  Errors: E < 0, nrhs < 1, null pointers,
 * X == Y -> AX_ERR_ARG; N outside [1,15] or an unknown geom/prec -> AX_ERR_UNSUPPORTED.
 */
int ax_local(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
             const double* w, int nrhs, int prec, const void* X, void* Y, void* stream);

/*
 * ax_local_gathered - Y = AxLocal(Q Xg): the element-local operator applied to a global vector,
 * the gather Q of Eq. (1) fused into the operator's load (node l of element e reads
 * Xg[l2g[e N1^3 + l]]), so the local copy Q Xg is never stored.  This is the operator
 * application of the CG solver (cg_solve).  l2g [dev] int32 [E*N1^3], every entry in
 * [0, n_global) (not range-checked here: gs_build_csr checks a map); Xg [dev] [nrhs][n_global];
 * Y [dev] [nrhs][E][N1^3]; both of the storage type of prec, AX_FP64 or AX_FP32 (AX_FP16_ACC32
 * -> AX_ERR_UNSUPPORTED).  geom, geo, D, xi, w as ax_local; D must be a GLL differentiation
 * matrix (centro-antisymmetric, AX_ERR_UNSUPPORTED otherwise).  The result equals gs_assemble
 * (GS_Q) followed by ax_local bit for bit.  Errors: as ax_local, plus l2g NULL, n_global < 1 or
 * Xg == Y -> AX_ERR_ARG.
 */
int ax_local_gathered(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                      const double* w, int nrhs, int prec, const int32_t* l2g, int64_t n_global,
                      const void* Xg, void* Y, void* stream);

/*
 * ax_local_gathered_energy - ax_local_gathered for one FP32 column that also returns the energy
 * of the local operator, energy[0] = sum_e X_e^T Y_e = (Q Xg)^T A_L (Q Xg) with A_L the block
 * diagonal of Eq. (3) (when Xg vanishes on the Dirichlet nodes this is Xg^T A Xg, the p^T A p of
 * CG, Sec. 2.1).  Each node contributes (D X)^T G (D X), formed in FP32 in the pointwise stage of
 * the kernel; the sums over nodes of an element column are FP32, every further sum FP64 in a
 * fixed order (reproducible run to run).  This is the FP32 inner operator of cg_solve.
 * Xg [dev] float [n_global]; Y [dev] float [E][N1^3]; work [dev] double [E] scratch (one sum
 * per work-group); energy [dev] double [1].  Other arguments as ax_local_gathered with nrhs = 1
 * and prec = AX_FP32.  Errors: as ax_local_gathered; work (E > 0) or energy NULL -> AX_ERR_ARG.
 */
int ax_local_gathered_energy(int64_t E, int N, int geom, const double* geo, const double* D,
                             const double* xi, const double* w, const int32_t* l2g, int64_t n_global,
                             const float* Xg, float* Y, double* work, double* energy, void* stream);

/*
 * ax_local_vector - AxLocal on a vector field (n_col = 3, Sec. 2.1: X and Y hold three columns,
 * one per component), in the component-interleaved layout X, Y [dev] [E][3][N1^3] (the three
 * components of an element contiguous).  The three components share the element's geometric
 * set-up (the geometry loop outermost, Sec. 4.1: vertices read and the per-column coefficients of
 * the factors formed once per element; the per-node evaluation repeated per component), so the
 * traffic per element is 2 x 3 N1^3 values plus the geometry input once.  geom AX_TRILINEAR (geo = vertices) or
 * AX_PARALLELEPIPED (geo = h), prec AX_FP64 or AX_FP32 (AX_FP16_ACC32 -> AX_ERR_UNSUPPORTED);
 * other arguments and errors as ax_local.
 */
int ax_local_vector(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                    const double* w, int prec, const void* X, void* Y, void* stream);

/*
 * ax_tune_set / ax_tune_get - [host] the launch variants of the AxLocal kernels, one entry per
 * (order N, tuning kind, precision AX_FP64 or AX_FP32).  Kinds: AX_TUNE_TRILINEAR (ax_local on
 * trilinear elements, also ax_local_vector and the CG operators), AX_TUNE_PARALLELEPIPED,
 * AX_TUNE_STORED (ax_local_precomputedG), AX_TUNE_PARTIAL (ax_local_partial),
 * AX_TUNE_HELMHOLTZ (ax_local_helmholtz) and AX_TUNE_BATCHED (the per-order kernels of the
 * batched launches; N <= 9).  Every variant computes the same result; only the speed differs.
 * Fields of ax_tune:
 *   kernel     AX_KERNEL_AUTO (the measured default), AX_KERNEL_TILE (the prefetching kernel:
 *              several elements per work-group, next element's input loaded during the current
 *              one) or AX_KERNEL_ITEM (the per-item kernel: element groups handed out one at a
 *              time, tables reloaded per output row); ITEM exists for the trilinear full form
 *              (every order) and the partial form (N >= 8) on GLL bases: elsewhere the tile
 *              kernel runs.  AX_TUNE_BATCHED: AX_KERNEL_TILE runs the tile kernel (default
 *              shape): with tile_alt 0 over the work list where the order has that form (FP64
 *              N <= 6, FP32 N <= 9), with tile_alt 1 over mesh slices (each work-group walks one
 *              mesh, every order); AUTO and ITEM the per-item kernel.
 *   tile_alt   tile kernel: 0 default elements per work-group, 1 the alternative shape;
 *   item_alt   per-item kernels (single-mesh and batched): 0 a 256-lane work-group, 1 the
 *              order's alternative shape (N <= 12; see elems_per_group and block);
 *   waves_alt  single-mesh per-item kernel: 0 the default register budget, 1 the alternative
 *              (one wave per SIMD more where the default is two, one fewer where it is five);
 *   grid_mult  persistent grid = grid_mult x the resident work-group capacity, 1..64.
 * ax_tune_get also fills the read-only fields: kernel_used (what AUTO resolves to for this
 * entry: AX_KERNEL_TILE or AX_KERNEL_ITEM), elems_per_group and block (the work-group shape that
 * will run) and waves (the waves per SIMD its register budget targets).  The table is
 * process-wide and applies to launches enqueued after the call; a batched work list keeps the
 * shape it was prepared with.  Written by the autotuner from its cache
 * (paper_2504_07042_amd/autotune.py).  Errors: N outside [1,15] -> AX_ERR_UNSUPPORTED; unknown
 * kind, precision or field value, or AX_TUNE_BATCHED with N > 9 -> AX_ERR_ARG.
 */
enum { AX_STORED_G = 2 };
enum { AX_TUNE_TRILINEAR = 0, AX_TUNE_PARALLELEPIPED = 1, AX_TUNE_STORED = 2, AX_TUNE_PARTIAL = 3,
       AX_TUNE_HELMHOLTZ = 4, AX_TUNE_BATCHED = 5 };
enum { AX_KERNEL_AUTO = 0, AX_KERNEL_TILE = 1, AX_KERNEL_ITEM = 2 };
typedef struct {
    int kernel;
    int tile_alt;
    int item_alt;
    int waves_alt;
    int grid_mult;
    /* filled by ax_tune_get, ignored by ax_tune_set */
    int kernel_used;
    int elems_per_group;
    int block;
    int waves;
} ax_tune;
int ax_tune_set(int N, int kind, int prec, const ax_tune* t);
int ax_tune_get(int N, int kind, int prec, ax_tune* t);

/*
 * ax_local_precomputedG - the same operator with the six factors streamed from memory, the
 * baseline the paper improves on (Algorithm 1 and Algorithm 4 with getFactors = memory loads).
 * G [dev] [E][6][N1^3] in order G00,G01,G02,G11,G12,G22, weights included; double for AX_FP64,
 * float for AX_FP32 and AX_FP16_ACC32.  Other arguments as ax_local.
 */
int ax_local_precomputedG(int64_t E, int N, const void* G, const double* D, int nrhs, int prec,
                          const void* X, void* Y, void* stream);

/*
 * ax_local_partial - the trilinear operator with partial recomputation (Sec. 4.2.2, Table 3,
 * the Poisson form): the per-node scale lam = 0.125 w_i w_j w_k / det(8J) of Eq. (12) is read
 * from memory and the kernel recomputes only K = (8J)^T (8J) and adj(K) per node, with no
 * determinant and no division (F_geo = 72 N1 + 45 N1^2 + 60 N1^3 per element, one more word per
 * node of traffic).  verts [dev] double [E][8][3] as ax_local; lam [dev] [E][N1^3], double for
 * AX_FP64, float for AX_FP32 (written by ax_geom_lambda); prec AX_FP64 or AX_FP32 (AX_FP16_ACC32
 * -> AX_ERR_UNSUPPORTED); xi, w [host] double[N1]; other arguments and errors as ax_local.
 */
int ax_local_partial(int64_t E, int N, const double* verts, const void* lam, const double* D,
                     const double* xi, const double* w, int nrhs, int prec, const void* X, void* Y,
                     void* stream);

/*
 * ax_local_helmholtz - the trilinear Helmholtz operator of Eq. (3),
 *   Y_e = D^T (Lambda0 G_e) D X_e + Lambda1 Gwj X_e,
 * with the merged scalar factors of Sec. 4.2.1 read per node: Lambda2 = lam lambda0 scales
 * adj(K) (K, adj(K) recomputed from the vertices as in ax_local_partial) and Lambda3 =
 * gwj lambda1 scales the mass term; no determinant and no division in the kernel.
 * L23 [dev] [E][2][N1^3] (Lambda2 block, then Lambda3 block, per element), double for AX_FP64,
 * float for AX_FP32 (written by ax_helmholtz_factors); prec AX_FP64 or AX_FP32 (AX_FP16_ACC32
 * -> AX_ERR_UNSUPPORTED); other arguments and errors as ax_local_partial.
 */
int ax_local_helmholtz(int64_t E, int N, const double* verts, const void* L23, const double* D,
                       const double* xi, const double* w, int nrhs, int prec, const void* X, void* Y,
                       void* stream);

/*
 * ax_helmholtz_factors - set-up for ax_local_helmholtz (Sec. 4.2.1): from the nodal values of
 * the coefficient fields lambda0, lambda1 [dev] double [E][N1^3] of Eq. (2), writes
 * L23[e][0][node] = 0.125 w_i w_j w_k / det(8J) * lambda0 and L23[e][1][node] =
 * w_i w_j w_k det J * lambda1 (the lumped mass Gwj of Eq. 3), double if prec == AX_FP64, float
 * if AX_FP32.  verts [dev] double [E][8][3]; xi, w [host] double[N1].  AX_ERR_ARG for NULL
 * arrays, AX_ERR_UNSUPPORTED for N outside [1,15] or another prec.  Asynchronous on `stream`.
 */
int ax_helmholtz_factors(int64_t E, int N, const double* verts, const double* xi, const double* w,
                         const double* lambda0, const double* lambda1, int prec, void* L23, void* stream);

/*
 * ax_geom_lambda - set-up for ax_local_partial: lam [dev] [E][N1^3] = 0.125 w_i w_j w_k / det(8J)
 * at every node of the trilinear elements (8J: the Jacobian of Eq. 9 without its factor 1/8, as
 * in Algorithm 2), double if prec == AX_FP64, float if AX_FP32.  verts [dev] double [E][8][3];
 * xi, w [host] double[N1].  AX_ERR_ARG for NULL arrays, AX_ERR_UNSUPPORTED for N outside [1,15]
 * or another prec.  Asynchronous on `stream`.
 */
int ax_geom_lambda(int64_t E, int N, const double* verts, const double* xi, const double* w, int prec,
                   void* lam, void* stream);

/*
 * ax_local_diag - the diagonal of every element matrix D^T G_e D of Eq. (3) (Poisson), with the
 * factors recomputed as in ax_local (trilinear: from the vertices, Eq. 12; parallelepiped: w h).
 * Only the GLL line through a node in each direction contributes to its diagonal (the gradient
 * blocks of Table 1 act on one index each), plus the off-diagonal factors at the node itself.
 * out [dev] double [E][N1^3]; D [host] N1*N1, xi, w [host] N1 (xi may be NULL for
 * AX_PARALLELEPIPED); geo as ax_local.  Errors as ax_local.  Asynchronous on `stream`.
 */
int ax_local_diag(int64_t E, int N, int geom, const double* geo, const double* D, const double* xi,
                  const double* w, double* out, void* stream);

/*
 * ax_geom_factors - set-up: write the stored factors of Eq. (7) for trilinear elements,
 * G [dev] [E][6][N1^3] (double if prec == AX_FP64, float if AX_FP32) and, if gwj is not NULL,
 * gwj [dev] double [E][N1^3] = w_i w_j w_k det J (the lumped mass, second factor of Eq. 7).
 * verts [dev] double [E][8][3]; xi, w [host] double[N1].  G may be NULL.
 */
int ax_geom_factors(int64_t E, int N, const double* verts, const double* xi, const double* w,
                    int prec, void* G, double* gwj, void* stream);

/*
 * ax_parallelepiped_factors - set-up for Algorithm 3: h [dev] double [E][6] = det J J^-1 J^-T
 * (order 00,01,02,11,12,22, no weights) of each element's constant Jacobian
 * J = 1/2 [v1 - v0, v2 - v0, v4 - v0] (Eq. 9 for an affine element).  verts [dev] [E][8][3].
 * The elements must be parallelepipeds; this is not checked.
 */
int ax_parallelepiped_factors(int64_t E, const double* verts, double* h, void* stream);

/*
 * ax_check_mesh - set-up: reject inverted or degenerate elements.  Evaluates det J of the
 * trilinear map (Eq. 8-9) at every GLL node of every element; the geometric factors of Eq. (7)
 * divide by det J, so the operator is defined only where det J > 0.  verts [dev] double
 * [E][8][3]; xi [host] double[N1] (the nodes of the order the mesh will be used with).  On
 * return *bad_element [host] is the lowest index of an element with det J <= 0 or not finite at
 * some node (-1 if none) and *min_det [host] the smallest finite det J over all nodes (+inf if
 * E == 0); either pointer may be NULL.  Returns AX_ERR_ARG naming the element if one fails.
 * Unlike the other entry points this call synchronises `stream` (it reads the result back) and
 * allocates 16 bytes of device memory for the reduction, so it cannot be captured in a graph.
 * Parallelepipeds are covered too (their det J is constant).  Errors: E < 0, xi or verts NULL
 * -> AX_ERR_ARG; N outside [1,15] -> AX_ERR_UNSUPPORTED.
 */
int ax_check_mesh(int64_t E, int N, const double* verts, const double* xi, int64_t* bad_element,
                  double* min_det, void* stream);

/*
 * ax_node_coords - physical coordinates of every GLL node, x = sum_v sigma_v(xi_i,xi_j,xi_k) v
 * (Eq. 8).  XYZ [dev] double [E][3][N1^3].  verts [dev]; xi [host] double[N1].
 */
int ax_node_coords(int64_t E, int N, const double* verts, const double* xi, double* XYZ,
                   void* stream);

/*
 * Gather-scatter (the binary matrix Q of Sec. 2.1 and the assembly A = Q^T blockdiag(A_e) Q of
 * Eq. 1).  l2g[l] = global id of local node l (int32, 0 <= l2g[l] < n_global).
 *
 * gs_build_csr - [host] the inverse map of l2g in CSR form: the local ids of global node g are
 * gidx[gptr[g] .. gptr[g+1]-1] in ascending order.  gptr int64 [n_global + 1], gidx int32
 * [n_local].  Returns AX_ERR_ARG if some l2g entry is out of range.
 */
int gs_build_csr(int64_t n_local, int64_t n_global, const int32_t* l2g, int64_t* gptr,
                 int32_t* gidx);

/* Modes of gs_assemble. */
enum {
    GS_QT = 0,  /* out[global] = sum of in[local] over the local copies (ascending local id)   */
    GS_Q = 1,   /* out[local]  = in[l2g[local]]                                              */
    GS_QQT = 2  /* out[local]  = (Q Q^T in)[local]: sum over all copies of the node, then copy */
};

/*
 * gs_assemble - apply Q^T, Q or Q Q^T to nrhs vectors.  l2g, gptr, gidx [dev] (the CSR of
 * gs_build_csr); mask [dev] uint8 [n_global] or NULL: where mask[g] != 0 the global value is
 * set to 0 (homogeneous Dirichlet) in GS_QT output and before the copy-out of GS_QQT.
 * dtype AX_FP64 (double) or AX_FP32 (float).  in/out [dev] are [nrhs][n_local] or
 * [nrhs][n_global] as the mode implies.  Sums are taken in ascending local id with no atomics,
 * so results are deterministic.  in and out must not overlap.
 */
int gs_assemble(int64_t n_local, int64_t n_global, const int32_t* l2g, const int64_t* gptr,
                const int32_t* gidx, const uint8_t* mask, int mode, int nrhs, int dtype,
                const void* in, void* out, void* stream);

/* A Poisson problem on one mesh: the assembled operator y = mask o Q^T AxLocal(Q x). */
typedef struct {
    int64_t E;
    int N;
    int geom;              /* AX_TRILINEAR or AX_PARALLELEPIPED                          */
    const double* geo;     /* [dev] vertices [E][8][3] or h [E][6] (see ax_local)        */
    const double* D;       /* [host] N1*N1                                               */
    const double* xi;      /* [host] N1                                                  */
    const double* w;       /* [host] N1                                                  */
    int64_t n_global;
    const int32_t* l2g;    /* [dev] [E*N1^3]                                             */
    const int64_t* gptr;   /* [dev] [n_global + 1]                                       */
    const int32_t* gidx;   /* [dev] [E*N1^3]                                             */
    const uint8_t* mask;   /* [dev] [n_global] Dirichlet mask, or NULL                   */
} ax_problem;

typedef struct {
    double rtol;           /* target ||b - A x||_2 / ||b||_2 (true residual, FP64)        */
    int max_it;            /* iteration limit (plain CG) / inner limit per outer step     */
    int inner_prec;        /* AX_FP64: plain FP64 CG; AX_FP32 / AX_FP16_ACC32: iterative
                              refinement with an inner CG in that precision               */
    double inner_rtol;     /* relative tolerance of each inner solve (refinement only)    */
    int max_outer;         /* refinement steps limit                                      */
    void* workspace;       /* [dev] at least cg_workspace_bytes() bytes                   */
    size_t workspace_bytes;
    int use_graph;         /* 1: capture the CG iteration block in a HIP graph and replay it */
    int refine;            /* AX_REFINE_RESTART or AX_REFINE_RELIABLE (refinement only)    */
    int precond;           /* AX_PRECOND_NONE or AX_PRECOND_JACOBI                         */
} ax_cg_opts;

/* Preconditioners of the CG iterations (ax_cg_opts.precond):
 * AX_PRECOND_NONE   - plain CG;
 * AX_PRECOND_JACOBI - z = diag(A)^-1 r with the diagonal of the assembled operator (the element
 *                     diagonals of ax_local_diag, factors recomputed, assembled by Q^T; zero on
 *                     the Dirichlet nodes); the paper does not name the preconditioner of the
 *                     solves of Sec. 5.6, the diagonal one is this library's reading.
 *                     The same diagonal (in float) serves the reduced-precision iterations of
 *                     the mixed-precision solves.  The convergence test stays on ||r||_2. */
enum { AX_PRECOND_NONE = 0, AX_PRECOND_JACOBI = 1 };

/* Refinement schemes of the mixed-precision solves (ax_cg_opts.refine):
 * AX_REFINE_RESTART  - each correction A d = r / ||r|| is an inner CG started from scratch and
 *                      solved to inner_rtol; max_outer bounds the number of corrections.
 * AX_REFINE_RELIABLE - one reduced-precision CG recurrence runs throughout; each time its
 *                      iterated residual has dropped by the factor inner_rtol (< 1) its iterate
 *                      is added to x in FP64 and its residual is replaced by the FP64 true
 *                      residual b - A x, keeping the search direction (reliable updates);
 *                      max_outer bounds the number of such updates. */
enum { AX_REFINE_RESTART = 0, AX_REFINE_RELIABLE = 1 };

typedef struct {
    int status;            /* ax_status of the solve                                      */
    int outer_it;          /* refinement steps (1 for plain CG)                           */
    int inner_it_total;    /* CG iterations summed over all steps                          */
    double rel_res_true;   /* ||b - A x|| / ||b|| recomputed in FP64 at exit              */
    double seconds;        /* wall time of the solve                                      */
} ax_cg_report;

/* cg_workspace_bytes - [host] bytes of device workspace cg_solve needs. */
int cg_workspace_bytes(const ax_problem* p, int nrhs, const ax_cg_opts* o, size_t* bytes);

/*
 * cg_solve - solve A x = b (each of nrhs columns independently) by conjugate gradients on the
 * assembled operator; the iterative solve in which AxLocal is the dominant kernel (Sec. 1,
 * Sec. 5.6).  b, x [dev] double [nrhs][n_global]; x holds the initial guess on entry (warm
 * start / resume) and the solution on exit.  Entries of b under the mask must be 0: the
 * assembled rows there are zero, so a nonzero entry is rejected with AX_ERR_ARG (checked on the
 * device, with one stream synchronisation, before the first iteration).
 * inner_prec == AX_FP64 runs plain CG in FP64.  Otherwise mixed-precision iterative refinement:
 * the outer residual r = b - A x, its norm and the update of x are FP64; the corrections come
 * from CG iterations whose AxLocal runs in inner_prec with float vectors and FP64-accumulated
 * dot products, restarted per correction or continued through reliable updates (o->refine).  All scalars stay on the device; the host polls the
 * convergence flags every 8 iterations, and with use_graph those 8 iterations are captured once
 * in a HIP graph and replayed.  The work runs on a private stream of the calling thread after
 * `stream` has been synchronised, and both are synchronised before returning (rep is filled).
 * Returns AX_OK, AX_ERR_NOT_CONVERGED or AX_ERR_BREAKDOWN (rep->status holds the same);
 * AX_ERR_UNSUPPORTED, before any work, for more than 2^31 - 1 local nodes (local ids are int32).
 */
int cg_solve(const ax_problem* p, int nrhs, const double* b, double* x, const ax_cg_opts* o,
             ax_cg_report* rep, void* stream);

/*
 * Batched AxLocal over many independent trilinear meshes of uneven E and order N (1 <= N <= 9),
 * each with nrhs columns, in one persistent kernel launch per order present (the n_col /
 * multi-column reuse of Sec. 4.1 extended to many meshes), each kernel walking the work items of
 * its order.  Only E, N, geom (must be AX_TRILINEAR), geo, D, xi, w of
 * each ax_problem are read; D must be a GLL differentiation matrix (centro-antisymmetric).
 *
 * ax_batched_workspace_bytes - [host] device workspace needed for this set of meshes.
 * ax_batched_prepare - [host, synchronous] build the work list of (mesh, element group) items
 *   (ordered by decreasing cost) and upload it, the per-mesh pointers X[m], Y[m] ([dev] local
 *   vectors [nrhs][E_m][N1_m^3], double for AX_FP64, float for AX_FP32; column c of mesh m
 *   starts at X[m] + c * col_stride[m] (col_stride may be NULL: E_m * N1_m^3)) and the GLL tables into
 *   `workspace` [dev]; fills the host `plan`.  The workspace must stay untouched while it is
 *   in use; X/Y pointers are baked in (re-prepare to change them).
 * ax_local_batched - enqueue the persistent launches described by plan + workspace (one per
 *   order, on `stream`).  They read nothing from the host beyond `plan`, so they can be captured
 *   in a HIP graph and replayed.
 */
typedef struct {
    int64_t n_items;  /* work items (element groups) over all meshes */
    int nrhs;
    int prec;         /* AX_FP64 or AX_FP32 */
    size_t bytes;     /* workspace bytes in use */
    int n_mesh;
    int gather;       /* 0 (internal use: 1 for the solver's plans reading a global vector) */
    int64_t order_first[11];  /* items of order N1 = N + 1 (2..10): [order_first[N1], +order_count[N1]) */
    int64_t order_count[11];
    int order_variant[11];    /* kernel and work-group shape of order N1 at prepare time: 0, 1 the
                                 per-item shapes (ax_tune.item_alt), 2 the tile kernel over the
                                 work list, 3 the tile kernel over mesh slices */
} ax_batch_plan;

int ax_batched_workspace_bytes(int n_mesh, const ax_problem* meshes, size_t* bytes);
int ax_batched_prepare(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const void* const* X,
                       void* const* Y, const int64_t* col_stride, void* workspace, size_t workspace_bytes,
                       ax_batch_plan* plan);
int ax_local_batched(const ax_batch_plan* plan, const void* workspace, void* stream);

/*
 * ax_local_batched_noalloc - the batched AxLocal of ax_batched_prepare + ax_local_batched in one
 * call that allocates nothing, for callers that cannot allocate (code under stream capture, tight
 * serving loops, harnesses that forbid allocation).  The work list, mesh descriptors and basis
 * tables go to a static device array of the library (8 MiB per device, held until the process
 * ends) instead of a workspace; they are written there by small kernels from their kernel
 * arguments, so the call makes no hipMalloc/hipFree, no host heap allocation and no host-device
 * copy, and only enqueues kernels on `stream`.  Arguments as ax_batched_prepare (X, Y [dev],
 * col_stride [host] or NULL); the result equals ax_local_batched's bit for bit.  Limits:
 * n_mesh <= 4096 and a work list of at most 8 MiB (about 10^6 element groups); larger batches
 * -> AX_ERR_ARG with the size needed.  Every call on one device shares the array, which keeps
 * the last call's contents: calls that overlap on one device (different streams or threads) race
 * and must be serialised by the caller.
 */
int ax_local_batched_noalloc(int n_mesh, const ax_problem* meshes, int nrhs, int prec, const void* const* X,
                             void* const* Y, const int64_t* col_stride, void* stream);

/*
 * cg_solve_batched - CG (or mixed-precision refinement, inner_prec AX_FP32) on many independent
 * trilinear meshes at once: the meshes' global numberings are concatenated by the caller into
 * one index space of n_global nodes (l2g maps the concatenated local vectors, mesh after mesh,
 * to it; gptr/gidx its CSR inverse; mask its Dirichlet nodes), so the union operator is block
 * diagonal.  Each CG step applies the union operator with ONE batched persistent AxLocal launch
 * between two gather-scatter kernels.  Each of the nrhs columns runs its own CG over the union
 * (one alpha and beta per column).  b, x [dev] double [nrhs][n_global].  Other conventions and
 * return values as cg_solve.
 */
int cg_batched_workspace_bytes(int n_mesh, const ax_problem* meshes, int64_t n_global, int nrhs,
                               const ax_cg_opts* o, size_t* bytes);
int cg_solve_batched(int n_mesh, const ax_problem* meshes, int64_t n_global, const int32_t* l2g,
                     const int64_t* gptr, const int32_t* gidx, const uint8_t* mask, int nrhs,
                     const double* b, double* x, const ax_cg_opts* o, ax_cg_report* rep, void* stream);

/*
 * Machine probes for the time-based roofline of Sec. 3.4, whose memory time divides the traffic
 * by the measured bandwidth and whose compute time divides the flops by the peak of the units
 * that run them (Table 4 lists measured bandwidths beside the theoretical ones).  The caller
 * times the launches (e.g. with events on `stream`); the probes only enqueue work.
 *
 * ax_probe_copy - dst = src over `bytes` bytes [dev] (a multiple of 16, both pointers 16-byte
 *   aligned, no overlap): one read and one write of every byte, for the sustained HBM bandwidth
 *   (time the copy of a footprint well above the 256 MB Infinity Cache).  AX_ERR_ARG otherwise.
 * ax_probe_compute - one launch of an arithmetic loop, `iters` iterations, 32 waves per compute
 *   unit; *flops [host] receives the flops it executes.  kind:
 *     AX_PROBE_FMA_F64 / AX_PROBE_FMA_F32   fused multiply-add on the vector ALU (FP32 without
 *                                           packed instructions, as the library is built),
 *     AX_PROBE_MFMA_F64 / AX_PROBE_MFMA_F32 16x16x4 matrix-core instructions,
 *     AX_PROBE_MIX_F64                      both FP64 loops in the same waves: a time near the
 *                                           sum of the two separate times means the units do
 *                                           not overlap, near the larger one that they do.
 *   out [dev] receives one value per thread: at least ax_probe_compute_elems() elements of the
 *   kind's type (double for *_F64, float for *_F32).
 */
enum { AX_PROBE_FMA_F64 = 0, AX_PROBE_FMA_F32 = 1, AX_PROBE_MFMA_F64 = 2, AX_PROBE_MFMA_F32 = 3,
       AX_PROBE_MIX_F64 = 4 };
int ax_probe_copy(const void* src, void* dst, size_t bytes, void* stream);
int ax_probe_compute_elems(size_t* n);
int ax_probe_compute(int kind, int iters, void* out, double* flops, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AXHOSFEM_H */
