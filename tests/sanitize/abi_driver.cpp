// Exercises the host side of the C ABI without a GPU: argument validation of every entry point,
// the GLL tables, the tuning table, the CSR inverse of a numbering and the workspace sizing, with
// every host buffer at its exact size.  Built by test_sanitizers.py against a host-only
// AddressSanitizer + UndefinedBehaviorSanitizer build of the library sources.  Device pointers
// here are placeholders that the validation must reject or never touch.  Prints
// "abi-sanitize: ok" and exits 0 when every call returned the documented status.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "axhosfem.h"

static int g_fail = 0;
#define EXPECT(call, want)                                                                     \
    do {                                                                                       \
        const int got_ = (call);                                                               \
        if (got_ != (want)) {                                                                  \
            std::fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, \
                         got_, (int)(want), ax_last_error());                                  \
            g_fail = 1;                                                                        \
        }                                                                                      \
    } while (0)
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "line %d: check failed: %s\n", __LINE__, #c);    \
            g_fail = 1;                                                           \
        }                                                                         \
    } while (0)

static void* P(uintptr_t v) { return reinterpret_cast<void*>(v); }

struct Gll {
    std::vector<double> xi, w, D;
    explicit Gll(int N) : xi(N + 1), w(N + 1), D((N + 1) * (N + 1)) { ax_gll(N, xi.data(), w.data(), D.data()); }
};

// lexicographic numbering of an nx x ny x nz box of order-N elements
static int64_t box_numbering(int nx, int ny, int nz, int N, std::vector<int32_t>& l2g)
{
    const int N1 = N + 1, gx = nx * N + 1, gy = ny * N + 1, gz = nz * N + 1;
    l2g.assign((size_t)nx * ny * nz * N1 * N1 * N1, 0);
    size_t q = 0;
    for (int ez = 0; ez < nz; ++ez)
        for (int ey = 0; ey < ny; ++ey)
            for (int ex = 0; ex < nx; ++ex)
                for (int k = 0; k < N1; ++k)
                    for (int j = 0; j < N1; ++j)
                        for (int i = 0; i < N1; ++i)
                            l2g[q++] = (ex * N + i) + gx * ((ey * N + j) + gy * (ez * N + k));
    return (int64_t)gx * gy * gz;
}

int main()
{
    CHECK(std::strlen(ax_version()) > 0);
    for (int N = 1; N <= 31; ++N) {
        std::vector<double> xi(N + 1), w(N + 1), D((N + 1) * (N + 1));
        EXPECT(ax_gll(N, xi.data(), w.data(), D.data()), AX_OK);
        double sw = 0;
        for (double v : w) sw += v;
        CHECK(std::fabs(sw - 2.0) < 1e-12);
    }
    double t[64];
    EXPECT(ax_gll(0, t, t, t), AX_ERR_UNSUPPORTED);
    EXPECT(ax_gll(32, t, t, t), AX_ERR_UNSUPPORTED);
    CHECK(std::strlen(ax_last_error()) > 0);

    // tuning table
    ax_tune t0{}, t1{};
    EXPECT(ax_tune_get(7, AX_TUNE_TRILINEAR, AX_FP64, &t0), AX_OK);
    t1 = t0;
    t1.kernel = AX_KERNEL_ITEM;
    t1.item_alt = 1;
    t1.grid_mult = 4;
    EXPECT(ax_tune_set(7, AX_TUNE_TRILINEAR, AX_FP64, &t1), AX_OK);
    ax_tune t2{};
    EXPECT(ax_tune_get(7, AX_TUNE_TRILINEAR, AX_FP64, &t2), AX_OK);
    CHECK(t2.kernel_used == AX_KERNEL_ITEM && t2.grid_mult == 4 && t2.block == 128);
    EXPECT(ax_tune_set(7, AX_TUNE_TRILINEAR, AX_FP64, &t0), AX_OK);
    t1.tile_alt = 2;
    EXPECT(ax_tune_set(7, AX_TUNE_TRILINEAR, AX_FP64, &t1), AX_ERR_ARG);
    EXPECT(ax_tune_set(16, AX_TUNE_TRILINEAR, AX_FP64, &t0), AX_ERR_UNSUPPORTED);
    EXPECT(ax_tune_set(7, 6, AX_FP64, &t0), AX_ERR_ARG);
    EXPECT(ax_tune_set(10, AX_TUNE_BATCHED, AX_FP64, &t0), AX_ERR_ARG);
    EXPECT(ax_tune_get(7, AX_TUNE_TRILINEAR, AX_FP64, nullptr), AX_ERR_ARG);
    for (int N = 1; N <= 15; ++N)
        for (int k = 0; k < 6; ++k)
            for (int p = 0; p < 2; ++p) {
                ax_tune t{};
                EXPECT(ax_tune_get(N, k, p, &t), (k == AX_TUNE_BATCHED && N > 9) ? AX_ERR_ARG : AX_OK);
            }

    // element-local operators: validation only
    Gll b3(3);
    const double *D = b3.D.data(), *xi = b3.xi.data(), *w = b3.w.data();
    EXPECT(ax_local(-1, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_ARG);
    EXPECT(ax_local(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 0, AX_FP64, P(16), P(24), nullptr), AX_ERR_ARG);
    EXPECT(ax_local(4, 0, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(ax_local(4, 3, 9, (double*)P(8), D, xi, w, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(ax_local(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, 7, P(16), P(24), nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(ax_local(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, AX_FP64, P(16), P(16), nullptr), AX_ERR_ARG);
    EXPECT(ax_local(4, 3, AX_TRILINEAR, (double*)P(8), nullptr, xi, w, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_ARG);
    EXPECT(ax_local(4, 3, AX_TRILINEAR, nullptr, D, xi, w, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_ARG);
    EXPECT(ax_local(0, 3, AX_TRILINEAR, nullptr, D, xi, w, 1, AX_FP64, nullptr, nullptr, nullptr), AX_OK);
    EXPECT(ax_local_vector(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, AX_FP16_ACC32, P(16), P(24), nullptr),
           AX_ERR_UNSUPPORTED);
    EXPECT(ax_local_vector(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, AX_FP64, P(16), P(16), nullptr), AX_ERR_ARG);
    EXPECT(ax_local_precomputedG(3, 2, nullptr, D, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_ARG);
    EXPECT(ax_local_precomputedG(3, 99, P(8), D, 1, AX_FP64, P(16), P(24), nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(ax_local_partial(2, 3, nullptr, nullptr, D, xi, w, 1, AX_FP64, P(8), P(16), nullptr), AX_ERR_ARG);
    EXPECT(ax_local_partial(2, 3, (double*)P(8), P(8), D, xi, w, 1, AX_FP16_ACC32, P(8), P(16), nullptr),
           AX_ERR_UNSUPPORTED);
    EXPECT(ax_local_helmholtz(2, 3, (double*)P(8), nullptr, D, xi, w, 1, AX_FP64, P(8), P(16), nullptr), AX_ERR_ARG);
    EXPECT(ax_helmholtz_factors(2, 3, (double*)P(8), xi, w, nullptr, (double*)P(8), AX_FP64, P(8), nullptr),
           AX_ERR_ARG);
    EXPECT(ax_geom_lambda(-1, 3, (double*)P(8), xi, w, AX_FP64, P(8), nullptr), AX_ERR_ARG);
    EXPECT(ax_local_diag(2, 3, AX_TRILINEAR, nullptr, D, xi, w, (double*)P(8), nullptr), AX_ERR_ARG);
    EXPECT(ax_geom_factors(2, 3, (double*)P(8), nullptr, w, AX_FP64, P(8), nullptr, nullptr), AX_ERR_ARG);
    EXPECT(ax_geom_factors(2, 3, (double*)P(8), xi, w, AX_FP64, nullptr, nullptr, nullptr), AX_OK);
    EXPECT(ax_parallelepiped_factors(-2, (double*)P(8), (double*)P(16), nullptr), AX_ERR_ARG);
    EXPECT(ax_parallelepiped_factors(0, nullptr, nullptr, nullptr), AX_OK);
    EXPECT(ax_node_coords(2, 3, (double*)P(8), nullptr, (double*)P(16), nullptr), AX_ERR_ARG);
    // the gathering operator and its energy form reject bad arguments before any launch
    const int32_t* map = (const int32_t*)P(32);
    EXPECT(ax_local_gathered(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, AX_FP64, nullptr, 10, P(16), P(24),
                             nullptr), AX_ERR_ARG);
    EXPECT(ax_local_gathered(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, 1, AX_FP16_ACC32, map, 10, P(16), P(24),
                             nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(ax_local_gathered(0, 3, AX_TRILINEAR, nullptr, D, xi, w, 1, AX_FP64, nullptr, 10, nullptr, nullptr,
                             nullptr), AX_OK);
    EXPECT(ax_local_gathered_energy(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, map, 10, (const float*)P(16),
                                    (float*)P(24), (double*)P(40), nullptr, nullptr), AX_ERR_ARG);
    EXPECT(ax_local_gathered_energy(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, map, 10, (const float*)P(16),
                                    (float*)P(24), nullptr, (double*)P(48), nullptr), AX_ERR_ARG);
    EXPECT(ax_local_gathered_energy(4, 3, AX_TRILINEAR, (double*)P(8), D, xi, w, map, 0, (const float*)P(16),
                                    (float*)P(24), (double*)P(40), (double*)P(48), nullptr), AX_ERR_ARG);
    int64_t bad = 7;
    double dmin = 0;
    EXPECT(ax_check_mesh(0, 3, nullptr, xi, &bad, &dmin, nullptr), AX_OK);
    CHECK(bad == -1 && std::isinf(dmin));
    EXPECT(ax_check_mesh(2, 3, nullptr, xi, &bad, &dmin, nullptr), AX_ERR_ARG);
    EXPECT(ax_check_mesh(2, 3, (double*)P(8), nullptr, nullptr, nullptr, nullptr), AX_ERR_ARG);

    // gather-scatter: the CSR inverse of a box numbering, and validation
    std::vector<int32_t> l2g;
    const int64_t ng = box_numbering(3, 2, 2, 3, l2g);
    const int64_t nl = (int64_t)l2g.size();
    std::vector<int64_t> gptr(ng + 1);
    std::vector<int32_t> gidx(nl);
    EXPECT(gs_build_csr(nl, ng, l2g.data(), gptr.data(), gidx.data()), AX_OK);
    CHECK(gptr[0] == 0 && gptr[ng] == nl);
    for (int64_t q = 0; q < ng; ++q)
        for (int64_t r = gptr[q]; r < gptr[q + 1]; ++r) {
            CHECK(l2g[gidx[r]] == q);
            if (r > gptr[q]) CHECK(gidx[r] > gidx[r - 1]);
        }
    std::vector<int32_t> badmap = {0, 5};
    std::vector<int64_t> gp3(4);
    std::vector<int32_t> gi2(2);
    EXPECT(gs_build_csr(2, 3, badmap.data(), gp3.data(), gi2.data()), AX_ERR_ARG);
    EXPECT(gs_assemble(4, 2, nullptr, nullptr, nullptr, nullptr, 9, 1, 0, P(8), P(16), nullptr), AX_ERR_UNSUPPORTED);
    EXPECT(gs_assemble(4, 2, nullptr, nullptr, nullptr, nullptr, GS_QT, 1, 0, P(8), P(16), nullptr), AX_ERR_ARG);
    EXPECT(gs_assemble(-1, 2, nullptr, nullptr, nullptr, nullptr, GS_Q, 1, 0, nullptr, nullptr, nullptr), AX_ERR_ARG);

    // CG and batched workspace sizing (host arithmetic only)
    Gll b7(7);
    ax_problem p{};
    p.E = 32768;
    p.N = 7;
    p.geom = AX_TRILINEAR;
    p.geo = (const double*)P(8);
    p.D = b7.D.data();
    p.xi = b7.xi.data();
    p.w = b7.w.data();
    p.n_global = 225LL * 225 * 225;
    p.l2g = (const int32_t*)P(16);
    p.gptr = (const int64_t*)P(24);
    p.gidx = (const int32_t*)P(32);
    ax_cg_opts o{};
    o.rtol = 1e-10;
    o.max_it = 100;
    o.inner_prec = AX_FP64;
    o.inner_rtol = 0.1;
    o.max_outer = 10;
    o.refine = AX_REFINE_RELIABLE;
    size_t n0 = 0, n1 = 0;
    EXPECT(cg_workspace_bytes(&p, 1, &o, &n0), AX_OK);
    o.precond = AX_PRECOND_JACOBI;
    o.inner_prec = AX_FP32;
    EXPECT(cg_workspace_bytes(&p, 2, &o, &n1), AX_OK);
    CHECK(n1 > n0);
    o.precond = 9;
    EXPECT(cg_workspace_bytes(&p, 1, &o, &n1), AX_ERR_ARG);
    o.precond = AX_PRECOND_NONE;
    o.rtol = 0.0;
    EXPECT(cg_workspace_bytes(&p, 1, &o, &n1), AX_ERR_ARG);
    o.rtol = 1e-10;
    ax_cg_report rep{};
    EXPECT(cg_solve(nullptr, 1, (double*)P(8), (double*)P(16), &o, &rep, nullptr), AX_ERR_ARG);

    std::vector<ax_problem> ms(5);
    std::vector<Gll> bases;
    for (int q = 0; q < 5; ++q) bases.emplace_back(1 + 2 * q % 9);
    for (int q = 0; q < 5; ++q) {
        ms[q] = p;
        ms[q].E = 100 + 37 * q;
        ms[q].N = 1 + 2 * q % 9;
        ms[q].D = bases[q].D.data();
        ms[q].xi = bases[q].xi.data();
        ms[q].w = bases[q].w.data();
    }
    size_t nb = 0;
    EXPECT(ax_batched_workspace_bytes(5, ms.data(), &nb), AX_OK);
    CHECK(nb > 0);
    EXPECT(cg_batched_workspace_bytes(5, ms.data(), 1000, 1, &o, &nb), AX_OK);
    ms[2].N = 10;
    EXPECT(ax_batched_workspace_bytes(5, ms.data(), &nb), AX_ERR_UNSUPPORTED);
    ms[2].N = 5;
    ms[3].geom = AX_PARALLELEPIPED;
    CHECK(ax_batched_workspace_bytes(5, ms.data(), &nb) != AX_OK);
    ms[3].geom = AX_TRILINEAR;
    std::vector<const void*> xs(5, P(64));
    std::vector<void*> ys(5, P(128));
    ax_batch_plan plan{};
    EXPECT(ax_batched_prepare(5, ms.data(), 1, AX_FP64, xs.data(), ys.data(), nullptr, nullptr, 0, &plan), AX_ERR_ARG);
    ax_problem big = ms[0];
    big.E = (int64_t)1 << 30;
    EXPECT(ax_local_batched_noalloc(1, &big, 1, AX_FP64, xs.data(), ys.data(), nullptr, nullptr), AX_ERR_ARG);
    std::vector<ax_problem> many(5000, ms[0]);
    for (auto& m : many) m.E = 0;
    std::vector<const void*> xm(5000, P(64));
    std::vector<void*> ym(5000, P(128));
    EXPECT(ax_local_batched_noalloc(5000, many.data(), 1, AX_FP64, xm.data(), ym.data(), nullptr, nullptr),
           AX_ERR_ARG);

    // probes: validation only
    EXPECT(ax_probe_copy(nullptr, P(16), 64, nullptr), AX_ERR_ARG);
    EXPECT(ax_probe_copy(P(16), P(64), 40, nullptr), AX_ERR_ARG);
    EXPECT(ax_probe_copy(nullptr, nullptr, 0, nullptr), AX_OK);
    double fl = 0;
    EXPECT(ax_probe_compute(0, 0, P(16), &fl, nullptr), AX_ERR_ARG);
    EXPECT(ax_probe_compute(0, 10, nullptr, &fl, nullptr), AX_ERR_ARG);

    std::printf(g_fail ? "abi-sanitize: FAILED\n" : "abi-sanitize: ok\n");
    return g_fail;
}
