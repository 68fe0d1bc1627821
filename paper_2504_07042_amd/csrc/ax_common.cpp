// Error reporting, version and the GLL tables of the library (host code).
#include <cmath>
#include <cstring>
#include <mutex>

#include "ax_internal.h"
#include "ax_kernels.h"

namespace ax {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

// Legendre L_n(x) and L_n'(x) by the three-term recurrence.
static void legendre(int n, double x, double& L, double& dL)
{
    double pm1 = 1.0, p = x, dpm1 = 0.0, dp = 1.0;
    if (n == 0) {
        L = 1.0;
        dL = 0.0;
        return;
    }
    for (int m = 1; m < n; ++m) {
        const double pn = ((2 * m + 1) * x * p - m * pm1) / (m + 1);
        const double dpn = dpm1 + (2 * m + 1) * p;  // L'_{m+1} = L'_{m-1} + (2m+1) L_m
        pm1 = p;
        p = pn;
        dpm1 = dp;
        dp = dpn;
    }
    L = p;
    dL = dp;
}

// Process-wide launch tuning table (filled by ax_tune_set, e.g. from the autotuner's cache).
constexpr TuneEntry kTuneDefault{AX_KERNEL_AUTO, 0, 0, 0, 2};
static TuneEntry g_tune[kMaxN1 + 1][TUNE_KINDS][2];
static std::once_flag g_tune_once;

static void tune_init()
{
    std::call_once(g_tune_once, [] {
        for (auto& a : g_tune)
            for (auto& b : a)
                for (auto& c : b) c = kTuneDefault;
    });
}

TuneEntry tune_get(int N1, int kind, int prec)
{
    tune_init();
    if (N1 < 2 || N1 > kMaxN1 || kind < 0 || kind >= TUNE_KINDS || prec < 0 || prec > 1) return kTuneDefault;
    return g_tune[N1][kind][prec];
}

static int tile_epb(int N1, bool alt)
{
    switch (N1) {
#define AX_E(n) \
    case n: return alt ? Shape<n>::EPB_ALT : Shape<n>::EPB;
        AX_E(2) AX_E(3) AX_E(4) AX_E(5) AX_E(6) AX_E(7) AX_E(8) AX_E(9) AX_E(10) AX_E(11) AX_E(12) AX_E(13)
        AX_E(14) AX_E(15) AX_E(16)
#undef AX_E
    default: return 1;
    }
}

static int tune_check(int N, int kind, int prec)
{
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (kind < 0 || kind >= TUNE_KINDS) return fail(AX_ERR_ARG, "tuning kind %d", kind);
    if (kind == TUNE_BATCHED && N > 9) return fail(AX_ERR_ARG, "batched launches take N <= 9");
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_ARG, "precision %d (FP64 or FP32)", prec);
    return AX_OK;
}

}  // namespace ax

using namespace ax;

extern "C" int ax_tune_set(int N, int kind, int prec, const ax_tune* t)
{
    clear_error();
    AX_TRY(tune_check(N, kind, prec));
    if (!t) return fail(AX_ERR_ARG, "t is NULL");
    if (t->kernel < AX_KERNEL_AUTO || t->kernel > AX_KERNEL_ITEM) return fail(AX_ERR_ARG, "kernel %d", t->kernel);
    if ((t->tile_alt | t->item_alt | t->waves_alt) & ~1)
        return fail(AX_ERR_ARG, "tile_alt, item_alt and waves_alt must be 0 or 1");
    if (t->grid_mult < 1 || t->grid_mult > 64) return fail(AX_ERR_ARG, "grid_mult %d outside [1,64]", t->grid_mult);
    tune_init();
    g_tune[N + 1][kind][prec] = TuneEntry{t->kernel, t->tile_alt, t->item_alt, t->waves_alt, t->grid_mult};
    return AX_OK;
}

extern "C" int ax_tune_get(int N, int kind, int prec, ax_tune* t)
{
    clear_error();
    AX_TRY(tune_check(N, kind, prec));
    if (!t) return fail(AX_ERR_ARG, "t is NULL");
    const int N1 = N + 1;
    const bool fp32 = prec == AX_FP32;
    const TuneEntry e = tune_get(N1, kind, prec);
    const int geo = (kind == TUNE_TRI || kind == TUNE_BATCHED) ? GEO_TRI : kind == TUNE_PARTIAL ? GEO_TRIL
                  : kind == TUNE_PARA ? GEO_PARA : kind == TUNE_STORED ? GEO_STORED : GEO_HELM;
    // the batched kernels: the per-item kernel unless the entry asks for the tile kernel (it takes
    // the default tile shape; tile_alt 0 walks the work list where the order has that form,
    // tile_alt 1 gives each work-group a slice of one mesh)
    const bool item = kind == TUNE_BATCHED
                          ? !(e.kernel == AX_KERNEL_TILE && (e.tile_alt != 0 || batched_tile_available(N1, fp32)))
                          : (item_available(N1, geo) &&
                             (e.kernel == AX_KERNEL_ITEM || (e.kernel == AX_KERNEL_AUTO && item_default(N1, geo, fp32))));
    *t = ax_tune{e.kernel, e.tile_alt, e.item_alt, e.waves_alt, e.grid_mult, 0, 0, 0, 0};
    t->kernel_used = item ? AX_KERNEL_ITEM : AX_KERNEL_TILE;
    if (item) {
        const ItemShape sh = item_shape(N1, item_has_alt(N1) ? e.item_alt : 0);
        t->elems_per_group = sh.epb;
        t->block = sh.block;
        t->waves = kind == TUNE_BATCHED ? batch_waves(fp32) : item_waves(N1, fp32, geo == GEO_TRIL, e.waves_alt);
    } else {
        t->elems_per_group = tile_epb(N1, kind != TUNE_BATCHED && e.tile_alt != 0);
        t->block = ((t->elems_per_group * N1 * N1 + 63) / 64) * 64;
        t->waves = tile_waves(N1, geo, fp32);
    }
    return AX_OK;
}

extern "C" const char* ax_last_error(void) { return g_err; }

extern "C" const char* ax_version(void) { return "axhosfem 0.2 (gfx950)"; }

// GLL tables (Sec. 2.1, Table 1).  The interior points are the zeros of q(x) = (1-x^2) L_N'(x);
// Newton's method uses q'(x) = -N(N+1) L_N(x) (Legendre's equation), started from the
// Chebyshev-Gauss-Lobatto points.
extern "C" int ax_gll(int N, double* xi, double* w, double* D)
{
    clear_error();
    if (N < 1 || N > 31) return fail(AX_ERR_UNSUPPORTED, "ax_gll: N=%d outside [1,31]", N);
    if (!xi || !w || !D) return fail(AX_ERR_ARG, "ax_gll: NULL output");
    const int N1 = N + 1;
    const double nn = double(N) * (N + 1);
    for (int i = 0; i < N1; ++i) {
        if (i == 0 || i == N) {
            xi[i] = (i == 0) ? -1.0 : 1.0;
            continue;
        }
        double x = -std::cos(M_PI * i / N);
        for (int it = 0; it < 100; ++it) {
            double L, dL;
            legendre(N, x, L, dL);
            const double q = (1.0 - x * x) * dL;
            const double dq = -nn * L;
            const double step = q / dq;
            x -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        xi[i] = x;
    }
    for (int i = 0; i < N1 / 2; ++i) {  // enforce the symmetry of the point set
        const double m = 0.5 * (xi[N - i] - xi[i]);
        xi[i] = -m;
        xi[N - i] = m;
    }
    if (N1 % 2) xi[N / 2] = 0.0;
    double Lx[32];
    for (int i = 0; i < N1; ++i) {
        double L, dL;
        legendre(N, xi[i], L, dL);
        Lx[i] = L;
        w[i] = 2.0 / (nn * L * L);
    }
    for (int i = 0; i < N1; ++i) {
        double off = 0.0;
        for (int j = 0; j < N1; ++j) {
            if (j == i) continue;
            const double v = Lx[i] / (Lx[j] * (xi[i] - xi[j]));
            D[i * N1 + j] = v;
            off += v;
        }
        D[i * N1 + i] = -off;
    }
    return AX_OK;
}
