// Error reporting, version and the GLL tables of the library (host code).
#include <cmath>
#include <cstring>

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
static TuneEntry g_tune[kMaxN1 + 1][3][2];
static bool g_tune_init = false;

static void tune_init()
{
    if (g_tune_init) return;
    for (auto& a : g_tune)
        for (auto& b : a)
            for (auto& c : b) c = TuneEntry{0, 2};
    g_tune_init = true;
}

TuneEntry tune_get(int N1, int geo_kind, int prec)
{
    tune_init();
    if (N1 < 2 || N1 > kMaxN1 || geo_kind < 0 || geo_kind > 2 || prec < 0 || prec > 1) return TuneEntry{0, 2};
    return g_tune[N1][geo_kind][prec];
}

static int epb_of(int N1, bool alt)
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

}  // namespace ax

using namespace ax;

extern "C" int ax_tune_set(int N, int geom_kind, int prec, int epb_alt, int grid_mult)
{
    clear_error();
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (geom_kind < 0 || geom_kind > 2) return fail(AX_ERR_ARG, "geometry kind %d", geom_kind);
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_ARG, "precision %d (FP64 or FP32)", prec);
    if ((epb_alt != 0 && epb_alt != 1) || grid_mult < 1 || grid_mult > 64)
        return fail(AX_ERR_ARG, "epb_alt must be 0/1 and grid_mult in [1,64]");
    tune_init();
    g_tune[N + 1][geom_kind][prec] = TuneEntry{epb_alt, grid_mult};
    return AX_OK;
}

extern "C" int ax_tune_get(int N, int geom_kind, int prec, int* epb_alt, int* grid_mult, int* elems_per_group)
{
    clear_error();
    if (N < 1 || N > 15) return fail(AX_ERR_UNSUPPORTED, "order N=%d outside [1,15]", N);
    if (geom_kind < 0 || geom_kind > 2) return fail(AX_ERR_ARG, "geometry kind %d", geom_kind);
    if (prec != AX_FP64 && prec != AX_FP32) return fail(AX_ERR_ARG, "precision %d (FP64 or FP32)", prec);
    const TuneEntry t = tune_get(N + 1, geom_kind, prec);
    if (epb_alt) *epb_alt = t.epb_alt;
    if (grid_mult) *grid_mult = t.grid_mult;
    if (elems_per_group) *elems_per_group = epb_of(N + 1, t.epb_alt != 0);
    return AX_OK;
}

extern "C" const char* ax_last_error(void) { return g_err; }

extern "C" const char* ax_version(void) { return "axhosfem 0.1 (gfx950)"; }

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
