// Single-mesh per-item AxLocal kernels, FP64: every order and both run-time variants (see item.h).
#include "item.h"

namespace ax {

int tri_item_dispatch_f64(int N1, int64_t E, int nrhs, const double* verts, const double* X, double* Y,
                          const Basis<double>& bs, int grid_mult, int variant, int waves, hipStream_t st,
                          const double* lam, int64_t es, int64_t ccs)
{
    return tri_item_dispatch<double>(N1, E, nrhs, verts, X, Y, bs, grid_mult, variant, waves, st, lam, es, ccs);
}

}  // namespace ax
