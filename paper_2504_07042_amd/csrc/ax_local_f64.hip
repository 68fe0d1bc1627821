// AxLocal kernels instantiated for double arithmetic.
#include "ax_local_impl.h"

namespace ax {

int axl_dispatch_f64(int geo_kind, int N, int64_t E, int nrhs, const double* geo, const double* Gs,
                      const double* X, double* Y, const double* D, const double* xi, const double* w,
                      hipStream_t st, const int32_t* l2g, int64_t ldg, int64_t es, int64_t ccs, FusedOut* fo)
{
    switch (geo_kind) {
    case GEO_TRI: return dispatch<GEO_TRI, double>(N, E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
    case GEO_PARA: return dispatch<GEO_PARA, double>(N, E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
    case GEO_TRIL: return dispatch<GEO_TRIL, double>(N, E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
    case GEO_HELM: return dispatch<GEO_HELM, double>(N, E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
    default: return dispatch<GEO_STORED, double>(N, E, nrhs, geo, Gs, X, Y, D, xi, w, st, l2g, ldg, es, ccs, fo);
    }
}

}  // namespace ax
