// Conjugate gradients on the assembled operator (placeholder; implemented below in a later step).
#include "ax_internal.h"

extern "C" int cg_workspace_bytes(const ax_problem*, int, const ax_cg_opts*, size_t* bytes)
{
    ax::clear_error();
    if (bytes) *bytes = 0;
    return ax::fail(AX_ERR_UNSUPPORTED, "cg_solve not available yet");
}

extern "C" int cg_solve(const ax_problem*, int, const double*, double*, const ax_cg_opts*,
                        ax_cg_report*, void*)
{
    ax::clear_error();
    return ax::fail(AX_ERR_UNSUPPORTED, "cg_solve not available yet");
}
