// Batched persistent AxLocal over many meshes (placeholder; implemented in a later step).
#include "ax_internal.h"

extern "C" int ax_batched_workspace_bytes(int, const ax_problem*, size_t* bytes)
{
    ax::clear_error();
    if (bytes) *bytes = 0;
    return ax::fail(AX_ERR_UNSUPPORTED, "batched AxLocal not available yet");
}

extern "C" int ax_local_batched(int, const ax_problem*, int, int, const void* const*, void* const*,
                                void*, size_t, void*)
{
    ax::clear_error();
    return ax::fail(AX_ERR_UNSUPPORTED, "batched AxLocal not available yet");
}
