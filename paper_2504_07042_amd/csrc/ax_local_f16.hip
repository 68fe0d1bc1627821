// FP16-operand / FP32-accumulate AxLocal (matrix cores).  Placeholder until implemented.
#include "ax_internal.h"

namespace ax {

int ax_local_f16(int64_t, int, int, const double*, const float*, const double*, const double*,
                 const double*, int, const float*, float*, hipStream_t)
{
    return fail(AX_ERR_UNSUPPORTED, "AX_FP16_ACC32 is not available yet");
}

}  // namespace ax
