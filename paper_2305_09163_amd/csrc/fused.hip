// Fused right-hand side (placeholder until the LDS-tiled kernel lands).
#include "internal.h"

namespace mfc {

int launch_rhs_fused(mfc_grid *, const double *, const double *, double *, int, double, const double *, hipStream_t)
{
    return fail(MFC_E_UNSUPPORTED, "fused kernel not built yet; use MFC_KERNEL_STAGED");
}

}  // namespace mfc
