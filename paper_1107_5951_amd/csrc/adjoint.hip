// Adjoint (transpose) evaluation.
#include "eval_common.hpp"

using namespace grav;

extern "C" grav_status grav_adjoint(grav_plan_t plan, const double *resid, double *drho_out,
                                    void *stream)
{
    (void)stream;
    if (!plan || !resid || !drho_out)
        return GRAV_EINVAL;
    return GRAV_EUNSUPPORTED;
}
