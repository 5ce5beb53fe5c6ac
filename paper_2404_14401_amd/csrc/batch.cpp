// batch.cpp -- batched and adjoint entry points (placeholders until implemented).
#include <hip/hip_runtime.h>

#include "../../include/gpe.h"

extern "C" {

int gpe_batch_create(gpe_batch **out, int n, const gpe_plan_desc *descs, const gpe_potential_desc *pots)
{
    (void)n; (void)descs; (void)pots;
    if (out) *out = nullptr;
    return GPE_ERR_UNSUPPORTED;
}

int gpe_batch_destroy(gpe_batch *b) { (void)b; return GPE_OK; }

int gpe_step_batched(gpe_batch *b, gpe_c64 *const *psis, int64_t nsteps, double t0)
{
    (void)b; (void)psis; (void)nsteps; (void)t0;
    return GPE_ERR_UNSUPPORTED;
}

int gpe_adjoint(gpe_batch *b, const gpe_c64 *const *psi0, const gpe_c64 *const *target, int64_t nsteps, double t0,
                const double *knots, int nknots, int loss_kind, int mode, double drift_tol, double *loss,
                double *grad, gpe_c64 *const *psi_final, double *info)
{
    (void)b; (void)psi0; (void)target; (void)nsteps; (void)t0; (void)knots; (void)nknots; (void)loss_kind;
    (void)mode; (void)drift_tol; (void)loss; (void)grad; (void)psi_final; (void)info;
    return GPE_ERR_UNSUPPORTED;
}

}
