// Right preconditioners for the GMRES solve (placeholder until the learned and
// block-Jacobi preconditioners are built).
#include "internal.h"

namespace rbf {

int pc_ready(rbf_plan *p, int kind) {
    (void)p;
    set_error("rbf_interp_solve: preconditioner %d is not available in this build", kind);
    return RBF_EUNSUPPORTED;
}

int pc_apply(rbf_plan *p, const double *v, double *z) {
    (void)p; (void)v; (void)z;
    set_error("rbf_interp_solve: no preconditioner loaded");
    return RBF_ESTATE;
}

}  // namespace rbf
