// Entry points whose kernels are not built yet.
#include "lbkm_abi_internal.h"
using namespace lbkm;
extern "C" {
lbkm_status lbkm_adjoint_step(lbkm_ctx* c, const double*, const double*, const double*, const double*, double*, double*, double*) { return fail(c, LBKM_ESTATE, "adjoint not built"); }
lbkm_status lbkm_adjoint_init(lbkm_ctx* c, const double*, const double*, const double*, const double*, const double*, double*, double*, double*, double*) { return fail(c, LBKM_ESTATE, "adjoint not built"); }
lbkm_status lbkm_tne_loss(lbkm_ctx* c, const double*, double*, double*) { return fail(c, LBKM_ESTATE, "not built"); }
}
