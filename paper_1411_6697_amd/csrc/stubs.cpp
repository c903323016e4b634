// Entry points whose kernels are not built yet.
#include "lbkm_abi_internal.h"
using namespace lbkm;
namespace lbkm { void destroy_extras(lbkm_ctx*) {} }
extern "C" {
lbkm_status lbkm_adjoint_step(lbkm_ctx* c, const double*, const double*, const double*, const double*, double*, double*, double*) { return fail(c, LBKM_ESTATE, "adjoint not built"); }
lbkm_status lbkm_adjoint_init(lbkm_ctx* c, const double*, const double*, const double*, const double*, const double*, double*, double*, double*, double*) { return fail(c, LBKM_ESTATE, "adjoint not built"); }
lbkm_status lbkm_tne_loss(lbkm_ctx* c, const double*, double*, double*) { return fail(c, LBKM_ESTATE, "not built"); }
lbkm_status lbkm_batch_create(int32_t, const int32_t*, const lbkm_grid*, void*, lbkm_ctx** out) { if (out) *out = nullptr; return LBKM_ESTATE; }
lbkm_status lbkm_batch_set_params(lbkm_ctx* c, const double*, const double*, double, double, const lbkm_rates*) { return fail(c, LBKM_ESTATE, "batch not built"); }
lbkm_status lbkm_batch_init_fields(lbkm_ctx* c, const double*, const double*, const double*, const double*, const double*) { return fail(c, LBKM_ESTATE, "batch not built"); }
lbkm_status lbkm_batch_autotune(lbkm_ctx* c, int32_t*) { return fail(c, LBKM_ESTATE, "batch not built"); }
lbkm_status lbkm_batch_step(lbkm_ctx* c, int64_t) { return fail(c, LBKM_ESTATE, "batch not built"); }
lbkm_status lbkm_batch_get_moments(lbkm_ctx* c, double*, double*, double*, double*, double*, double*) { return fail(c, LBKM_ESTATE, "batch not built"); }
lbkm_status lbkm_batch_total_cells(lbkm_ctx* c, int64_t*) { return fail(c, LBKM_ESTATE, "batch not built"); }
}
