// lbm_step_inst.hip -- the per-step kernels for one population storage form
// (LBM_STEP_ST, an lbm_storage code) and one collision model (LBM_STEP_COLL,
// a COLL_* code of lbm_internal.hpp).  The build compiles this file once per
// pair, so the kernel variants compile in parallel; the band pre-pass and the
// immersed-boundary kernels come with the central-moment unit of each form.
#include "lbm_step.hpp"

#if !defined(LBM_STEP_ST) || !defined(LBM_STEP_COLL)
#error "compile with -DLBM_STEP_ST=<storage> -DLBM_STEP_COLL=<model>"
#endif

namespace lbm {
template hipError_t fused_st<LBM_STEP_ST, LBM_STEP_COLL>(lbm_ctx *c);
#if LBM_STEP_COLL == 0
template hipError_t band_ib_st<LBM_STEP_ST>(lbm_ctx *c, const void *state, double *ftot, bool spread, bool pieces);
#endif
}  // namespace lbm
