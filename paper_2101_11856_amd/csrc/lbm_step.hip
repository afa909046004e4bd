// lbm_step.hip -- dispatch of the per-step kernels by storage form and
// collision model (the kernels are in lbm_step.hpp, instantiated per pair by
// lbm_step_inst.hip).
#include "lbm_ctx.hpp"

namespace lbm {

template <int ST, int COLL> hipError_t fused_st(lbm_ctx *c);
template <int ST> hipError_t band_ib_st(lbm_ctx *c, const void *state, double *ftot, bool spread);

template <int ST> static hipError_t fused_model(lbm_ctx *c)
{
    switch (c->coll) {
    case COLL_CM: return fused_st<ST, COLL_CM>(c);
    case COLL_CM_UNIT_HIGH: return fused_st<ST, COLL_CM_UNIT_HIGH>(c);
    case COLL_BGK: return fused_st<ST, COLL_BGK>(c);
    case COLL_RM: return fused_st<ST, COLL_RM>(c);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fused(lbm_ctx *c)
{
    switch (c->p.storage) {
    case LBM_F32: return fused_model<LBM_F32>(c);
    case LBM_F16DEV: return fused_model<LBM_F16DEV>(c);
    case LBM_BF16DEV: return fused_model<LBM_BF16DEV>(c);
    case LBM_F64: return fused_model<LBM_F64>(c);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_band_ib(lbm_ctx *c, const void *state, double *ftot, bool spread)
{
    if (c->nm <= 0) return hipSuccess;
    switch (c->p.storage) {
    case LBM_F32: return band_ib_st<LBM_F32>(c, state, ftot, spread);
    case LBM_F16DEV: return band_ib_st<LBM_F16DEV>(c, state, ftot, spread);
    case LBM_BF16DEV: return band_ib_st<LBM_BF16DEV>(c, state, ftot, spread);
    case LBM_F64: return band_ib_st<LBM_F64>(c, state, ftot, spread);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
