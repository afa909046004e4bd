// lbm_step.hip -- dispatch of the per-step kernels by storage form and
// collision model (the kernels are in lbm_step.hpp, instantiated per pair by
// lbm_step_inst.hip).
#include "lbm_ctx.hpp"

namespace lbm {

template <int ST, int COLL> hipError_t fused_st(lbm_ctx *c);
template <int ST> hipError_t band_ib_st(lbm_ctx *c, const void *state, double *ftot, bool spread, bool pieces);

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

// Bit r of feeds[w]: the tile of wavefront w's segment in row r = 3 (dz + 1) +
// dy + 1 of its 9 rows (y+dy, z+dz) is away from the y and z faces and holds
// band nodes.  Once per band; the fused kernel loads one word per wavefront
// and the others (most of them) skip the pieces.
__global__ void __launch_bounds__(256)
    k_push_feeds(Geom g, const uint64_t *__restrict__ tile_mask, uint32_t *__restrict__ feeds)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= g.W) return;
    const int64_t row = w / g.ntx;
    const int y = (int)(row % g.ny), z = (int)(row / g.ny);
    uint32_t f = 0;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        if (y + dy < 1 || y + dy > g.ny - 2 || z + dz < 1 || z + dz > g.nz - 2) continue;
        if (tile_mask[w + ((int64_t)dz * g.ny + dy) * g.ntx] != 0) f |= 1u << r;
    }
    feeds[w] = f;
}

hipError_t launch_push_feeds(lbm_ctx *c)
{
    const unsigned nb = (unsigned)((c->g.W + 255) / 256);
    hipLaunchKernelGGL(k_push_feeds, dim3(nb), dim3(256), 0, c->stream, c->g, c->tile_mask, c->push_feeds);
    return hipGetLastError();
}

hipError_t launch_band_ib(lbm_ctx *c, const void *state, double *ftot, bool spread, bool pieces)
{
    if (c->nm <= 0) return hipSuccess;
    switch (c->p.storage) {
    case LBM_F32: return band_ib_st<LBM_F32>(c, state, ftot, spread, pieces);
    case LBM_F16DEV: return band_ib_st<LBM_F16DEV>(c, state, ftot, spread, pieces);
    case LBM_BF16DEV: return band_ib_st<LBM_BF16DEV>(c, state, ftot, spread, pieces);
    case LBM_F64: return band_ib_st<LBM_F64>(c, state, ftot, spread, pieces);
    }
    return hipErrorInvalidValue;
}

}  // namespace lbm
