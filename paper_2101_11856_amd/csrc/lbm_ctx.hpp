// lbm_ctx.hpp -- host-side context of liblbm and the launchers each kernel
// translation unit provides.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "lbm.h"
#include "lbm_internal.hpp"

struct lbm_ctx {
    lbm_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    lbm::Geom g{};
    int64_t N = 0;         // nx*ny*nz
    int64_t rows = 0;      // ny*nz
    size_t esize = 4;      // bytes per stored population
    size_t rsize = 4;      // bytes of the arithmetic type
    bool buffer_path = false;  // fused kernel stores through per-row buffer descriptors
    bool load32 = false;       // with buffer_path: interior loads by 32-bit offsets from a per-wave base
    uint32_t span32 = 0;       // bytes that cover the 9 source rows from the lowest one
    bool row_stage = false;    // fused kernel stages whole rows in LDS (segments per row == waves per block, periodic x)
    int coll = 0;              // collision variant of the fused kernel (COLL_* of lbm_internal.hpp)
    // caller workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *fA = nullptr, *fB = nullptr;  // fA = current state
    float *scA = nullptr, *scB = nullptr;
    double *red_part = nullptr;  // [red_blocks][4]
    int *red_flag = nullptr;     // non-finite count
    double *red_out = nullptr;   // [4]
    double *ftot = nullptr;      // [6] IB force and torque of the last step
    double *ftot_eval = nullptr; // [6] IB force and torque evaluated by lbm_ib_force_eval
    int red_blocks = 0;
    // relaxation rates
    double s_nu = 1, s_b = 1, s_h[4] = {1, 1, 1, 1};
    // solid samples (marker workspace, caller-owned)
    int64_t nm = 0;
    int64_t nband = 0;             // band nodes: exact when counts_exact, else the last count read (a launch hint)
    int64_t nbcap = 0;             // band capacity of the marker workspace (stride of band_src)
    bool counts_exact = true;      // nband and nruns match the device counts
    bool pose_pending = false;     // a pose placed without waiting: its out-of-domain count is still unread
    bool pose_no_wait = false;     // LBM_POSE_NO_WAIT: place every pose without waiting (guard test)
    int32_t *dcounts = nullptr;    // device {band nodes, runs} of the last set-up
    int *dbad = nullptr;           // device count of samples placed outside the domain
    int box_state = 0;             // body-frame bounding box: 0 not taken, 1 valid, -1 non-finite samples
    double box_lo[3] = {0, 0, 0}, box_hi[3] = {0, 0, 0};
    char *mws = nullptr;
    size_t mws_bytes = 0;
    float *m_pos = nullptr, *m_ub = nullptr, *m_area = nullptr, *m_gain = nullptr;  // sorted order
    int32_t *m_slot = nullptr;     // [8][nm] band slot of each stencil node
    int32_t *m_cell = nullptr;     // [nm] base cell, input order (one of two buffers)
    int32_t *m_cell_next = nullptr;// [nm] the other buffer, written by the next placement
    float *b_xyz = nullptr, *b_ub = nullptr, *b_area = nullptr, *b_gain = nullptr;  // body samples, input order
    float *w_xyz = nullptr, *w_ub = nullptr;  // placed samples, input order (staging for a new pose)
    double pose_o[3] = {0, 0, 0};  // reference point of the torque (the pose origin)
    int32_t *m_perm = nullptr;     // [nm] input index of sorted sample k
    uint64_t *tile_mask = nullptr; // [W]
    int32_t *tile_start = nullptr; // [W]
    int32_t *band_cell = nullptr;  // [nband]
    void *band_ru = nullptr;       // [nband] real4 (rho, u)
    void *band_force = nullptr;    // [nband] real4 (g, 0)
    double *ib_part = nullptr;     // [ceil(nruns/256)][8] per-block force and torque partials
    int64_t nruns = 0;             // runs: samples of one base cell, cut at every 64 sorted samples (as nband)
    int32_t *run_start = nullptr;  // [nruns + 1] first sorted sample of each run
    int32_t *run_id = nullptr;     // [nm] run of each sorted sample
    uint8_t *run_cont = nullptr;   // [nruns + 1] 1 if the run continues the cell of the run before it (last: 0)
    bool ib_lane_per_run = false;  // spreading sums by one lane per run instead of the wavefront scan
    int spread_mode = -1;          // -1: by band size (fused_spread()), 0: k_spread pass, 1: in the fused kernel
    void *run_sum = nullptr;       // [8][nm] real4: a K_d g summed over run r (r < nruns), per stencil offset d
    int32_t *band_src = nullptr;   // [8][nbcap] run feeding band node j (j < nband) through offset d, or -1
    void *band_push = nullptr;     // [9][nbcap] real pairs: band pieces of the state in fA (band_push_on)
    int push_mode = -1;            // -1: by band size (band_push_on()), 0: never, 1: always
    bool push_valid = false;       // band_push holds the pieces of the state in fA for the current band
    uint32_t *push_feeds = nullptr;// [W] rows of the band each wavefront of the fused kernel feeds
    bool feeds_valid = false;      // push_feeds describes the current band
    // adjoint workspace (caller-owned)
    char *aws = nullptr;
    size_t aws_bytes = 0;
    int64_t adj_band_cap = -1;     // band capacity the adjoint workspace was sized for (-1 = unbound)
    // real planes like the populations: lam = dJ/df (or, while adj_pending,
    // only its face-rule part), adjM = mu of the last reverse step, adjM2 the next
    void *lam = nullptr, *adjM = nullptr, *adjM2 = nullptr;
    bool adj_pending = false;      // lambda = (plain pulls transposed)(adjM) + lam, not yet formed
    void *band_phi = nullptr;      // [nband] real4 adjoint of the band force
    void *band_bar = nullptr;      // [nband] real4 adjoint of (rho, u0) at band nodes
    std::string err;
};

namespace lbm {

// Whether the step's fused kernel finishes the spreading itself (each band
// lane gathers its run sums) instead of a separate k_spread pass.  Measured
// on MI355X: the gather pays on small bands, where k_spread is one more
// latency-bound launch (dense sphere, 9.4k band nodes: 0.349 -> 0.338 ms per
// step), and costs on large ones, where it lengthens the waves of every band
// tile (city, 7.16M band nodes: 11.22 -> 11.50 ms).
constexpr int64_t FUSED_SPREAD_MAX_BAND = int64_t(1) << 20;
inline bool fused_spread(const lbm_ctx *c)
{
    return c->spread_mode >= 0 ? c->spread_mode == 1 : c->nband <= FUSED_SPREAD_MAX_BAND;
}

// Whether the fused kernel writes the band pieces of the state it produces,
// for the next step's band pre-pass to read instead of pulling.  Measured on
// MI355X (city, 7.16M band nodes, one box, three runs): FP32 10.91-10.96 ->
// 10.44-10.48 ms per step (the pre-pass 0.86 -> 0.17 ms), FP16 7.34-7.69 ->
// 7.12-7.34 ms.  On small bands the pre-pass is a few microseconds anyway.  So:
// bands above 2^20 nodes, unless LBM_BAND_PUSH = 0 / 1 forces it.
constexpr int64_t BAND_PUSH_MIN_BAND = int64_t(1) << 20;
inline bool band_push_on(const lbm_ctx *c)
{
    if (c->nm <= 0 || !c->band_push) return false;
    if (c->push_mode >= 0) return c->push_mode == 1;
    return c->nband > BAND_PUSH_MIN_BAND;
}

// Marker workspace carve-up, shared by the size query and lbm_set_solids.
struct SolidsLayout {
    size_t pos, ub, area, gain, slot, cell, cell2, perm, keys, tkk, tb, bcount, bstart, big, occ;
    size_t tile_mask, tile_start, tile_count, scan_tmp, scan_tmp_bytes, band_cell, band_ru, band_force, ib_part, misc;
    size_t run_head, run_id, run_start, run_cont, run_sum, band_src, band_push, push_feeds;
    size_t body_xyz, body_ub, body_area, body_gain, world_xyz, world_ub;
    size_t total;
};
hipError_t solids_layout(const lbm_ctx *c, int64_t n, SolidsLayout *L);
// most band nodes n samples can mark (the stride of band_src)
int64_t band_capacity(const lbm_ctx *c, int64_t n);

// launchers (return the first HIP error)
hipError_t launch_fused(lbm_ctx *c);
// the fused kernel's per-wavefront rows of the band it feeds (push_feeds)
hipError_t launch_push_feeds(lbm_ctx *c);
// band pull + interpolation/spreading of `state`; `spread` = also finish the
// band forces (k_spread) rather than leave that to the fused kernel
// `pieces`: read the band pieces the last fused kernel wrote instead of pulling
hipError_t launch_band_ib(lbm_ctx *c, const void *state, double *ftot, bool spread = true, bool pieces = false);
hipError_t launch_init_eq(lbm_ctx *c, const void *rho, const void *u);
hipError_t launch_set_pop(lbm_ctx *c, const void *f);
hipError_t launch_get_pop(lbm_ctx *c, void *f);
hipError_t launch_macros(lbm_ctx *c, void *rho, void *u);
hipError_t launch_conserved(lbm_ctx *c);
// lbm_conserved_static: the same reduction with its partials, counter and
// totals in the library's static scratch array of this GPU (no workspace use)
constexpr int MAX_RED_BLOCKS = 1024;                    // per-block partials of the conservation totals
constexpr size_t STATIC_SCRATCH_BYTES = 64 * 1024;      // static scratch array per GPU
size_t conserved_static_need(const lbm_ctx *c);
hipError_t launch_conserved_static(lbm_ctx *c, double out[4], int *flag);
hipError_t launch_copy(lbm_ctx *c, void *dst, const void *src, size_t bytes);
hipError_t launch_zero(lbm_ctx *c, void *dst, size_t bytes);
hipError_t launch_scalar_io(lbm_ctx *c, float *dst, const float *src, bool to_state);
// Sample set-up (keys, sort, band, slots, runs) of n samples at xyz.  wait:
// read the count of samples outside the domain (and stop if it is not zero)
// and the band and run counts back, else leave them on the device.
hipError_t solids_setup(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area, const float *gain,
                        bool wait, int *bad_count_host);
hipError_t read_counts(lbm_ctx *c);
// body-frame bounding box of the samples (box_lo, box_hi, box_state); waits
hipError_t body_box(lbm_ctx *c);
// body copy of the caller's samples (lbm_set_solids) and a rigid placement of them (lbm_set_pose)
hipError_t solids_store_body(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area,
                             const float *gain);
hipError_t solids_pose(lbm_ctx *c, const double R[9], const double o[3], const double v[3], const double w[3],
                       bool wait, int *bad_count_host);
hipError_t launch_solid_maps(lbm_ctx *c, uint8_t *flags, int32_t *cell, int32_t *perm);
hipError_t launch_set_gains(lbm_ctx *c, const float *gain);

// adjoint (lbm_adjoint.hip)
size_t adjoint_ws_bytes(const lbm_ctx *c);
void adjoint_bind(lbm_ctx *c, void *ws, size_t bytes);
hipError_t adjoint_step_one(lbm_ctx *c, const void *state, double *g_inlet, double *g_gain);
hipError_t adjoint_seed_macros(lbm_ctx *c, const void *g_rho, const void *g_u, double *g_inlet);
hipError_t adjoint_seed_force(lbm_ctx *c, const double g_force[3], double *g_inlet, double *g_gain);
hipError_t adjoint_io(lbm_ctx *c, void *dense, bool to_state);

}  // namespace lbm
