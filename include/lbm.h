/*
 * lbm.h -- C-ABI of liblbm: one time step of the D3Q27 central-moment MRT
 * lattice Boltzmann method with immersed-boundary coupling, on one MI355X
 * (gfx950), after Chen, Li, Fan, Liu, "GPU Optimization for High-Quality
 * Kinetic Fluid Simulation" (arXiv:2101.11856).
 *
 * General rules
 *  - Every function has C linkage, returns an lbm_status (except
 *    lbm_destroy / lbm_last_error) and never throws or aborts.
 *  - The library never allocates device memory: the caller passes one device
 *    workspace at create time (size from lbm_workspace_size) and one for the
 *    solid samples (size from lbm_solids_ws_size).  Both stay owned by the
 *    caller and must outlive the context.  The one device memory of the
 *    library's own is a static 64 KiB array per GPU (lbm_conserved_static).
 *  - All work is enqueued on the caller's HIP stream given to lbm_create (or
 *    lbm_set_stream).  Calls marked "sync" wait for that stream; all others are
 *    asynchronous and return after enqueueing.
 *  - Arguments are validated on the host before any launch; a failure returns
 *    LBM_E_INVAL and leaves the state unchanged.  HIP errors map to LBM_E_HIP.
 *    lbm_last_error() gives a message for the last failure on a context.
 *  - "real" below is float, except double when storage == LBM_F64.
 *  - Grid arrays are [nz][ny][nx] with x fastest (linear index
 *    x + nx*(y + ny*z)); vector fields are [3][nz][ny][nx]; population arrays
 *    are [27][nz][ny][nx].  N = nx*ny*nz must stay below 2^31.
 *
 * Lattice (Sec. 3, Eq. 1 and Fig. 1; the values come from the paper's
 * supplementary document, which is not available, so they are this
 * library's reading): c_i in {-1,0,1}^3; index 0 rest, 1-6 faces, 7-18 edges
 * (xy, xz, yz planes), 19-26 corners; inside each group the sign patterns run
 * with x fastest, so c_1 = (1,0,0), c_2 = (-1,0,0), ..., c_26 = (-1,-1,-1).
 * This order reproduces the coefficients printed in the paper's expression
 * for Omega_26 (Sec. 4.4.2) and in Table 2.  Weights 8/27, 2/27, 1/54, 1/216.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_E_INVAL = 1,       /* bad argument, detected before any launch     */
    LBM_E_NOMEM = 2,       /* a caller workspace is too small              */
    LBM_E_HIP = 3,         /* a HIP runtime call failed                    */
    LBM_E_NONFINITE = 4,   /* a check found NaN/Inf in the state           */
    LBM_E_STATE = 5,       /* call made in the wrong order                 */
    LBM_E_UNSUPPORTED = 6  /* valid request this build does not implement  */
} lbm_status;

/* Domain faces, order -x, +x, -y, +y, -z, +z (Sec. 4.3.3: the domain boundary
 * is treated by bounce-back, Alg. 1).  Readings of the face types:
 *  NOSLIP   halfway bounce-back: f*_i(x) = f_opp(i)(x), the opposite
 *           population of the same node as it left the collision.  Alg. 1
 *           prints the copy of the opposite population after streaming,
 *           f*_opp(i)(x); this library takes the traditional scheme that
 *           Sec. 4.3.3 names instead (post-collision value), which keeps the
 *           mass that meets the wall and puts the wall halfway between nodes
 *  INLET    (face -x only) bounce-back with the wall velocity of the inflow:
 *           f*_i(x) = f_opp(i)(x) + 2 w_i rho_w (c_i . u_in(y,z)) / cs^2,
 *           rho_w = 1, cs^2 = 1/3
 *  OUTFLOW  (face +x only) zero gradient: the streamed value is copied from
 *           the node one step inward
 *  FREESLIP specular reflection of the normal velocity component
 *  PERIODIC wrap-around; must be set on both faces of an axis.
 * Where the source x - c_i crosses several faces the rule of the highest
 * precedence applies: NOSLIP > INLET > OUTFLOW > FREESLIP > PERIODIC. */
typedef enum { LBM_PERIODIC = 0, LBM_NOSLIP = 1, LBM_FREESLIP = 2, LBM_INLET = 3, LBM_OUTFLOW = 4 } lbm_face;

/* Population storage.  Every 16-bit and 32-bit form stores the deviation
 * d_i = f_i - w_i from the lattice weights; arithmetic is FP32 except LBM_F64
 * (FP64 storage and arithmetic).  16-bit forms round to nearest even.
 * Measured velocity error against an FP64 reference after 100 steps of 64^3
 * turbulence: FP32 2.4e-7, FP16 2.5e-4, BF16 2.0e-3 -- BF16 (8-bit
 * significand) misses a 1e-3 target; FP16 meets it. */
typedef enum { LBM_F32 = 0, LBM_F16DEV = 1, LBM_BF16DEV = 2, LBM_F64 = 3 } lbm_storage;

/* Collision model of the fused step.  LBM_CM is the paper's central-moment
 * MRT (Sec. 3, Eqs. 4-5).  LBM_BGK and LBM_RMMRT are the comparison models of
 * its Sec. 5.1 (collision-cost figure), which the paper names but does not
 * print; readings: both use the same product-form equilibrium, half-force
 * velocity u = (j + F/2)/rho and Guo forcing as LBM_CM.  LBM_BGK relaxes every
 * population at the one rate s_nu (s_bulk and s_high unused):
 *     f' = f - s_nu (f - f_eq(rho, u)) + (1 - s_nu/2) F . dPhi/du,
 * f_eq = rho Phi(u).  LBM_RMMRT relaxes the moments of the central-moment
 * model's combination basis taken about zero velocity (raw moments) at the
 * same per-group rates.  With all rates equal the three coincide. */
typedef enum { LBM_CM = 0, LBM_BGK = 1, LBM_RMMRT = 2 } lbm_collision;

typedef struct {
    int32_t nx, ny, nz;          /* nodes per axis (>= 1; >= 2 on an axis with a non-periodic face) */
    double nu;                   /* lattice kinematic viscosity > 0; shear rate s_nu = 1/(3 nu + 1/2) (Sec. 3) */
    int32_t face[6];             /* lbm_face codes, -x,+x,-y,+y,-z,+z */
    double u_in[3];              /* uniform inlet velocity used when inlet_profile == NULL */
    const void *inlet_profile;   /* optional device real[3][nz][ny], caller-owned; read at every step */
    double body_force[3];        /* uniform body force density added to every node */
    double s_bulk;               /* relaxation rate of the second-order trace (bulk), 0 < s < 2 */
    double s_high[4];            /* rates of central moments of order 3, 4, 5, 6 (0 < s < 2) */
    int32_t storage;             /* lbm_storage */
    int32_t passive_scalar;      /* 0/1: advect a passive scalar (first-order upwind) */
    int32_t scalar_inlet_height; /* scalar held at 1 on inlet nodes with y < this height */
    int32_t collision;           /* lbm_collision (default LBM_CM) */
} lbm_params;

/* Fill *p with defaults: periodic faces, s_bulk = s_high = 1, FP32, no scalar,
 * central-moment collision. */
lbm_status lbm_default_params(lbm_params *p, int32_t nx, int32_t ny, int32_t nz, double nu);

/* Device bytes the caller must provide to lbm_create for these parameters. */
lbm_status lbm_workspace_size(const lbm_params *p, size_t *bytes);

/* Create a context on the current HIP device.  `workspace` is device memory of
 * at least lbm_workspace_size() bytes (256-byte aligned), `hip_stream` a
 * hipStream_t (NULL = default stream).  The state is zero (f = w) until
 * lbm_init_equilibrium / lbm_set_populations / lbm_restore.  Sync.
 * Storage choices read from the environment at lbm_workspace_size and
 * lbm_create (for measurements; results are the same up to FP32 round-off):
 * LBM_BLOCK_ROWS = rows per population block (0 = plane-major layout; default
 * the largest power of two with at most 2048 padded nodes per block),
 * LBM_POINTER_PATH = 1 stores through plain pointers instead of per-row buffer
 * descriptors, LBM_ROW_STAGE = 0 / 1 disables / forces LDS row staging of the
 * pull (default: FP32 rows that fill one workgroup with periodic x),
 * LBM_CM_GENERAL = 1 keeps the general central-moment collision when the
 * orders 3 to 6 have unit rates (by default a form specialised to unit rates
 * runs, which needs the forward transform only up to order 2),
 * LBM_IB_LANE_PER_RUN = 1 sums the spreading terms of the samples of one
 * cell in one lane instead of the default wavefront scan over one lane per
 * sample (results equal up to FP32 round-off), LBM_FUSED_SPREAD = 0 / 1
 * finishes the spreading in a separate pass / inside the fused kernel (by
 * default the fused kernel does it when the band has at most 2^20 nodes;
 * bit-identical either way), LBM_POSE_NO_WAIT = 1 makes lbm_set_pose place
 * every pose without waiting, also one it cannot show to be inside the
 * domain (a test of the clamping guard and the deferred LBM_E_INVAL
 * described there), LBM_BAND_PUSH = 0 / 1 stops / forces the fused kernel
 * writing, for the next step's band nodes, their streamed sums split by
 * source row, which the band pass then reads instead of pulling 27 scattered
 * values (by default: more than 2^20 band nodes; bit-identical either way).  Keep them unchanged between the two calls. */
lbm_status lbm_create(const lbm_params *p, void *workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out);

lbm_status lbm_set_stream(lbm_ctx *ctx, void *hip_stream);

/* Equilibrium initialisation f_i = f_eq_i(rho, u).  The paper fixes no
 * initial state; this library's reading is the product form
 * rho prod_a phi_{c_ia}(u_a), phi_0 = 2/3 - u^2, phi_{+-1} = (1/3 +- u + u^2)/2,
 * whose central moments are those of the Maxwellian).  rho: device real[N],
 * u: device real[3][N].  Async. */
lbm_status lbm_init_equilibrium(lbm_ctx *ctx, const void *rho, const void *u);

/* Full populations f_i (not deviations) in and out, device real[27][N]. Async. */
lbm_status lbm_set_populations(lbm_ctx *ctx, const void *f);
lbm_status lbm_get_populations(lbm_ctx *ctx, void *f);

/* Passive scalar field in and out, device float[N] (needs passive_scalar). Async. */
lbm_status lbm_set_scalar(lbm_ctx *ctx, const float *s);
lbm_status lbm_get_scalar(lbm_ctx *ctx, float *s);

/* Device bytes of the sample workspace for n samples (lbm_set_solids). */
lbm_status lbm_solids_ws_size(const lbm_ctx *ctx, int64_t n, size_t *bytes);

/* Immersed solid samples (Sec. 3.1).  xyz: device float[3][n] positions in
 * lattice units (node k at coordinate k); ub: device float[3][n] boundary
 * velocity u_b; area: device float[n] area weight a_s of Eq. (8) (NULL = 1);
 * gain: device float[n] penalty gain gamma_s of Eq. (7) (NULL = 1).
 * A sample must lie in [0, n_a) on a periodic axis and in [0, n_a - 1) on an
 * axis with non-periodic faces (its 2x2x2 stencil stays inside).  The samples
 * are sorted (Sec. 4.2.2: l^3 blocks, l = 4, in x-y-z order, Morton order of
 * the position inside a block, original index on ties) and copied into
 * marker_ws (device, caller-owned, lbm_solids_ws_size bytes), so the inputs
 * may be freed afterwards; a body copy in input order stays there for
 * lbm_set_pose.  n = 0 removes all samples.  Sync. */
lbm_status lbm_set_solids(lbm_ctx *ctx, int64_t n, const float *xyz, const float *ub, const float *area,
                          const float *gain, void *marker_ws, size_t marker_ws_bytes);

/* Rigid motion of the samples: the per-step sample update of Alg. 2 (c) for a
 * solid in prescribed motion (the paper's rotating torus and moving airplane;
 * it gives no kinematics rule, so the reading is rigid motion).  The samples
 * of the last lbm_set_solids are body coordinates X_s with body-frame boundary
 * velocity ub_s; this call places them at
 *     x_s = o + R X_s,       u_b = R ub_s + v + w x (x_s - o),
 * R a row-major 3x3 matrix (host), o the body origin, v its velocity and w the
 * angular velocity (host double[3] each, lattice units), then re-sorts the
 * samples and rebuilds the force band as lbm_set_solids does.  x_s is formed
 * in FP64 as o_a + ((R_a0 X + R_a1 Y) + R_a2 Z), one rounding per operation,
 * and rounded to FP32, so the base cells and maps are reproducible; the
 * identity pose (R = I, o = v = w = 0) reproduces lbm_set_solids exactly.
 * o becomes the reference point of lbm_ib_torque.  If a placed sample leaves
 * the domain (same rule as lbm_set_solids) the call returns LBM_E_INVAL and
 * the previous pose stays in force.  Call it before each lbm_step(1) to move
 * the solid every step.  Any adjoint workspace must be bound again
 * (lbm_adjoint_init) afterwards.
 * Waiting: the first call after lbm_set_solids / lbm_set_body takes the
 * body-frame bounding box of the samples (Sync).  A pose for which that box
 * shows on the host that every sample stays inside (interval bounds with a
 * margin far above the placement's rounding) is placed without waiting
 * (Async): the new band and run counts stay on the device, where the kernels
 * of lbm_step read them.  Any other pose first has the device count the
 * samples outside the domain (Sync), which decides the LBM_E_INVAL above.
 * Should a pose placed without waiting still put a sample outside, that
 * sample is clamped into the domain and the next call that waits for the
 * device (lbm_ib_force, lbm_ib_torque, lbm_ib_force_eval, lbm_conserved, an
 * adjoint call, or an lbm_set_pose that waits) returns LBM_E_INVAL. */
lbm_status lbm_set_pose(lbm_ctx *ctx, const double R[9], const double o[3], const double v[3], const double w[3]);

/* lbm_set_solids for a moving solid: X (device float[3][n]) are body
 * coordinates, which need not lie in the domain; the samples are stored and
 * placed at the pose (R, o, v, w) as lbm_set_pose does.  ub, area, gain,
 * marker_ws as for lbm_set_solids.  If a placed sample is outside the domain
 * it returns LBM_E_INVAL and the context has no samples.  Sync. */
lbm_status lbm_set_body(lbm_ctx *ctx, int64_t n, const float *X, const float *ub, const float *area,
                        const float *gain, void *marker_ws, size_t marker_ws_bytes, const double R[9],
                        const double o[3], const double v[3], const double w[3]);

/* Advance n time steps (Alg. 2): for each step, pull streaming with the face
 * rules (Eq. 3), rho and u (Eq. 2), then if samples are set: interpolation
 * and penalty force (Eqs. 6-7) and spreading (Eq. 8) in a deterministic
 * order (the samples of one base cell are summed per stencil offset, then
 * every band node gathers its at most 8 run sums; no floating-point atomics,
 * so repeated runs are bit-identical), then the central-moment collision with
 * force (Eqs. 4-5), stored to the other population buffer.  Async. */
lbm_status lbm_step(lbm_ctx *ctx, int32_t nsteps);

/* rho and u = j / rho (Eq. 2) of the populations that the next step would
 * stream in (a read-only pull of the current state).  rho: device real[N],
 * u: device real[3][N].  Async. */
lbm_status lbm_macros(lbm_ctx *ctx, void *rho, void *u);

/* FP64 totals of the stored populations: out = {sum f, sum c_x f, sum c_y f,
 * sum c_z f} (Eq. 1 conserves them).  Returns LBM_E_NONFINITE if any stored
 * value is NaN or Inf.  Sync. */
lbm_status lbm_conserved(lbm_ctx *ctx, double out[4]);

/* lbm_conserved for callers that cannot allocate device memory at all (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same totals and the same LBM_E_NONFINITE check, computed
 * by the same kernels, but the per-block partial sums, the non-finite counter
 * and the totals live in a library-owned static device array of 64 KiB per
 * GPU (held until the process ends) instead of the context's workspace.  It
 * allocates nothing and calls no allocating routine.  The array of one GPU is
 * shared by every context and stream on it and keeps the last call's
 * contents (the counter is cleared by a kernel at every call), so calls that
 * overlap on one GPU race.  A context whose reduction needs more than the
 * array holds (at most 1024 per-block partials are used, so no valid grid
 * does) gets LBM_E_INVAL.  out: host double[4].  Sync. */
lbm_status lbm_conserved_static(lbm_ctx *ctx, double out[4]);

/* FP64 total sum_s a_s g_s of the penalty force applied in the last step
 * (Alg. 2 (c), total force; Eqs. 7-8 with the area weights): the force on
 * the fluid, so the drag on the solid is its negative.  Sync. */
lbm_status lbm_ib_force(lbm_ctx *ctx, double out[3]);

/* FP64 total torque sum_s (x_s - o) x (a_s g_s) of the penalty forces applied
 * in the last step (Alg. 2 (c)), about the origin o of the current pose (the
 * coordinate origin after lbm_set_solids); the torque on the solid is its
 * negative.  Sync. */
lbm_status lbm_ib_torque(lbm_ctx *ctx, double out[3]);

/* FP64 total penalty force that the next step would apply, evaluated from the
 * current state without changing it.  Sync. */
lbm_status lbm_ib_force_eval(lbm_ctx *ctx, double out[3]);

/* Integer maps of the samples (bit-exact).  flags: device uint8[N], bit 0 =
 * node inside some sample's 2x2x2 stencil (receives force), bit 1 = base cell
 * floor(x_s) of some sample; marker_cell: device int32[n], linear index of the
 * base cell of sample s (input order); marker_perm: device int32[n], input
 * index of the k-th sample in sorted order.  Any pointer may be NULL.  Async. */
lbm_status lbm_solid_maps(lbm_ctx *ctx, uint8_t *flags, int32_t *marker_cell, int32_t *marker_perm);

/* Snapshot of the state (populations and scalar) into / from device memory of
 * lbm_state_bytes() bytes, caller-owned.  The bytes are the internal storage
 * (population deviations in the blocked layout, in the storage type): opaque,
 * and valid only for a context created with the same parameters.  Async. */
lbm_status lbm_state_bytes(const lbm_ctx *ctx, size_t *bytes);
lbm_status lbm_checkpoint(lbm_ctx *ctx, void *dst);
lbm_status lbm_restore(lbm_ctx *ctx, const void *src);

/* Replace the penalty gains gamma_s of the current samples (device float[n],
 * input order) without re-sorting; later poses keep them.  Async. */
lbm_status lbm_set_gains(lbm_ctx *ctx, const float *gain);

/* ---- adjoint (reverse mode of lbm_step) ----------------------------------
 * The adjoint state lambda = dJ/df has the layout of the populations, in the
 * arithmetic type (float, double for LBM_F64), and lives in a caller-owned
 * adjoint workspace.  Gradients accumulate in FP64.  Reading of the paper: the
 * objective depends on the final state only (drag from lbm_ib_force_eval,
 * velocities from lbm_macros), so the reverse sweep starts from seeds on that
 * state and walks the steps backwards over a tape of forward states.  The
 * tape holds states, not sample placements: every taped step is
 * differentiated with the samples where they are when lbm_adjoint_step runs,
 * so a solid moved by lbm_set_pose during the taped steps is not supported. */

/* Device bytes of the adjoint workspace for the current grid and samples. */
lbm_status lbm_adjoint_ws_size(const lbm_ctx *ctx, size_t *bytes);

/* Bind the adjoint workspace (device, 256-byte aligned) and set lambda = 0.
 * Must be called again after lbm_set_solids or lbm_set_pose.  The adjoint
 * differentiates the central-moment collision: a context with another
 * collision model returns LBM_E_UNSUPPORTED.  Async. */
lbm_status lbm_adjoint_init(lbm_ctx *ctx, void *adj_ws, size_t bytes);

/* lambda += (d(rho, u0)/df)^T (g_rho, g_u) for the lbm_macros outputs of the
 * current state (Eq. 2 after the pull).  g_rho: device real[N] or NULL;
 * g_u: device real[3][N] or NULL; g_inlet: device double[3][nz][ny] (+=) for
 * dJ/du_in, or NULL.  Async. */
lbm_status lbm_adjoint_seed_macros(lbm_ctx *ctx, const void *g_rho, const void *g_u, double *g_inlet);

/* lambda += (dF/df)^T g_force for the penalty force F = lbm_ib_force_eval of
 * the current state (Eqs. 6-8); g_gain: device double[n] (+=, input order)
 * receives dF/dgamma . g_force, or NULL.  Async. */
lbm_status lbm_adjoint_seed_force(lbm_ctx *ctx, const double g_force[3], double *g_inlet, double *g_gain);

/* Advance nsteps forward (as lbm_step), leaving the state before step k in
 * tape + k * lbm_state_bytes (device, caller-owned, nsteps slots).  When the
 * tape and the slot size are 256-byte aligned, step k reads slot k and writes
 * slot k + 1 directly (one state copy per call); otherwise each slot is copied
 * before its step.  The results are the same bits either way.  Async. */
lbm_status lbm_record_tape(lbm_ctx *ctx, int32_t nsteps, void *tape);

/* Reverse sweep over a tape of nsteps forward states (as written by
 * lbm_record_tape): for k = nsteps-1 .. 0, lambda <- (df(k+1)/df(k))^T lambda,
 * with f(k) read from the tape.  g_inlet (double[3][nz][ny]) and g_gain
 * (double[n], input order) accumulate dJ/du_in and dJ/dgamma; either may be
 * NULL.  The context's own population state is not touched.  Async. */
lbm_status lbm_adjoint_step(lbm_ctx *ctx, int32_t nsteps, const void *tape, double *g_inlet, double *g_gain);

/* lambda out of / into a dense device real[27][N] array.  Async. */
lbm_status lbm_adjoint_get(lbm_ctx *ctx, void *lambda);
lbm_status lbm_adjoint_set(lbm_ctx *ctx, const void *lambda);

/* Release the host-side context (the workspaces stay with the caller). */
void lbm_destroy(lbm_ctx *ctx);

/* Message of the last failure on ctx (or of the last failed lbm_create when
 * ctx is NULL); never NULL. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Library version string. */
const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
