// lbm_api.hip -- the extern "C" surface of liblbm (include/lbm.h): argument
// validation on the host, carving of the caller's workspaces, and launch
// sequencing on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "lbm_ctx.hpp"

using namespace lbm;

namespace {

std::string g_create_err = "no error";

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

lbm_status fail(lbm_ctx *c, lbm_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_create_err = msg;
    return s;
}

lbm_status hip_fail(lbm_ctx *c, hipError_t e, const char *where)
{
    return fail(c, LBM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

bool valid_rate(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

// Rows per population block (a power of two): the largest with at most
// BLOCK_NODES padded nodes per block, at least 1, at most the row count.
// LBM_BLOCK_ROWS overrides it for measurements (0 = plain plane-major layout).
constexpr int64_t BLOCK_NODES = 2048;
int block_log2_rows(int64_t rows, int64_t nxp)
{
    int64_t want = -1;
    if (const char *e = std::getenv("LBM_BLOCK_ROWS")) want = std::strtol(e, nullptr, 10);
    if (want == 0) return 31;
    int lr = 0;
    if (want > 0) {
        while ((int64_t(2) << lr) <= want && (int64_t(2) << lr) <= rows) ++lr;
        return lr;
    }
    while ((int64_t(2) << lr) * nxp <= BLOCK_NODES && (int64_t(2) << lr) <= rows) ++lr;
    return lr;
}

lbm_status validate(const lbm_params *p, std::string &err)
{
    if (!p) return err = "params is NULL", LBM_E_INVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return err = "grid dimensions must be >= 1", LBM_E_INVAL;
    const int64_t nxp = (int64_t)align_up((size_t)p->nx, 32);
    if ((int64_t)p->nx * p->ny * p->nz >= (1ll << 31) || nxp * p->ny * p->nz >= (1ll << 31))
        return err = "grid too large: nx*ny*nz (padded) must stay below 2^31", LBM_E_INVAL;
    if (!std::isfinite(p->nu) || !(p->nu > 0.0)) return err = "nu must be finite and > 0", LBM_E_INVAL;
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int f = 0; f < 6; ++f)
        if (p->face[f] < LBM_PERIODIC || p->face[f] > LBM_OUTFLOW) return err = "unknown face code", LBM_E_INVAL;
    for (int a = 0; a < 3; ++a) {
        const bool pm = p->face[2 * a] == LBM_PERIODIC, pp = p->face[2 * a + 1] == LBM_PERIODIC;
        if (pm != pp) return err = "PERIODIC must be set on both faces of an axis", LBM_E_INVAL;
        if (!pm && n[a] < 2) return err = "an axis with non-periodic faces needs >= 2 nodes", LBM_E_INVAL;
    }
    for (int f = 0; f < 6; ++f) {
        if (p->face[f] == LBM_INLET && f != 0) return err = "INLET is supported on face -x only", LBM_E_INVAL;
        if (p->face[f] == LBM_OUTFLOW && f != 1) return err = "OUTFLOW is supported on face +x only", LBM_E_INVAL;
    }
    if (!valid_rate(p->s_bulk)) return err = "s_bulk must be in (0, 2)", LBM_E_INVAL;
    for (int k = 0; k < 4; ++k)
        if (!valid_rate(p->s_high[k])) return err = "s_high rates must be in (0, 2)", LBM_E_INVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->u_in[a]) || !std::isfinite(p->body_force[a]))
            return err = "u_in and body_force must be finite", LBM_E_INVAL;
    if (p->storage < LBM_F32 || p->storage > LBM_F64) return err = "unknown storage", LBM_E_INVAL;
    if (p->passive_scalar != 0 && p->passive_scalar != 1) return err = "passive_scalar must be 0 or 1", LBM_E_INVAL;
    if (p->collision < LBM_CM || p->collision > LBM_RMMRT) return err = "unknown collision model", LBM_E_INVAL;
    return LBM_OK;
}

struct Layout {
    int nxp, ntx, lr;
    int64_t plane, bstride, pop_elems, W, rows;
    size_t esize, rsize;
    size_t offA, offB, offSA, offSB, offPart, offOut, offFt, offFe, offFlag, total;
    int red_blocks;
};

Layout layout(const lbm_params *p)
{
    Layout L{};
    L.nxp = (int)align_up((size_t)p->nx, 32);
    L.ntx = (p->nx + SEG - 1) / SEG;
    L.rows = (int64_t)p->ny * p->nz;
    L.W = (int64_t)L.ntx * L.rows;
    L.lr = block_log2_rows(L.rows, L.nxp);
    if (L.lr == 31) {
        L.plane = (int64_t)align_up((size_t)(L.rows * L.nxp), 64);
        L.bstride = 0;
        L.pop_elems = (int64_t)Q * L.plane;
    } else {
        const int64_t R = int64_t(1) << L.lr;
        L.plane = R * L.nxp;
        L.bstride = (int64_t)Q * L.plane;
        L.pop_elems = ((L.rows + R - 1) >> L.lr) * L.bstride;
    }
    L.esize = p->storage == LBM_F32 ? 4 : p->storage == LBM_F64 ? 8 : 2;
    L.rsize = p->storage == LBM_F64 ? 8 : 4;
    const int64_t N = (int64_t)p->nx * p->ny * p->nz;
    L.red_blocks = (int)std::min<int64_t>(MAX_RED_BLOCKS, std::max<int64_t>(1, (N + 255) / 256));
    const size_t fbytes = align_up((size_t)L.pop_elems * L.esize, ALIGN);
    const size_t sbytes = p->passive_scalar ? align_up((size_t)L.rows * L.nxp * 4, ALIGN) : 0;
    size_t o = 0;
    L.offA = o;
    o += fbytes;
    L.offB = o;
    o += fbytes;
    L.offSA = o;
    o += sbytes;
    L.offSB = o;
    o += sbytes;
    L.offPart = o;
    o += align_up((size_t)L.red_blocks * 4 * 8, ALIGN);
    L.offOut = o;
    o += ALIGN;
    L.offFt = o;
    o += ALIGN;
    L.offFe = o;
    o += ALIGN;
    L.offFlag = o;
    o += ALIGN;
    L.total = o;
    return L;
}

size_t state_bytes(const lbm_ctx *c)
{
    size_t b = (size_t)c->g.total * c->esize;
    if (c->p.passive_scalar) b += (size_t)c->rows * c->g.nxp * 4;
    return b;
}

#define CHECK_CTX(c)                                                             \
    do {                                                                         \
        if (!(c)) return fail(nullptr, LBM_E_INVAL, "context is NULL");          \
    } while (0)
#define HIP_TRY(c, expr, where)                                                  \
    do {                                                                         \
        const hipError_t e_ = (expr);                                            \
        if (e_ != hipSuccess) return hip_fail((c), e_, (where));                 \
    } while (0)

}  // namespace

extern "C" {

lbm_status lbm_default_params(lbm_params *p, int32_t nx, int32_t ny, int32_t nz, double nu)
{
    if (!p) return fail(nullptr, LBM_E_INVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->nx = nx;
    p->ny = ny;
    p->nz = nz;
    p->nu = nu;
    p->s_bulk = 1.0;
    for (int k = 0; k < 4; ++k) p->s_high[k] = 1.0;
    p->storage = LBM_F32;
    return LBM_OK;
}

lbm_status lbm_workspace_size(const lbm_params *p, size_t *bytes)
{
    std::string err;
    const lbm_status s = validate(p, err);
    if (s != LBM_OK) return fail(nullptr, s, err);
    if (!bytes) return fail(nullptr, LBM_E_INVAL, "bytes is NULL");
    *bytes = layout(p).total;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params *p, void *workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out)
{
    std::string err;
    lbm_status s = validate(p, err);
    if (s != LBM_OK) return fail(nullptr, s, err);
    if (!out) return fail(nullptr, LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!workspace) return fail(nullptr, LBM_E_INVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % ALIGN)
        return fail(nullptr, LBM_E_INVAL, "workspace must be 256-byte aligned");
    const Layout L = layout(p);
    if (ws_bytes < L.total)
        return fail(nullptr, LBM_E_NOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_E_NOMEM, "host allocation failed");
    c->p = *p;
    c->stream = static_cast<hipStream_t>(hip_stream);
    (void)hipGetDevice(&c->device);
    c->g.nx = p->nx;
    c->g.ny = p->ny;
    c->g.nz = p->nz;
    c->g.nxp = L.nxp;
    c->g.ntx = L.ntx;
    c->g.lr = L.lr;
    c->g.rmask = L.lr == 31 ? (int64_t)0x7fffffff : (int64_t(1) << L.lr) - 1;
    c->g.plane = L.plane;
    c->g.bstride = L.bstride;
    c->g.total = L.pop_elems;
    c->g.dntx = make_divisor((uint32_t)L.ntx);
    c->g.dny = make_divisor((uint32_t)p->ny);
    c->g.W = L.W;
    for (int f = 0; f < 6; ++f) c->g.face[f] = p->face[f];
    c->N = (int64_t)p->nx * p->ny * p->nz;
    c->rows = L.rows;
    c->esize = L.esize;
    c->rsize = L.rsize;
    // per-row buffer descriptors for the fused kernel's stores when the 27
    // populations of a row span less than 2^31 bytes (always for the blocked
    // layout; FP64 keeps pointers); LBM_POINTER_PATH=1 forces pointers
    {
        const char *e = std::getenv("LBM_POINTER_PATH");
        const bool force_ptr = e && std::strtol(e, nullptr, 10) != 0;
        c->buffer_path = !force_ptr && p->storage != LBM_F64 &&
                         (uint64_t)Q * (uint64_t)L.plane * L.esize < (uint64_t(1) << 31);
        // interior loads by 32-bit offsets from each wavefront's lowest source
        // row (blocked layout): rows (z-1, y-1) .. (z+1, y+1) span 2 ny + 3
        // rows, i.e. at most (2 ny + 2) / R + 2 blocks, which must stay below
        // 2^31 bytes (LBM_BUF_LOADS=0 keeps pointer loads)
        const char *bl = std::getenv("LBM_BUF_LOADS");
        const uint64_t rpb = uint64_t(1) << (L.lr < 31 ? L.lr : 0);
        const uint64_t span = ((2 * (uint64_t)p->ny + 2) / rpb + 2) * (uint64_t)L.bstride * L.esize;
        c->load32 = c->buffer_path && L.lr < 31 && !(bl && std::strtol(bl, nullptr, 10) == 0) &&
                    span < (uint64_t(1) << 31);
        c->span32 = c->load32 ? (uint32_t)span : 0u;
        // LDS row staging: one workgroup per row, periodic x, FP32 storage (measured at 256^3:
        // 0.6% faster in FP32, 5.6% slower in the ALU-bound 16-bit forms); LBM_ROW_STAGE=0
        // disables it, =1 also enables it for 16-bit storage (measurements and tests)
        const char *r = std::getenv("LBM_ROW_STAGE");
        const long rs = r ? std::strtol(r, nullptr, 10) : -1;
        c->row_stage = rs != 0 && L.ntx == WAVES_PER_BLOCK && p->face[0] == LBM_PERIODIC &&
                       (p->storage == LBM_F32 || rs == 1);
        // collision variant: the central-moment form specialised to unit
        // rates of orders 3 to 6 when they are (LBM_CM_GENERAL=1 keeps the
        // general form, for measurements)
        const char *g = std::getenv("LBM_CM_GENERAL");
        const bool general = g && std::strtol(g, nullptr, 10) != 0;
        const bool unit_high = p->s_high[0] == 1.0 && p->s_high[1] == 1.0 && p->s_high[2] == 1.0 && p->s_high[3] == 1.0;
        c->coll = p->collision == LBM_BGK     ? COLL_BGK
                  : p->collision == LBM_RMMRT ? COLL_RM
                  : (unit_high && !general)   ? COLL_CM_UNIT_HIGH
                                              : COLL_CM;
        // spreading sums: wavefront scan, one lane per sample (default), or
        // one lane per run with LBM_IB_LANE_PER_RUN=1 (for measurements)
        const char *ib = std::getenv("LBM_IB_LANE_PER_RUN");
        c->ib_lane_per_run = ib && std::strtol(ib, nullptr, 10) != 0;
        // spreading finished by the fused kernel's band lanes or by a
        // k_spread pass: chosen by band size (fused_spread()) unless
        // LBM_FUSED_SPREAD = 0 / 1 forces one (for measurements)
        const char *fs = std::getenv("LBM_FUSED_SPREAD");
        c->spread_mode = fs ? (std::strtol(fs, nullptr, 10) != 0 ? 1 : 0) : -1;
        // every pose placed without waiting, shown inside or not (a test of the
        // device's clamping guard and of the deferred LBM_E_INVAL)
        const char *pw = std::getenv("LBM_POSE_NO_WAIT");
        c->pose_no_wait = pw && std::strtol(pw, nullptr, 10) != 0;
        // band pieces written by the fused kernel: by band size
        // (band_push_on()) unless LBM_BAND_PUSH = 0 / 1 forces it
        const char *bp = std::getenv("LBM_BAND_PUSH");
        c->push_mode = bp ? (std::strtol(bp, nullptr, 10) != 0 ? 1 : 0) : -1;
    }
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = ws_bytes;
    c->fA = c->ws + L.offA;
    c->fB = c->ws + L.offB;
    if (p->passive_scalar) {
        c->scA = reinterpret_cast<float *>(c->ws + L.offSA);
        c->scB = reinterpret_cast<float *>(c->ws + L.offSB);
    }
    c->red_part = reinterpret_cast<double *>(c->ws + L.offPart);
    c->red_out = reinterpret_cast<double *>(c->ws + L.offOut);
    c->ftot = reinterpret_cast<double *>(c->ws + L.offFt);
    c->ftot_eval = reinterpret_cast<double *>(c->ws + L.offFe);
    c->red_flag = reinterpret_cast<int *>(c->ws + L.offFlag);
    c->red_blocks = L.red_blocks;
    c->s_nu = 1.0 / (3.0 * p->nu + 0.5);
    c->s_b = p->s_bulk;
    for (int k = 0; k < 4; ++k) c->s_h[k] = p->s_high[k];
    // state f = w (zero deviations), zero scalar and force totals
    hipError_t e = launch_zero(c, c->ws, L.offPart);
    if (e == hipSuccess) e = launch_zero(c, c->ws + L.offOut, L.total - L.offOut);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_create_err = std::string("lbm_create: ") + hipGetErrorString(e);
        delete c;
        return LBM_E_HIP;
    }
    *out = c;
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_ctx *c, void *hip_stream)
{
    CHECK_CTX(c);
    c->stream = static_cast<hipStream_t>(hip_stream);
    return LBM_OK;
}

lbm_status lbm_init_equilibrium(lbm_ctx *c, const void *rho, const void *u)
{
    CHECK_CTX(c);
    if (!rho || !u) return fail(c, LBM_E_INVAL, "rho and u must be non-NULL");
    c->push_valid = false;
    HIP_TRY(c, launch_init_eq(c, rho, u), "lbm_init_equilibrium");
    return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx *c, const void *f)
{
    CHECK_CTX(c);
    if (!f) return fail(c, LBM_E_INVAL, "f is NULL");
    c->push_valid = false;
    HIP_TRY(c, launch_set_pop(c, f), "lbm_set_populations");
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx *c, void *f)
{
    CHECK_CTX(c);
    if (!f) return fail(c, LBM_E_INVAL, "f is NULL");
    HIP_TRY(c, launch_get_pop(c, f), "lbm_get_populations");
    return LBM_OK;
}

lbm_status lbm_set_scalar(lbm_ctx *c, const float *s)
{
    CHECK_CTX(c);
    if (!c->p.passive_scalar) return fail(c, LBM_E_STATE, "context was created without a passive scalar");
    if (!s) return fail(c, LBM_E_INVAL, "s is NULL");
    HIP_TRY(c, launch_scalar_io(c, c->scA, s, true), "lbm_set_scalar");
    return LBM_OK;
}

lbm_status lbm_get_scalar(lbm_ctx *c, float *s)
{
    CHECK_CTX(c);
    if (!c->p.passive_scalar) return fail(c, LBM_E_STATE, "context was created without a passive scalar");
    if (!s) return fail(c, LBM_E_INVAL, "s is NULL");
    HIP_TRY(c, launch_scalar_io(c, s, c->scA, false), "lbm_get_scalar");
    return LBM_OK;
}

lbm_status lbm_solids_ws_size(const lbm_ctx *c, int64_t n, size_t *bytes)
{
    if (!c) return fail(nullptr, LBM_E_INVAL, "context is NULL");
    if (n < 0 || n >= (1ll << 31) || !bytes) return fail(const_cast<lbm_ctx *>(c), LBM_E_INVAL, "bad sample count");
    SolidsLayout L;
    const hipError_t e = solids_layout(c, n, &L);
    if (e != hipSuccess) return hip_fail(const_cast<lbm_ctx *>(c), e, "lbm_solids_ws_size");
    *bytes = L.total;
    return LBM_OK;
}

static bool finite_pose(const double R[9], const double o[3], const double v[3], const double w[3])
{
    for (int k = 0; k < 9; ++k)
        if (!std::isfinite(R[k])) return false;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(o[a]) || !std::isfinite(v[a]) || !std::isfinite(w[a])) return false;
    return true;
}

// Shared by lbm_set_solids (R == NULL: the samples are placed as given) and
// lbm_set_body (the samples are body coordinates, placed at the pose).
static lbm_status set_samples(lbm_ctx *c, const char *who, int64_t n, const float *xyz, const float *ub,
                              const float *area, const float *gain, void *marker_ws, size_t marker_ws_bytes,
                              const double *R, const double *o, const double *v, const double *w)
{
    if (n < 0 || n >= (1ll << 31)) return fail(c, LBM_E_INVAL, "sample count out of range");
    c->pose_o[0] = c->pose_o[1] = c->pose_o[2] = 0.0;
    if (n == 0) {
        c->nm = 0;
        c->nband = 0;
        HIP_TRY(c, launch_zero(c, c->ftot, 6 * sizeof(double)), who);
        return LBM_OK;
    }
    if (!xyz) return fail(c, LBM_E_INVAL, "xyz is NULL");
    if (R && !finite_pose(R, o, v, w)) return fail(c, LBM_E_INVAL, "R, o, v and w must be finite");
    if (!marker_ws || reinterpret_cast<uintptr_t>(marker_ws) % ALIGN)
        return fail(c, LBM_E_INVAL, "marker_ws must be non-NULL and 256-byte aligned");
    SolidsLayout L;
    hipError_t e = solids_layout(c, n, &L);
    if (e != hipSuccess) return hip_fail(c, e, who);
    if (marker_ws_bytes < L.total)
        return fail(c, LBM_E_NOMEM, "marker workspace too small: need " + std::to_string(L.total) + " bytes");
    c->nm = 0;
    c->nband = 0;
    c->counts_exact = true;
    c->pose_pending = false;
    c->mws = static_cast<char *>(marker_ws);
    c->mws_bytes = marker_ws_bytes;
    int bad = 0;
    e = solids_store_body(c, n, xyz, ub, area, gain);
    if (e == hipSuccess) {
        if (R) {
            c->nm = n;  // solids_pose places the c->nm body samples
            e = solids_pose(c, R, o, v, w, true, &bad);
            if (e != hipSuccess || bad) c->nm = 0;
        } else {
            e = solids_setup(c, n, c->b_xyz, c->b_ub, c->b_area, c->b_gain, true, &bad);
        }
    }
    if (e != hipSuccess) return hip_fail(c, e, who);
    if (bad) {
        return fail(c, LBM_E_INVAL,
                    std::to_string(bad) + (R ? " placed" : "") +
                        " sample(s) outside the domain (need [0,n) on periodic axes, [0,n-1) on bounded axes)");
    }
    c->nm = n;
    if (R)
        for (int a = 0; a < 3; ++a) c->pose_o[a] = o[a];
    return LBM_OK;
}

lbm_status lbm_set_solids(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area,
                          const float *gain, void *marker_ws, size_t marker_ws_bytes)
{
    CHECK_CTX(c);
    return set_samples(c, "lbm_set_solids", n, xyz, ub, area, gain, marker_ws, marker_ws_bytes, nullptr, nullptr,
                       nullptr, nullptr);
}

lbm_status lbm_set_body(lbm_ctx *c, int64_t n, const float *X, const float *ub, const float *area, const float *gain,
                        void *marker_ws, size_t marker_ws_bytes, const double R[9], const double o[3],
                        const double v[3], const double w[3])
{
    CHECK_CTX(c);
    if (!R || !o || !v || !w) return fail(c, LBM_E_INVAL, "R, o, v and w must be non-NULL");
    return set_samples(c, "lbm_set_body", n, X, ub, area, gain, marker_ws, marker_ws_bytes, R, o, v, w);
}

// Whether every sample placed at (R, o) is inside the domain, shown from the
// body-frame bounding box (pose_inside_box); false when that cannot be shown
// (the device then counts the samples outside).
static bool pose_inside(const lbm_ctx *c, const double R[9], const double o[3])
{
    if (c->box_state != 1) return false;
    const int n[3] = {c->g.nx, c->g.ny, c->g.nz};
    double top[3];
    for (int a = 0; a < 3; ++a) top[a] = c->g.face[2 * a] == LBM_PERIODIC ? n[a] : n[a] - 1;
    return pose_inside_box(R, o, c->box_lo, c->box_hi, top);
}

// Reads the device counts of a set-up that did not wait for them and, for a
// pose placed without waiting, its count of samples outside the domain
// (which the host bound makes zero; a nonzero count is reported here).
static lbm_status settle_counts(lbm_ctx *c, const char *who)
{
    if (c->nm == 0 || (c->counts_exact && !c->pose_pending)) return LBM_OK;
    int bad = 0;
    HIP_TRY(c, hipMemcpyAsync(&bad, c->dbad, sizeof(int), hipMemcpyDeviceToHost, c->stream), who);
    HIP_TRY(c, read_counts(c), who);
    const bool pending = c->pose_pending;
    c->pose_pending = false;
    if (pending && bad) {
        HIP_TRY(c, launch_zero(c, c->dbad, sizeof(int)), who);
        return fail(c, LBM_E_INVAL,
                    std::to_string(bad) + " sample(s) of an earlier pose were placed outside the domain and clamped");
    }
    return LBM_OK;
}

lbm_status lbm_set_pose(lbm_ctx *c, const double R[9], const double o[3], const double v[3], const double w[3])
{
    CHECK_CTX(c);
    if (!R || !o || !v || !w) return fail(c, LBM_E_INVAL, "R, o, v and w must be non-NULL");
    if (!finite_pose(R, o, v, w)) return fail(c, LBM_E_INVAL, "R, o, v and w must be finite");
    if (c->nm == 0) return fail(c, LBM_E_STATE, "no solid samples (lbm_set_solids)");
    if (c->box_state == 0) HIP_TRY(c, body_box(c), "lbm_set_pose");
    // Shown inside on the host: no wait (the set-up runs behind the caller's
    // queue).  Otherwise the device counts the samples outside first.
    const bool inside = c->pose_no_wait || pose_inside(c, R, o);
    if (!inside) {
        const lbm_status st = settle_counts(c, "lbm_set_pose");
        if (st != LBM_OK) return st;
    }
    int bad = 0;
    const hipError_t e = solids_pose(c, R, o, v, w, !inside, &bad);
    if (e != hipSuccess) return hip_fail(c, e, "lbm_set_pose");
    if (inside) c->pose_pending = true;
    if (bad) {
        return fail(c, LBM_E_INVAL,
                    std::to_string(bad) +
                        " placed sample(s) outside the domain (need [0,n) on periodic axes, [0,n-1) on bounded "
                        "axes); the previous pose stays");
    }
    for (int a = 0; a < 3; ++a) c->pose_o[a] = o[a];
    return LBM_OK;
}

// one step from (fA, scA) into (fB, scB), without the swap.  The band
// pre-pass reads the band pieces when the fused kernel that wrote fA left them
// for the current band; the fused kernel leaves them for the next step.
static hipError_t one_step(lbm_ctx *c)
{
    const bool push = band_push_on(c);
    if (c->nm > 0) {
        const hipError_t e = launch_band_ib(c, c->fA, c->ftot, !fused_spread(c), push && c->push_valid);
        if (e != hipSuccess) return e;
    }
    c->push_valid = false;
    if (push && !c->feeds_valid) {
        const hipError_t e = launch_push_feeds(c);
        if (e != hipSuccess) return e;
        c->feeds_valid = true;
    }
    const hipError_t e = launch_fused(c);
    if (e == hipSuccess) c->push_valid = push;
    return e;
}

lbm_status lbm_step(lbm_ctx *c, int32_t nsteps)
{
    CHECK_CTX(c);
    if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps must be >= 0");
    for (int32_t t = 0; t < nsteps; ++t) {
        HIP_TRY(c, one_step(c), "lbm_step");
        std::swap(c->fA, c->fB);
        std::swap(c->scA, c->scB);
    }
    return LBM_OK;
}

lbm_status lbm_macros(lbm_ctx *c, void *rho, void *u)
{
    CHECK_CTX(c);
    if (!rho || !u) return fail(c, LBM_E_INVAL, "rho and u must be non-NULL");
    HIP_TRY(c, launch_macros(c, rho, u), "lbm_macros");
    return LBM_OK;
}

lbm_status lbm_conserved(lbm_ctx *c, double out[4])
{
    CHECK_CTX(c);
    if (!out) return fail(c, LBM_E_INVAL, "out is NULL");
    const lbm_status st = settle_counts(c, "lbm_conserved");
    if (st != LBM_OK) return st;
    HIP_TRY(c, launch_conserved(c), "lbm_conserved");
    int flag = 0;
    HIP_TRY(c, hipMemcpyAsync(out, c->red_out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "lbm_conserved");
    HIP_TRY(c, hipMemcpyAsync(&flag, c->red_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "lbm_conserved");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "lbm_conserved");
    if (flag) return fail(c, LBM_E_NONFINITE, "non-finite populations in the state");
    return LBM_OK;
}

lbm_status lbm_conserved_static(lbm_ctx *c, double out[4])
{
    CHECK_CTX(c);
    if (!out) return fail(c, LBM_E_INVAL, "out is NULL");
    const size_t need = conserved_static_need(c);
    if (need > STATIC_SCRATCH_BYTES)
        return fail(c, LBM_E_INVAL,
                    "lbm_conserved_static: the reduction needs " + std::to_string(need) +
                        " bytes of scratch, more than the static array's " + std::to_string(STATIC_SCRATCH_BYTES));
    int flag = 0;
    HIP_TRY(c, launch_conserved_static(c, out, &flag), "lbm_conserved_static");
    if (flag) return fail(c, LBM_E_NONFINITE, "non-finite populations in the state");
    return LBM_OK;
}

lbm_status lbm_ib_force(lbm_ctx *c, double out[3])
{
    CHECK_CTX(c);
    if (!out) return fail(c, LBM_E_INVAL, "out is NULL");
    const lbm_status st = settle_counts(c, "lbm_ib_force");
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(out, c->ftot, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "lbm_ib_force");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "lbm_ib_force");
    return LBM_OK;
}

lbm_status lbm_ib_torque(lbm_ctx *c, double out[3])
{
    CHECK_CTX(c);
    if (!out) return fail(c, LBM_E_INVAL, "out is NULL");
    const lbm_status st = settle_counts(c, "lbm_ib_torque");
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipMemcpyAsync(out, c->ftot + 3, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "lbm_ib_torque");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "lbm_ib_torque");
    return LBM_OK;
}

lbm_status lbm_ib_force_eval(lbm_ctx *c, double out[3])
{
    CHECK_CTX(c);
    if (!out) return fail(c, LBM_E_INVAL, "out is NULL");
    if (c->nm == 0) {
        out[0] = out[1] = out[2] = 0.0;
        return LBM_OK;
    }
    const lbm_status st = settle_counts(c, "lbm_ib_force_eval");
    if (st != LBM_OK) return st;
    HIP_TRY(c, launch_band_ib(c, c->fA, c->ftot_eval), "lbm_ib_force_eval");
    HIP_TRY(c, hipMemcpyAsync(out, c->ftot_eval, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
            "lbm_ib_force_eval");
    HIP_TRY(c, hipStreamSynchronize(c->stream), "lbm_ib_force_eval");
    return LBM_OK;
}

lbm_status lbm_solid_maps(lbm_ctx *c, uint8_t *flags, int32_t *marker_cell, int32_t *marker_perm)
{
    CHECK_CTX(c);
    HIP_TRY(c, launch_solid_maps(c, flags, marker_cell, marker_perm), "lbm_solid_maps");
    return LBM_OK;
}

lbm_status lbm_state_bytes(const lbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(const_cast<lbm_ctx *>(c), LBM_E_INVAL, "NULL argument");
    *bytes = state_bytes(c);
    return LBM_OK;
}

lbm_status lbm_checkpoint(lbm_ctx *c, void *dst)
{
    CHECK_CTX(c);
    if (!dst) return fail(c, LBM_E_INVAL, "dst is NULL");
    const size_t fb = (size_t)c->g.total * c->esize;
    HIP_TRY(c, launch_copy(c, dst, c->fA, fb), "lbm_checkpoint");
    if (c->p.passive_scalar)
        HIP_TRY(c, launch_copy(c, static_cast<char *>(dst) + fb, c->scA, (size_t)c->rows * c->g.nxp * 4),
                "lbm_checkpoint");
    return LBM_OK;
}

lbm_status lbm_restore(lbm_ctx *c, const void *src)
{
    CHECK_CTX(c);
    if (!src) return fail(c, LBM_E_INVAL, "src is NULL");
    const size_t fb = (size_t)c->g.total * c->esize;
    c->push_valid = false;
    HIP_TRY(c, launch_copy(c, c->fA, src, fb), "lbm_restore");
    if (c->p.passive_scalar)
        HIP_TRY(c, launch_copy(c, c->scA, static_cast<const char *>(src) + fb, (size_t)c->rows * c->g.nxp * 4),
                "lbm_restore");
    return LBM_OK;
}

lbm_status lbm_set_gains(lbm_ctx *c, const float *gain)
{
    CHECK_CTX(c);
    if (c->nm == 0) return fail(c, LBM_E_STATE, "no samples are set");
    if (!gain) return fail(c, LBM_E_INVAL, "gain is NULL");
    HIP_TRY(c, launch_set_gains(c, gain), "lbm_set_gains");
    return LBM_OK;
}

lbm_status lbm_record_tape(lbm_ctx *c, int32_t nsteps, void *tape)
{
    CHECK_CTX(c);
    if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps must be >= 0");
    if (nsteps > 0 && !tape) return fail(c, LBM_E_INVAL, "tape is NULL");
    const size_t sb = state_bytes(c), fb = (size_t)c->g.total * c->esize;
    char *t = static_cast<char *>(tape);
    if (nsteps < 2 || reinterpret_cast<uintptr_t>(t) % ALIGN || sb % ALIGN || fb % ALIGN) {
        for (int32_t k = 0; k < nsteps; ++k) {
            const lbm_status s = lbm_checkpoint(c, t + (size_t)k * sb);
            if (s != LBM_OK) return s;
            const lbm_status u = lbm_step(c, 1);
            if (u != LBM_OK) return u;
        }
        return LBM_OK;
    }
    // Slot 0 is a copy of the state; step k then reads slot k and writes its
    // result straight into slot k + 1 (the last step into the context's own
    // buffer), so the tape costs one copy per call instead of one per step.
    const lbm_status s0 = lbm_checkpoint(c, t);
    if (s0 != LBM_OK) return s0;
    void *ownA = c->fA, *ownB = c->fB;
    float *ownSA = c->scA, *ownSB = c->scB;
    auto slot_f = [&](int32_t k) { return static_cast<void *>(t + (size_t)k * sb); };
    auto slot_s = [&](int32_t k) { return c->p.passive_scalar ? reinterpret_cast<float *>(t + (size_t)k * sb + fb) : nullptr; };
    hipError_t e = hipSuccess;
    for (int32_t k = 0; k < nsteps && e == hipSuccess; ++k) {
        c->fA = k == 0 ? ownA : slot_f(k);
        c->scA = k == 0 ? ownSA : slot_s(k);
        c->fB = k == nsteps - 1 ? ownB : slot_f(k + 1);
        c->scB = k == nsteps - 1 ? ownSB : slot_s(k + 1);
        e = one_step(c);
    }
    // the context's buffers again; the final state is in ownB
    c->fA = ownB;
    c->fB = ownA;
    c->scA = ownSB;
    c->scB = ownSA;
    if (e != hipSuccess) return hip_fail(c, e, "lbm_record_tape");
    return LBM_OK;
}

lbm_status lbm_adjoint_ws_size(const lbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(const_cast<lbm_ctx *>(c), LBM_E_INVAL, "NULL argument");
    // the size depends on the band count, which may still be on the device
    const lbm_status st = settle_counts(const_cast<lbm_ctx *>(c), "lbm_adjoint_ws_size");
    if (st != LBM_OK) return st;
    *bytes = adjoint_ws_bytes(c);
    return LBM_OK;
}

lbm_status lbm_adjoint_init(lbm_ctx *c, void *adj_ws, size_t bytes)
{
    CHECK_CTX(c);
    if (c->p.collision != LBM_CM)
        return fail(c, LBM_E_UNSUPPORTED, "the adjoint differentiates the central-moment collision only");
    if (!adj_ws || reinterpret_cast<uintptr_t>(adj_ws) % ALIGN)
        return fail(c, LBM_E_INVAL, "adjoint workspace must be non-NULL and 256-byte aligned");
    const lbm_status st = settle_counts(c, "lbm_adjoint_init");
    if (st != LBM_OK) return st;
    if (bytes < adjoint_ws_bytes(c))
        return fail(c, LBM_E_NOMEM, "adjoint workspace too small: need " + std::to_string(adjoint_ws_bytes(c)) + " bytes");
    adjoint_bind(c, adj_ws, bytes);
    HIP_TRY(c, launch_zero(c, c->lam, (size_t)c->g.total * c->rsize), "lbm_adjoint_init");
    if (c->band_bar)  // the IB reverse scatter accumulates into it from zero
        HIP_TRY(c, launch_zero(c, c->band_bar, (size_t)c->adj_band_cap * 4 * c->rsize), "lbm_adjoint_init");
    return LBM_OK;
}

static lbm_status adjoint_ready(lbm_ctx *c)
{
    if (!c->aws) return fail(c, LBM_E_STATE, "lbm_adjoint_init has not been called");
    const lbm_status st = settle_counts(c, "adjoint");
    if (st != LBM_OK) return st;
    if (c->nm > 0 && c->nband > c->adj_band_cap)
        return fail(c, LBM_E_STATE, "samples changed after lbm_adjoint_init; call it again");
    return LBM_OK;
}

lbm_status lbm_adjoint_seed_macros(lbm_ctx *c, const void *g_rho, const void *g_u, double *g_inlet)
{
    CHECK_CTX(c);
    const lbm_status s = adjoint_ready(c);
    if (s != LBM_OK) return s;
    HIP_TRY(c, adjoint_seed_macros(c, g_rho, g_u, g_inlet), "lbm_adjoint_seed_macros");
    return LBM_OK;
}

lbm_status lbm_adjoint_seed_force(lbm_ctx *c, const double g_force[3], double *g_inlet, double *g_gain)
{
    CHECK_CTX(c);
    const lbm_status s = adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (!g_force) return fail(c, LBM_E_INVAL, "g_force is NULL");
    HIP_TRY(c, adjoint_seed_force(c, g_force, g_inlet, g_gain), "lbm_adjoint_seed_force");
    return LBM_OK;
}

lbm_status lbm_adjoint_step(lbm_ctx *c, int32_t nsteps, const void *tape, double *g_inlet, double *g_gain)
{
    CHECK_CTX(c);
    const lbm_status s = adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps must be >= 0");
    if (nsteps > 0 && !tape) return fail(c, LBM_E_INVAL, "tape is NULL");
    const size_t sb = state_bytes(c);
    for (int32_t k = nsteps - 1; k >= 0; --k)
        HIP_TRY(c, adjoint_step_one(c, static_cast<const char *>(tape) + (size_t)k * sb, g_inlet, g_gain),
                "lbm_adjoint_step");
    return LBM_OK;
}

lbm_status lbm_adjoint_get(lbm_ctx *c, void *lambda)
{
    CHECK_CTX(c);
    const lbm_status s = adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (!lambda) return fail(c, LBM_E_INVAL, "lambda is NULL");
    HIP_TRY(c, adjoint_io(c, lambda, false), "lbm_adjoint_get");
    return LBM_OK;
}

lbm_status lbm_adjoint_set(lbm_ctx *c, const void *lambda)
{
    CHECK_CTX(c);
    const lbm_status s = adjoint_ready(c);
    if (s != LBM_OK) return s;
    if (!lambda) return fail(c, LBM_E_INVAL, "lambda is NULL");
    HIP_TRY(c, adjoint_io(c, const_cast<void *>(lambda), true), "lbm_adjoint_set");
    return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) { delete c; }

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

const char *lbm_version(void) { return "liblbm 0.1 (gfx950)"; }

}  // extern "C"
