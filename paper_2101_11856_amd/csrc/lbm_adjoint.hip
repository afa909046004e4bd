// lbm_adjoint.hip -- reverse mode of one time step (adjoint of Alg. 2).
//
// For lambda = dJ/df(n+1) and the forward state f(n) (read from a tape), one
// adjoint step computes dJ/df(n) and accumulates parameter gradients:
//   k_adj_collide  per node: recompute the pull and the force, collision VJP
//                  (the general central-moment form, or the form for unit
//                  rates of orders 3 to 6 that the forward step then uses)
//                  -> mu = dJ/df*(x), phi = dJ/dF(x) at band nodes
//   k_adj_ib       per sample: spreading transposed = gather of phi;
//                  penalty (Eq. 7) reversed -> dJ/dgamma_s; interpolation
//                  transposed = scatter into the band adjoints of (rho, u0)
//   k_adj_band     per band node: (rho, u0) = moments of f* (Eq. 2) reversed
//   streaming transposed, for plain pulls: lambda_j(y) = mu_j(y + c_j), a
//                  gather that the next step's k_adj_collide performs while
//                  it loads lambda (k_adj_gather forms lambda on its own
//                  only when the caller reads it or seeds it)
//   k_adj_faces    face-layer nodes: streaming transposed for the face rules
//                  (atomic adds into the face part of lambda), with the
//                  inlet's wall-velocity term giving dJ/du_in(y, z)
//   k_adj_push     per node, all rules by scattering (adds to lambda; used by
//                  the seeds, which accumulate)
#include "lbm_adjoint.hpp"
#include "lbm_ctx.hpp"

namespace lbm {

template <typename R> struct V4;
template <> struct V4<float> {
    using type = float4;
};
template <> struct V4<double> {
    using type = double4;
};

template <int ST> struct AdjParams {
    using R = typename Store<ST>::R;
    using T = typename Store<ST>::T;
    using R4 = typename V4<R>::type;
    Geom g;
    const T *__restrict__ fin;  // forward state f(n)
    // lambda(n+1), population layout: all of it, or (pending) its face-rule
    // part, which the kernel reads and clears near the non-periodic faces
    R *__restrict__ lam;
    const R *__restrict__ Mprev;  // pending: mu of the step after, gathered
    int pending;
    R *__restrict__ M;            // mu, population layout
    Rates<R> rt;
    R body[3];
    Inlet<R> inlet;
    const uint64_t *__restrict__ tile_mask;
    const int32_t *__restrict__ tile_start;
    const R4 *__restrict__ band_force;
    R4 *__restrict__ band_phi;
};

__device__ __forceinline__ void node_of_item(const Geom &g, int64_t w, int lane, int &xs, int &x, int &y, int &z)
{
    xs = (int)(w % g.ntx);
    const int64_t row = w / g.ntx;
    y = (int)(row % g.ny);
    z = (int)(row / g.ny);
    x = xs * SEG + lane;
}

// Node reached from (x, y, z) by one lattice step c along an axis (c = -1, 0,
// +1), wrapped on a periodic axis, or -1 beyond a non-periodic face.
__device__ __forceinline__ int step_coord(int v, int c, int n, bool periodic)
{
    const int t = v + c;
    if (t >= 0 && t < n) return t;
    return periodic ? (t < 0 ? n - 1 : 0) : -1;
}

// lambda_j at (x, y, z) from the plain pulls transposed: mu_j of the node
// y + c_j that pulls f_j(y), or 0 when that node lies beyond a face.
template <typename R>
__device__ __forceinline__ void gather_plain(R (&lam)[3][3][3], const R *__restrict__ M, const Geom &g, int x, int y,
                                             int z)
{
    const bool px = g.face[0] == LBM_PERIODIC, py = g.face[2] == LBM_PERIODIC, pz = g.face[4] == LBM_PERIODIC;
    const int xd[3] = {step_coord(x, -1, g.nx, px), x, step_coord(x, 1, g.nx, px)};
    const int yd[3] = {step_coord(y, -1, g.ny, py), y, step_coord(y, 1, g.ny, py)};
    const int zd[3] = {step_coord(z, -1, g.nz, pz), z, step_coord(z, 1, g.nz, pz)};
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        const int tx = xd[CX[j] + 1], ty = yd[CY[j] + 1], tz = zd[CZ[j] + 1];
        R v = (R)0;
        if (tx >= 0 && ty >= 0 && tz >= 0) v = M[(int64_t)j * g.plane + row_off(g, ty, tz) + tx];
        lam[CZ[j] + 1][CY[j] + 1][CX[j] + 1] = v;
    }
}

// Nodes where a face rule can send a pull's adjoint: within one node of a
// non-periodic face (the rules read the node itself or a neighbour).
__device__ __forceinline__ bool near_face(const Geom &g, int x, int y, int z)
{
    return (g.face[0] != LBM_PERIODIC && (x <= 1 || x >= g.nx - 2)) ||
           (g.face[2] != LBM_PERIODIC && (y <= 1 || y >= g.ny - 2)) ||
           (g.face[4] != LBM_PERIODIC && (z <= 1 || z >= g.nz - 2));
}

// FP32 arithmetic forms: capped at 128 VGPRs (4 waves per SIMD instead of 3). The band variant
// then spills 2 VGPRs, the band-free one 26; the backward step still runs 4% faster. The form
// for unit high-order rates is capped at 96 (5 waves per SIMD; 2 / 9 VGPRs spilled, backward
// 0.205 -> 0.2035 ms/step).  The FP64 form would spill about 300 and keeps the compiler's choice.
// UNIT: the orders 3 to 6 relax at rate 1 (the forward step's collide_unit_high).
template <int ST, bool BAND, bool UNIT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(ST == LBM_F64 ? 1 : (UNIT ? 5 : 4))))
k_adj_collide(const AdjParams<ST> P)
{
    using R = typename Store<ST>::R;
    const Geom &g = P.g;
    const int lane = threadIdx.x & (SEG - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
    if (w >= g.W) return;
    int xs, x, y, z;
    node_of_item(g, w, lane, xs, x, y, z);
    const bool active = x < g.nx;
    const int xc = active ? x : g.nx - 1;
    R f[3][3][3];
    pull_wave<ST>(f, P.fin, xs, xc, y, z, g, P.inlet);
    R Fx = P.body[0], Fy = P.body[1], Fz = P.body[2];
    int slot = -1;
    if (BAND) {
        const uint64_t mask = P.tile_mask[w];
        if (mask != 0 && ((mask >> lane) & 1ull)) {
            slot = P.tile_start[w] + __popcll(mask & ((1ull << lane) - 1ull));
            const auto F = P.band_force[slot];
            Fx += F.x;
            Fy += F.y;
            Fz += F.z;
        }
    }
    const int64_t base = row_off(g, y, z) + xc;
    R lam[3][3][3];
    if (P.pending) {
        // lambda = plain pulls transposed (gather of the next step's mu) +
        // the face-rule part, which is then cleared for the next face pass
        gather_plain(lam, P.Mprev, g, xc, y, z);
        if (near_face(g, xc, y, z)) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                R *e = P.lam + (int64_t)i * g.plane + base;
                lam[CZ[i] + 1][CY[i] + 1][CX[i] + 1] += *e;
                if (active) *e = (R)0;
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) lam[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = P.lam[(int64_t)i * g.plane + base];
    }
    R Fb[3] = {0, 0, 0};
    if constexpr (UNIT) collide_unit_high_vjp(f, Fx, Fy, Fz, P.rt, lam, Fb[0], Fb[1], Fb[2]);
    else collide_vjp(f, Fx, Fy, Fz, P.rt, lam, Fb[0], Fb[1], Fb[2]);
    if (!active) return;
#pragma unroll
    for (int i = 0; i < Q; ++i) P.M[(int64_t)i * g.plane + base] = lam[CZ[i] + 1][CY[i] + 1][CX[i] + 1];
    if (BAND && slot >= 0) {
        typename AdjParams<ST>::R4 v;
        v.x = Fb[0];
        v.y = Fb[1];
        v.z = Fb[2];
        v.w = (R)0;
        P.band_phi[slot] = v;
    }
}

template <typename R> struct AdjIbParams {
    using R4 = typename V4<R>::type;
    int64_t n;
    const float *__restrict__ pos, *__restrict__ ub, *__restrict__ area, *__restrict__ gain;
    const int32_t *__restrict__ slot;
    const int32_t *__restrict__ perm;
    const R4 *__restrict__ band_ru;
    const R4 *__restrict__ band_phi;
    R4 *__restrict__ band_bar;
    double *__restrict__ g_gain;
};

template <typename R>
__global__ void __launch_bounds__(256) k_adj_ib(const AdjIbParams<R> P)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= P.n) return;
    const int64_t n = P.n;
    R t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = P.pos[a * n + s];
        t[a] = (R)(p - floorf(p));
    }
    R K[8], rs = 0, us[3] = {0, 0, 0}, psi[3] = {0, 0, 0};
    int32_t sl[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        sl[d] = P.slot[(int64_t)d * n + s];
        K[d] = ((d & 1) ? t[0] : (R)1 - t[0]) * ((d & 2) ? t[1] : (R)1 - t[1]) * ((d & 4) ? t[2] : (R)1 - t[2]);
        const auto v = P.band_ru[sl[d]];
        rs += K[d] * v.x;
        us[0] += K[d] * v.y;
        us[1] += K[d] * v.z;
        us[2] += K[d] * v.w;
        const auto ph = P.band_phi[sl[d]];
        psi[0] += K[d] * ph.x;
        psi[1] += K[d] * ph.y;
        psi[2] += K[d] * ph.z;
    }
    const R ar = (R)P.area[s], gam = (R)P.gain[s];
    R rb = 0, ubar[3];
    double gg = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        psi[a] *= ar;                        // dJ/dG_s (spreading carries a_s)
        const R diff = (R)P.ub[a * n + s] - us[a];
        gg += (double)(psi[a] * rs * diff);  // dG_s/dgamma_s = rho_s (u_b - u_s)
        rb += gam * psi[a] * diff;           // dG_s/drho_s
        ubar[a] = -gam * rs * psi[a];        // dG_s/du_s
    }
    if (P.g_gain) P.g_gain[P.perm[s]] += gg;  // one lane per sample: no race
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        R *dst = reinterpret_cast<R *>(P.band_bar + sl[d]);
        unsafeAtomicAdd(dst + 0, K[d] * rb);
        unsafeAtomicAdd(dst + 1, K[d] * ubar[0]);
        unsafeAtomicAdd(dst + 2, K[d] * ubar[1]);
        unsafeAtomicAdd(dst + 3, K[d] * ubar[2]);
    }
}

// Band nodes: (rho, u0) = (1 + sum d*, j / rho) reversed into mu.  Each
// lane clears its band_bar entry after reading it, so that the scatter of the
// next reverse step (k_adj_ib) starts from zeros without a fill launch.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_band(Geom g, const int32_t *__restrict__ band_cell, int64_t nband,
                                                  const typename V4<R>::type *__restrict__ band_ru,
                                                  typename V4<R>::type *__restrict__ band_bar, R *__restrict__ M)
{
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nband) return;
    const int64_t cell = band_cell[b];
    const int x = (int)(cell % g.nx);
    const int64_t r = cell / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const auto ru = band_ru[b];
    const auto bb = band_bar[b];
    band_bar[b] = typename V4<R>::type{(R)0, (R)0, (R)0, (R)0};
    const R inv = (R)1 / ru.x;
    const int64_t base = row_off(g, y, z) + x;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R add = bb.x + (bb.y * ((R)CX[i] - ru.y) + bb.z * ((R)CY[i] - ru.z) + bb.w * ((R)CZ[i] - ru.w)) * inv;
        M[(int64_t)i * g.plane + base] += add;
    }
}

// Streaming transposed: mu_i(x) is added to the adjoint of the population the
// pull of (i, x) read; the inlet term adds mu_i 2 w_i c_i / cs^2 to dJ/du_in.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_push(Geom g, const R *__restrict__ M, R *__restrict__ lam,
                                                  double *__restrict__ g_inlet)
{
    const int lane = threadIdx.x & (SEG - 1);
    const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
    if (w >= g.W) return;
    int xs, x, y, z;
    node_of_item(g, w, lane, xs, x, y, z);
    if (x >= g.nx) return;
    const int64_t base = row_off(g, y, z) + x;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R mu = M[(int64_t)i * g.plane + base];
        const PullSrc s = resolve(i, x, y, z, g);
        unsafeAtomicAdd(lam + (int64_t)s.pl * g.plane + row_off(g, s.sy, s.sz) + s.sx, mu);
        if (s.inlet && g_inlet) {
            const double c = 6.0 * weight(i) * (double)mu;
            const int64_t row = (int64_t)s.sz * g.ny + s.sy;
            const int64_t nyz = (int64_t)g.ny * g.nz;
            if (CX[i]) unsafeAtomicAdd(g_inlet + row, CX[i] * c);
            if (CY[i]) unsafeAtomicAdd(g_inlet + nyz + row, CY[i] * c);
            if (CZ[i]) unsafeAtomicAdd(g_inlet + 2 * nyz + row, CZ[i] * c);
        }
    }
}

// Streaming transposed for a whole step, in two parts.
// Plain part: a value f_j(y) read by a plain pull (source inside the domain,
// periodic axes wrapped) is read by node y + c_j only, so lambda_j(y) =
// mu_j(y + c_j) when that node exists, else 0: a gather, which the next
// reverse step's k_adj_collide does as it loads lambda.  k_adj_gather forms
// lambda = gather + (face part already in lam) in place, for the calls that
// need lambda itself (lbm_adjoint_get, the seeds).
template <typename R>
__global__ void __launch_bounds__(256) k_adj_gather(Geom g, const R *__restrict__ M, R *__restrict__ lam)
{
    const int lane = threadIdx.x & (SEG - 1);
    const uint32_t w = blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
    if (w >= (uint32_t)g.W) return;
    int xs, y, z;
    wave_coords(w, g, xs, y, z);
    const int x = xs * SEG + lane;
    if (x >= g.nx) return;
    R v[3][3][3];
    gather_plain(v, M, g, x, y, z);
    const int64_t base = row_off(g, y, z) + x;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        R *e = lam + (int64_t)j * g.plane + base;
        *e = v[CZ[j] + 1][CY[j] + 1][CX[j] + 1] + *e;
    }
}

// Face part (adds to the face part of lambda): every pull (i, x) whose source
// lies beyond a non-periodic face (bounce-back, inlet, outflow, free slip)
// adds mu_i(x) to the adjoint of the population the face rule read; the inlet
// term adds mu_i 2 w_i c_i / cs^2 to dJ/du_in.  Only face-layer nodes have such
// pulls; one lane per face-layer node.
template <typename R>
__global__ void __launch_bounds__(256) k_adj_faces(Geom g, FaceSet F, const R *__restrict__ M, R *__restrict__ lam,
                                                   double *__restrict__ g_inlet)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= F.na + F.nb) return;
    int x, y, z;
    face_node(k, g, F, x, y, z);
    const bool px = !F.xf, py = !F.yf, pz = !F.zf;
    const int64_t base = row_off(g, y, z) + x;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int sx = x - CX[i], sy = y - CY[i], sz = z - CZ[i];
        const bool plain = (px || (sx >= 0 && sx < g.nx)) && (py || (sy >= 0 && sy < g.ny)) &&
                           (pz || (sz >= 0 && sz < g.nz));
        if (plain) continue;
        const R mu = M[(int64_t)i * g.plane + base];
        const PullSrc s = resolve(i, x, y, z, g);
        unsafeAtomicAdd(lam + (int64_t)s.pl * g.plane + row_off(g, s.sy, s.sz) + s.sx, mu);
        if (s.inlet && g_inlet) {
            const double c = 6.0 * weight(i) * (double)mu;
            const int64_t row = (int64_t)s.sz * g.ny + s.sy;
            const int64_t nyz = (int64_t)g.ny * g.nz;
            if (CX[i]) unsafeAtomicAdd(g_inlet + row, CX[i] * c);
            if (CY[i]) unsafeAtomicAdd(g_inlet + nyz + row, CY[i] * c);
            if (CZ[i]) unsafeAtomicAdd(g_inlet + 2 * nyz + row, CZ[i] * c);
        }
    }
}

// Seed of an objective on lbm_macros: mu_i = g_rho + g_u . (c_i - u0) / rho
template <int ST>
__global__ void __launch_bounds__(256) k_adj_seed_macros(Geom g, const typename Store<ST>::T *__restrict__ fin,
                                                         Inlet<typename Store<ST>::R> inl,
                                                         const typename Store<ST>::R *__restrict__ g_rho,
                                                         const typename Store<ST>::R *__restrict__ g_u,
                                                         typename Store<ST>::R *__restrict__ M, int64_t N)
{
    using R = typename Store<ST>::R;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int x = (int)(k % g.nx);
    const int64_t r = k / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const Macro<R> m = node_moments<ST>(fin, x, y, z, g, inl);
    const R rho = (R)1 + m.drho, inv = (R)1 / rho;
    const R u[3] = {m.jx * inv, m.jy * inv, m.jz * inv};
    const R gr = g_rho ? g_rho[k] : (R)0;
    const R gu[3] = {g_u ? g_u[k] : (R)0, g_u ? g_u[N + k] : (R)0, g_u ? g_u[2 * N + k] : (R)0};
    const int64_t base = row_off(g, y, z) + x;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        M[(int64_t)i * g.plane + base] =
            gr + (gu[0] * ((R)CX[i] - u[0]) + gu[1] * ((R)CY[i] - u[1]) + gu[2] * ((R)CZ[i] - u[2])) * inv;
}

template <typename R>
__global__ void k_fill4(typename V4<R>::type *__restrict__ p, int64_t n, R a, R b, R c, R d)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    typename V4<R>::type v;
    v.x = a;
    v.y = b;
    v.z = c;
    v.w = d;
    p[k] = v;
}

// adjoint state in and out of a dense real[27][N] array
template <typename R>
__global__ void k_adj_io(Geom g, R *__restrict__ lam, R *__restrict__ dense, int64_t N, int to_state)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int x = (int)(k % g.nx);
    const int64_t r = k / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const int64_t base = row_off(g, y, z) + x;
    for (int i = 0; i < Q; ++i) {
        if (to_state) lam[(int64_t)i * g.plane + base] = dense[(int64_t)i * N + k];
        else dense[(int64_t)i * N + k] = lam[(int64_t)i * g.plane + base];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }
static inline dim3 g1(int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)); }

size_t adjoint_ws_bytes(const lbm_ctx *c)
{
    const size_t planes = a256((size_t)c->g.total * c->rsize);
    const size_t band = a256((size_t)std::max<int64_t>(c->nband, 1) * 4 * c->rsize);
    return 3 * planes + 2 * band;
}

void adjoint_bind(lbm_ctx *c, void *ws, size_t bytes)
{
    const size_t planes = a256((size_t)c->g.total * c->rsize);
    const size_t band = a256((size_t)std::max<int64_t>(c->nband, 1) * 4 * c->rsize);
    char *p = static_cast<char *>(ws);
    c->aws = p;
    c->aws_bytes = bytes;
    c->lam = p;
    c->adjM = p + planes;
    c->adjM2 = p + 2 * planes;
    c->adj_pending = false;
    c->band_phi = p + 3 * planes;
    c->band_bar = p + 3 * planes + band;
    c->adj_band_cap = std::max<int64_t>(c->nband, 1);
}

template <int ST> static AdjParams<ST> adj_params(lbm_ctx *c, const void *state)
{
    using R = typename Store<ST>::R;
    AdjParams<ST> P{};
    P.g = c->g;
    P.fin = static_cast<const typename Store<ST>::T *>(state);
    P.lam = static_cast<R *>(c->lam);
    P.Mprev = static_cast<const R *>(c->adjM);
    P.pending = c->adj_pending ? 1 : 0;
    P.M = static_cast<R *>(c->adjM2);
    P.rt = {(R)c->s_nu, (R)c->s_b, (R)c->s_h[0], (R)c->s_h[1], (R)c->s_h[2], (R)c->s_h[3]};
    for (int a = 0; a < 3; ++a) {
        P.body[a] = (R)c->p.body_force[a];
        P.inlet.u[a] = (R)c->p.u_in[a];
    }
    P.inlet.prof = static_cast<const R *>(c->p.inlet_profile);
    P.tile_mask = c->tile_mask;
    P.tile_start = c->tile_start;
    P.band_force = static_cast<const typename AdjParams<ST>::R4 *>(c->band_force);
    P.band_phi = static_cast<typename AdjParams<ST>::R4 *>(c->band_phi);
    return P;
}

// IB part of the reverse sweep: band_phi -> g_gain, band_bar -> mu (band_bar
// is zero on entry: cleared by lbm_adjoint_init, then by each k_adj_band)
template <typename R> static hipError_t adj_ib_part(lbm_ctx *c, double *g_gain)
{
    using R4 = typename V4<R>::type;
    AdjIbParams<R> Q{};
    Q.n = c->nm;
    Q.pos = c->m_pos;
    Q.ub = c->m_ub;
    Q.area = c->m_area;
    Q.gain = c->m_gain;
    Q.slot = c->m_slot;
    Q.perm = c->m_perm;
    Q.band_ru = static_cast<const R4 *>(c->band_ru);
    Q.band_phi = static_cast<const R4 *>(c->band_phi);
    Q.band_bar = static_cast<R4 *>(c->band_bar);
    Q.g_gain = g_gain;
    hipLaunchKernelGGL((k_adj_ib<R>), g1(c->nm), dim3(256), 0, c->stream, Q);
    hipLaunchKernelGGL((k_adj_band<R>), g1(c->nband), dim3(256), 0, c->stream, c->g, c->band_cell, c->nband,
                       static_cast<const R4 *>(c->band_ru), static_cast<R4 *>(c->band_bar),
                       static_cast<R *>(c->adjM2));
    return hipGetLastError();
}

template <int ST> static hipError_t step_st(lbm_ctx *c, const void *state, double *g_inlet, double *g_gain)
{
    using R = typename Store<ST>::R;
    hipError_t e;
    if (c->nm > 0 && (e = launch_band_ib(c, state, c->ftot_eval)) != hipSuccess) return e;
    const AdjParams<ST> P = adj_params<ST>(c, state);
    const dim3 grid((unsigned)((c->g.W + 3) / 4)), block(256);
    if (c->coll == COLL_CM_UNIT_HIGH) {
        if (c->nm > 0) hipLaunchKernelGGL((k_adj_collide<ST, true, true>), grid, block, 0, c->stream, P);
        else hipLaunchKernelGGL((k_adj_collide<ST, false, true>), grid, block, 0, c->stream, P);
    } else {
        if (c->nm > 0) hipLaunchKernelGGL((k_adj_collide<ST, true, false>), grid, block, 0, c->stream, P);
        else hipLaunchKernelGGL((k_adj_collide<ST, false, false>), grid, block, 0, c->stream, P);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (c->nm > 0 && (e = adj_ib_part<R>(c, g_gain)) != hipSuccess) return e;
    if (!c->adj_pending) {
        // lam held all of lambda(n+1); from now on it holds the face part only
        if ((e = launch_zero(c, c->lam, (size_t)c->g.total * c->rsize)) != hipSuccess) return e;
    }
    const FaceSet F = face_set(c->g);
    if (F.na + F.nb > 0)
        hipLaunchKernelGGL((k_adj_faces<R>), g1(F.na + F.nb), block, 0, c->stream, c->g, F,
                           static_cast<const R *>(c->adjM2), static_cast<R *>(c->lam), g_inlet);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    std::swap(c->adjM, c->adjM2);
    c->adj_pending = true;  // lambda(n) = plain pulls transposed (adjM) + lam
    return hipSuccess;
}

// lambda itself in lam (after a reverse step it is the gather of adjM plus the
// face part that lam holds)
template <typename R> static hipError_t adj_form(lbm_ctx *c)
{
    if (!c->adj_pending) return hipSuccess;
    hipLaunchKernelGGL((k_adj_gather<R>), dim3((unsigned)((c->g.W + 3) / 4)), dim3(256), 0, c->stream, c->g,
                       static_cast<const R *>(c->adjM), static_cast<R *>(c->lam));
    c->adj_pending = false;
    return hipGetLastError();
}

template <int ST> static hipError_t seed_macros_st(lbm_ctx *c, const void *g_rho, const void *g_u, double *g_inlet)
{
    using R = typename Store<ST>::R;
    const hipError_t e = adj_form<R>(c);  // the seed adds to lambda; adjM is scratch below
    if (e != hipSuccess) return e;
    Inlet<R> inl{};
    inl.prof = static_cast<const R *>(c->p.inlet_profile);
    for (int a = 0; a < 3; ++a) inl.u[a] = (R)c->p.u_in[a];
    hipLaunchKernelGGL((k_adj_seed_macros<ST>), g1(c->N), dim3(256), 0, c->stream, c->g,
                       static_cast<const typename Store<ST>::T *>(c->fA), inl, static_cast<const R *>(g_rho),
                       static_cast<const R *>(g_u), static_cast<R *>(c->adjM), c->N);
    hipLaunchKernelGGL((k_adj_push<R>), dim3((unsigned)((c->g.W + 3) / 4)), dim3(256), 0, c->stream, c->g,
                       static_cast<const R *>(c->adjM), static_cast<R *>(c->lam), g_inlet);
    return hipGetLastError();
}

template <int ST> static hipError_t seed_force_st(lbm_ctx *c, const double gf[3], double *g_inlet, double *g_gain)
{
    using R = typename Store<ST>::R;
    using R4 = typename V4<R>::type;
    hipError_t e;
    if ((e = adj_form<R>(c)) != hipSuccess) return e;  // the seed adds to lambda; adjM2 is scratch below
    if ((e = launch_band_ib(c, c->fA, c->ftot_eval)) != hipSuccess) return e;
    if ((e = launch_zero(c, c->adjM2, (size_t)c->g.total * c->rsize)) != hipSuccess) return e;
    // phi = g_force at every band node: the gather sum_d K_d phi then equals g_force
    hipLaunchKernelGGL((k_fill4<R>), g1(c->nband), dim3(256), 0, c->stream, static_cast<R4 *>(c->band_phi), c->nband,
                       (R)gf[0], (R)gf[1], (R)gf[2], (R)0);
    if ((e = adj_ib_part<R>(c, g_gain)) != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_push<R>), dim3((unsigned)((c->g.W + 3) / 4)), dim3(256), 0, c->stream, c->g,
                       static_cast<const R *>(c->adjM2), static_cast<R *>(c->lam), g_inlet);
    return hipGetLastError();
}

#define LBM_ADJ_DISPATCH(FN, ...)                                                               \
    switch (c->p.storage) {                                                                     \
    case LBM_F32: return FN<LBM_F32>(__VA_ARGS__);                                              \
    case LBM_F16DEV: return FN<LBM_F16DEV>(__VA_ARGS__);                                        \
    case LBM_BF16DEV: return FN<LBM_BF16DEV>(__VA_ARGS__);                                      \
    case LBM_F64: return FN<LBM_F64>(__VA_ARGS__);                                              \
    }                                                                                           \
    return hipErrorInvalidValue;

hipError_t adjoint_step_one(lbm_ctx *c, const void *state, double *g_inlet, double *g_gain)
{
    LBM_ADJ_DISPATCH(step_st, c, state, g_inlet, g_gain)
}
hipError_t adjoint_seed_macros(lbm_ctx *c, const void *g_rho, const void *g_u, double *g_inlet)
{
    LBM_ADJ_DISPATCH(seed_macros_st, c, g_rho, g_u, g_inlet)
}
hipError_t adjoint_seed_force(lbm_ctx *c, const double g_force[3], double *g_inlet, double *g_gain)
{
    if (c->nm <= 0) return hipSuccess;
    LBM_ADJ_DISPATCH(seed_force_st, c, g_force, g_inlet, g_gain)
}

hipError_t adjoint_io(lbm_ctx *c, void *dense, bool to_state)
{
    if (to_state) {
        c->adj_pending = false;  // lam takes all of lambda
    } else {
        const hipError_t e = c->rsize == 8 ? adj_form<double>(c) : adj_form<float>(c);
        if (e != hipSuccess) return e;
    }
    if (c->rsize == 8)
        hipLaunchKernelGGL((k_adj_io<double>), g1(c->N), dim3(256), 0, c->stream, c->g,
                           static_cast<double *>(c->lam), static_cast<double *>(dense), c->N, to_state ? 1 : 0);
    else
        hipLaunchKernelGGL((k_adj_io<float>), g1(c->N), dim3(256), 0, c->stream, c->g, static_cast<float *>(c->lam),
                           static_cast<float *>(dense), c->N, to_state ? 1 : 0);
    return hipGetLastError();
}

}  // namespace lbm
