// lbm_aux.hip -- initialisation, population I/O, macroscopic fields, FP64
// reductions, state copies and the set-up of the immersed solid samples.
#include <hipcub/hipcub.hpp>

#include "lbm_ctx.hpp"

namespace lbm {

template <int ST> using TT = typename Store<ST>::T;
template <int ST> using RR = typename Store<ST>::R;

__device__ __forceinline__ void cell_coords(int64_t k, const Geom &g, int &x, int &y, int &z)
{
    x = (int)(k % g.nx);
    const int64_t r = k / g.nx;
    y = (int)(r % g.ny);
    z = (int)(r / g.ny);
}
// scalar field: one plane [rows][nxp]
__device__ __forceinline__ int64_t padded(int x, int y, int z, const Geom &g)
{
    return ((int64_t)z * g.ny + y) * g.nxp + x;
}
// population 0 of node (x, y, z) in the blocked population layout
__device__ __forceinline__ int64_t pop_node(int x, int y, int z, const Geom &g) { return row_off(g, y, z) + x; }

// ---------------------------------------------------------------------------
// equilibrium: d_i = rho (prod phi(u) - prod phi(0)) + (rho - 1) w_i with the
// difference of products expanded so that nothing large cancels
// ---------------------------------------------------------------------------
template <int ST>
__global__ void k_init_eq(Geom g, const RR<ST> *__restrict__ rho, const RR<ST> *__restrict__ u, TT<ST> *__restrict__ f,
                          int64_t N)
{
    using R = RR<ST>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_coords(k, g, x, y, z);
    const R r = rho[k];
    const R uu[3] = {u[k], u[N + k], u[2 * N + k]};
    R p[3][3], d[3][3];  // [axis][c+1]: phi(0) and phi(u) - phi(0)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R v = uu[a], v2 = v * v;
        p[a][0] = p[a][2] = (R)(1.0 / 6.0);
        p[a][1] = (R)(2.0 / 3.0);
        d[a][0] = (R)0.5 * (v2 - v);
        d[a][1] = -v2;
        d[a][2] = (R)0.5 * (v2 + v);
    }
    const int64_t base = pop_node(x, y, z, g);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = CX[i] + 1, cy = CY[i] + 1, cz = CZ[i] + 1;
        const R dx = d[0][cx], dy = d[1][cy], dz = d[2][cz];
        const R px = p[0][cx], py = p[1][cy], pz = p[2][cz];
        const R D = dx * py * pz + px * dy * pz + px * py * dz + dx * dy * pz + dx * py * dz + px * dy * dz +
                    dx * dy * dz;
        const R dev = r * D + (r - (R)1) * (R)weight(i);
        f[(int64_t)i * g.plane + base] = Store<ST>::enc(dev);
    }
}

template <int ST>
__global__ void k_set_pop(Geom g, const RR<ST> *__restrict__ src, TT<ST> *__restrict__ f, int64_t N)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_coords(k, g, x, y, z);
    const int64_t base = pop_node(x, y, z, g);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[(int64_t)i * g.plane + base] = Store<ST>::enc(src[(int64_t)i * N + k] - (RR<ST>)weight(i));
}

template <int ST>
__global__ void k_get_pop(Geom g, const TT<ST> *__restrict__ f, RR<ST> *__restrict__ dst, int64_t N)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_coords(k, g, x, y, z);
    const int64_t base = pop_node(x, y, z, g);
#pragma unroll
    for (int i = 0; i < Q; ++i)
        dst[(int64_t)i * N + k] = Store<ST>::dec(f[(int64_t)i * g.plane + base]) + (RR<ST>)weight(i);
}

// rho and u0 = j / rho of the pulled current state, dense output
template <int ST>
__global__ void k_macros(Geom g, const TT<ST> *__restrict__ f, Inlet<RR<ST>> inl, RR<ST> *__restrict__ rho,
                         RR<ST> *__restrict__ u, int64_t N)
{
    using R = RR<ST>;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_coords(k, g, x, y, z);
    const Macro<R> m = node_moments<ST>(f, x, y, z, g, inl);
    const R r = (R)1 + m.drho;
    rho[k] = r;
    u[k] = m.jx / r;
    u[N + k] = m.jy / r;
    u[2 * N + k] = m.jz / r;
}

// ---------------------------------------------------------------------------
// FP64 conservation totals: per-block partials, then one ordered pass
// (deterministic).  Mass = N + sum d, momentum = sum c d (w has none).
// ---------------------------------------------------------------------------
template <int ST>
__global__ void __launch_bounds__(256) k_conserved(Geom g, const TT<ST> *__restrict__ f, int64_t N,
                                                   double *__restrict__ part, int *__restrict__ flag)
{
    __shared__ double sh[4][256];
    double acc[4] = {0, 0, 0, 0};
    int bad = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < N; k += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        cell_coords(k, g, x, y, z);
        const int64_t base = pop_node(x, y, z, g);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double v = (double)Store<ST>::dec(f[(int64_t)i * g.plane + base]);
            bad |= !isfinite(v);
            acc[0] += v;
            if (CX[i]) acc[1] += CX[i] * v;
            if (CY[i]) acc[2] += CY[i] * v;
            if (CZ[i]) acc[3] += CZ[i] * v;
        }
    }
    for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] = acc[a];
    if (bad) atomicAdd(flag, 1);
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 4; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 4; ++a) part[4 * blockIdx.x + a] = sh[a][0];
}

__global__ void k_conserved_final(const double *__restrict__ part, int nblk, double N, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double acc[4] = {0, 0, 0, 0};
    for (int b = 0; b < nblk; ++b)
        for (int a = 0; a < 4; ++a) acc[a] += part[4 * b + a];
    out[0] = N + acc[0];
    out[1] = acc[1];
    out[2] = acc[2];
    out[3] = acc[3];
}

__global__ void k_zero_int(int *p) { *p = 0; }

// plain 16-byte copy (also the calibration kernel for traffic counters)
__global__ void __launch_bounds__(256) k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n16)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = src[k];
}
__global__ void k_copy1(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}
__global__ void __launch_bounds__(256) k_zero16(uint4 *__restrict__ dst, int64_t n16)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += (int64_t)gridDim.x * blockDim.x)
        dst[k] = make_uint4(0, 0, 0, 0);
}
__global__ void k_zero1(uint8_t *__restrict__ dst, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = 0;
}

__global__ void k_scalar_io(Geom g, float *__restrict__ dst, const float *__restrict__ src, int64_t N, int to_state)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_coords(k, g, x, y, z);
    const int64_t p = padded(x, y, z, g);
    if (to_state) dst[p] = src[k];
    else dst[k] = src[p];
}

// ---------------------------------------------------------------------------
// solid samples (Sec. 4.2.2): keys, sort, band tiles, slots
// ---------------------------------------------------------------------------
constexpr int ELL = 4;

struct MarkerGeom {
    int nx, ny, nz, nbx, nby, ntx;
    int periodic[3];
};

// Checks, base cell and sort key of each sample (input order).
__global__ void k_mk_keys(MarkerGeom mg, int64_t n, const float *__restrict__ xyz, unsigned long long *__restrict__ keys,
                          int32_t *__restrict__ idx, int32_t *__restrict__ cell, int *__restrict__ bad)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int nn[3] = {mg.nx, mg.ny, mg.nz};
    int b[3], B[3];
    unsigned q[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = xyz[a * n + s];
        const float hi = mg.periodic[a] ? (float)nn[a] : (float)(nn[a] - 1);
        if (!(p >= 0.0f) || !(p < hi)) ok = false;
        b[a] = ok ? (int)floorf(p) : 0;
        B[a] = b[a] / ELL;
        // (x - l B) * (1024 / l): exact in FP32
        float r = floorf((p - (float)(ELL * B[a])) * (float)(1024 / ELL));
        r = fminf(fmaxf(r, 0.0f), 1023.0f);
        q[a] = ok ? (unsigned)r : 0u;
    }
    if (!ok) atomicAdd(bad, 1);
    unsigned long long morton = 0;
#pragma unroll
    for (int bit = 0; bit < 10; ++bit)
#pragma unroll
        for (int a = 0; a < 3; ++a) morton |= (unsigned long long)((q[a] >> bit) & 1u) << (3 * bit + a);
    const unsigned long long block =
        (unsigned long long)B[0] + (unsigned long long)mg.nbx * ((unsigned long long)B[1] + (unsigned long long)mg.nby * B[2]);
    keys[s] = (block << 30) | morton;
    idx[s] = (int32_t)s;
    cell[s] = (int32_t)((int64_t)b[0] + (int64_t)mg.nx * ((int64_t)b[1] + (int64_t)mg.ny * b[2]));
}

__global__ void k_mk_gather(int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ xyz,
                            const float *__restrict__ ub, const float *__restrict__ area, const float *__restrict__ gain,
                            float *__restrict__ pos_s, float *__restrict__ ub_s, float *__restrict__ area_s,
                            float *__restrict__ gain_s)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int64_t s = perm[k];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pos_s[a * n + k] = xyz[a * n + s];
        ub_s[a * n + k] = ub ? ub[a * n + s] : 0.0f;
    }
    area_s[k] = area ? area[s] : 1.0f;
    gain_s[k] = gain ? gain[s] : 1.0f;
}

__device__ __forceinline__ void stencil_node(const MarkerGeom &mg, const float *pos, int64_t n, int64_t k, int d, int &x,
                                             int &y, int &z)
{
    const int nn[3] = {mg.nx, mg.ny, mg.nz};
    int c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        int v = (int)floorf(pos[a * n + k]) + ((d >> a) & 1);
        if (v >= nn[a]) v -= nn[a];
        c[a] = v;
    }
    x = c[0];
    y = c[1];
    z = c[2];
}

__global__ void k_mk_mark(MarkerGeom mg, int64_t n, const float *__restrict__ pos, unsigned long long *__restrict__ mask)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    for (int d = 0; d < 8; ++d) {
        int x, y, z;
        stencil_node(mg, pos, n, k, d, x, y, z);
        const int64_t w = ((int64_t)z * mg.ny + y) * mg.ntx + x / SEG;
        atomicOr(mask + w, 1ull << (x % SEG));
    }
}

__global__ void k_tile_count(int64_t W, const unsigned long long *__restrict__ mask, int32_t *__restrict__ cnt)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w < W) cnt[w] = __popcll(mask[w]);
}

__global__ void k_band_list(MarkerGeom mg, int64_t W, const unsigned long long *__restrict__ mask,
                            const int32_t *__restrict__ start, int32_t *__restrict__ band_cell)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    unsigned long long m = mask[w];
    if (!m) return;
    const int xs = (int)(w % mg.ntx);
    const int64_t row = w / mg.ntx;
    int r = start[w];
    while (m) {
        const int bit = __ffsll((long long)m) - 1;
        m &= m - 1;
        band_cell[r++] = (int32_t)(row * mg.nx + xs * SEG + bit);
    }
}

__global__ void k_mk_slots(MarkerGeom mg, int64_t n, const float *__restrict__ pos,
                           const unsigned long long *__restrict__ mask, const int32_t *__restrict__ start,
                           int32_t *__restrict__ slot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    for (int d = 0; d < 8; ++d) {
        int x, y, z;
        stencil_node(mg, pos, n, k, d, x, y, z);
        const int64_t w = ((int64_t)z * mg.ny + y) * mg.ntx + x / SEG;
        const int bit = x % SEG;
        slot[(int64_t)d * n + k] = start[w] + __popcll(mask[w] & ((1ull << bit) - 1ull));
    }
}

// runs of sorted samples that share a base cell (slot of stencil offset 0)
__global__ void k_run_heads(int64_t n, const int32_t *__restrict__ slot0, int32_t *__restrict__ head)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) head[k] = (k == 0 || slot0[k] != slot0[k - 1]) ? 1 : 0;
}

__global__ void k_run_start(int64_t n, const int32_t *__restrict__ head, const int32_t *__restrict__ run_id,
                            int32_t *__restrict__ run_start)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (head[k]) run_start[run_id[k]] = (int32_t)k;
    if (k == n - 1) run_start[run_id[k] + head[k]] = (int32_t)n;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// band node t = base(run r) + d is fed by run r through offset d (one base
// per target and offset, so no two runs write the same entry)
__global__ void k_band_src(int64_t nruns, int64_t n, int64_t nband, const int32_t *__restrict__ run_start,
                           const int32_t *__restrict__ slot, int32_t *__restrict__ band_src)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    const int64_t k0 = run_start[r];
    for (int d = 0; d < 8; ++d) band_src[(int64_t)d * nband + slot[(int64_t)d * n + k0]] = (int32_t)r;
}

__global__ void k_flags_band(MarkerGeom mg, int64_t N, const unsigned long long *__restrict__ mask,
                             uint8_t *__restrict__ flags)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int x = (int)(k % mg.nx);
    const int64_t row = k / mg.nx;
    const int64_t w = row * mg.ntx + x / SEG;
    flags[k] = (uint8_t)((mask[w] >> (x % SEG)) & 1ull);
}

__global__ void k_flags_base(int64_t n, const int32_t *__restrict__ cell, uint8_t *__restrict__ flags)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n) flags[cell[s]] = 3;  // a base cell is always inside its own stencil
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline dim3 grid_for(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs > 0 ? (n + bs - 1) / bs : 1)); }

template <int ST> static hipError_t init_eq_st(lbm_ctx *c, const void *rho, const void *u)
{
    hipLaunchKernelGGL((k_init_eq<ST>), grid_for(c->N), dim3(256), 0, c->stream, c->g,
                       static_cast<const RR<ST> *>(rho), static_cast<const RR<ST> *>(u), static_cast<TT<ST> *>(c->fA),
                       c->N);
    return hipGetLastError();
}
template <int ST> static hipError_t set_pop_st(lbm_ctx *c, const void *f)
{
    hipLaunchKernelGGL((k_set_pop<ST>), grid_for(c->N), dim3(256), 0, c->stream, c->g, static_cast<const RR<ST> *>(f),
                       static_cast<TT<ST> *>(c->fA), c->N);
    return hipGetLastError();
}
template <int ST> static hipError_t get_pop_st(lbm_ctx *c, void *f)
{
    hipLaunchKernelGGL((k_get_pop<ST>), grid_for(c->N), dim3(256), 0, c->stream, c->g,
                       static_cast<const TT<ST> *>(c->fA), static_cast<RR<ST> *>(f), c->N);
    return hipGetLastError();
}
template <int ST> static hipError_t macros_st(lbm_ctx *c, void *rho, void *u)
{
    Inlet<RR<ST>> inl{};
    inl.prof = static_cast<const RR<ST> *>(c->p.inlet_profile);
    for (int a = 0; a < 3; ++a) inl.u[a] = (RR<ST>)c->p.u_in[a];
    hipLaunchKernelGGL((k_macros<ST>), grid_for(c->N), dim3(256), 0, c->stream, c->g,
                       static_cast<const TT<ST> *>(c->fA), inl, static_cast<RR<ST> *>(rho), static_cast<RR<ST> *>(u),
                       c->N);
    return hipGetLastError();
}
template <int ST> static hipError_t conserved_st(lbm_ctx *c)
{
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, c->stream, c->red_flag);
    hipLaunchKernelGGL((k_conserved<ST>), dim3(c->red_blocks), dim3(256), 0, c->stream, c->g,
                       static_cast<const TT<ST> *>(c->fA), c->N, c->red_part, c->red_flag);
    hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(64), 0, c->stream, c->red_part, c->red_blocks, (double)c->N,
                       c->red_out);
    return hipGetLastError();
}

#define LBM_DISPATCH(FN, ...)                                                                   \
    switch (c->p.storage) {                                                                     \
    case LBM_F32: return FN<LBM_F32>(__VA_ARGS__);                                              \
    case LBM_F16DEV: return FN<LBM_F16DEV>(__VA_ARGS__);                                        \
    case LBM_BF16DEV: return FN<LBM_BF16DEV>(__VA_ARGS__);                                      \
    case LBM_F64: return FN<LBM_F64>(__VA_ARGS__);                                              \
    }                                                                                           \
    return hipErrorInvalidValue;

hipError_t launch_init_eq(lbm_ctx *c, const void *rho, const void *u) { LBM_DISPATCH(init_eq_st, c, rho, u) }
hipError_t launch_set_pop(lbm_ctx *c, const void *f) { LBM_DISPATCH(set_pop_st, c, f) }
hipError_t launch_get_pop(lbm_ctx *c, void *f) { LBM_DISPATCH(get_pop_st, c, f) }
hipError_t launch_macros(lbm_ctx *c, void *rho, void *u) { LBM_DISPATCH(macros_st, c, rho, u) }
hipError_t launch_conserved(lbm_ctx *c) { LBM_DISPATCH(conserved_st, c) }

hipError_t launch_copy(lbm_ctx *c, void *dst, const void *src, size_t bytes)
{
    const int64_t n16 = (int64_t)(bytes / 16), tail = (int64_t)(bytes % 16);
    if (n16 > 0) {
        const int64_t nb = std::min<int64_t>((n16 + 255) / 256, 65536);
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)nb), dim3(256), 0, c->stream, static_cast<uint4 *>(dst),
                           static_cast<const uint4 *>(src), n16);
    }
    if (tail > 0)
        hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, c->stream, static_cast<uint8_t *>(dst) + 16 * n16,
                           static_cast<const uint8_t *>(src) + 16 * n16, tail);
    return hipGetLastError();
}

hipError_t launch_zero(lbm_ctx *c, void *dst, size_t bytes)
{
    const int64_t n16 = (int64_t)(bytes / 16), tail = (int64_t)(bytes % 16);
    if (n16 > 0) {
        const int64_t nb = std::min<int64_t>((n16 + 255) / 256, 65536);
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)nb), dim3(256), 0, c->stream, static_cast<uint4 *>(dst), n16);
    }
    if (tail > 0)
        hipLaunchKernelGGL(k_zero1, dim3(1), dim3(64), 0, c->stream, static_cast<uint8_t *>(dst) + 16 * n16, tail);
    return hipGetLastError();
}

hipError_t launch_scalar_io(lbm_ctx *c, float *dst, const float *src, bool to_state)
{
    hipLaunchKernelGGL(k_scalar_io, grid_for(c->N), dim3(256), 0, c->stream, c->g, dst, src, c->N, to_state ? 1 : 0);
    return hipGetLastError();
}

static MarkerGeom marker_geom(const lbm_ctx *c)
{
    MarkerGeom mg{};
    mg.nx = c->g.nx;
    mg.ny = c->g.ny;
    mg.nz = c->g.nz;
    mg.nbx = (c->g.nx + ELL - 1) / ELL;
    mg.nby = (c->g.ny + ELL - 1) / ELL;
    mg.ntx = c->g.ntx;
    for (int a = 0; a < 3; ++a) mg.periodic[a] = c->g.face[2 * a] == LBM_PERIODIC;
    return mg;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static int key_bits(const lbm_ctx *c)
{
    const int64_t nb = (int64_t)((c->g.nx + ELL - 1) / ELL) * ((c->g.ny + ELL - 1) / ELL) * ((c->g.nz + ELL - 1) / ELL);
    int bits = 1;
    while (bits < 40 && (1ll << bits) < nb) ++bits;
    return 30 + bits;
}

hipError_t solids_layout(const lbm_ctx *c, int64_t n, SolidsLayout *L)
{
    const size_t un = (size_t)(n > 0 ? n : 1);
    const size_t W = (size_t)c->g.W;
    const size_t nbmax = std::min<size_t>(8 * un, (size_t)c->N);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o += align256(bytes);
        return r;
    };
    L->pos = take(3 * un * 4);
    L->ub = take(3 * un * 4);
    L->area = take(un * 4);
    L->gain = take(un * 4);
    L->slot = take(8 * un * 4);
    L->cell = take(un * 4);
    L->perm = take(un * 4);
    L->keys_in = take(un * 8);
    L->keys_out = take(un * 8);
    L->idx_in = take(un * 4);
    size_t sort_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, (unsigned long long *)nullptr,
                                                      (unsigned long long *)nullptr, (int32_t *)nullptr,
                                                      (int32_t *)nullptr, (int)un, 0, key_bits(c));
    if (e != hipSuccess) return e;
    L->sort_tmp_bytes = sort_bytes;
    L->sort_tmp = take(sort_bytes);
    L->tile_mask = take(W * 8);
    L->tile_start = take(W * 4);
    L->tile_count = take(W * 4);
    size_t scan_bytes = 0;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t *)nullptr, (int32_t *)nullptr,
                                         (int)std::max<size_t>(W, un));
    if (e != hipSuccess) return e;
    L->scan_tmp_bytes = scan_bytes;
    L->scan_tmp = take(scan_bytes);
    L->band_cell = take(nbmax * 4);
    L->band_ru = take(nbmax * 4 * c->rsize);
    L->band_force = take(nbmax * 4 * c->rsize);
    L->ib_part = take(((un + 255) / 256) * 4 * 8);
    L->run_head = take(un * 4);
    L->run_id = take(un * 4);
    L->run_start = take((un + 1) * 4);
    L->run_sum = take(8 * un * 4 * c->rsize);
    L->band_src = take(8 * nbmax * 4);
    L->misc = take(256);
    L->total = o;
    return hipSuccess;
}

hipError_t solids_setup(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area, const float *gain,
                        int *bad_host)
{
    SolidsLayout L;
    hipError_t e = solids_layout(c, n, &L);
    if (e != hipSuccess) return e;
    char *m = c->mws;
    const MarkerGeom mg = marker_geom(c);
    auto *keys_in = reinterpret_cast<unsigned long long *>(m + L.keys_in);
    auto *keys_out = reinterpret_cast<unsigned long long *>(m + L.keys_out);
    auto *idx_in = reinterpret_cast<int32_t *>(m + L.idx_in);
    auto *perm = reinterpret_cast<int32_t *>(m + L.perm);
    auto *cell = reinterpret_cast<int32_t *>(m + L.cell);
    int *bad = reinterpret_cast<int *>(m + L.misc);
    int32_t *nband_dev = reinterpret_cast<int32_t *>(m + L.misc + 16);
    hipStream_t st = c->stream;

    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, bad);
    hipLaunchKernelGGL(k_mk_keys, grid_for(n), dim3(256), 0, st, mg, n, xyz, keys_in, idx_in, cell, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (*bad) return hipSuccess;

    size_t sort_bytes = L.sort_tmp_bytes;
    e = hipcub::DeviceRadixSort::SortPairs(m + L.sort_tmp, sort_bytes, keys_in, keys_out, idx_in, perm, (int)n, 0,
                                           key_bits(c), st);
    if (e != hipSuccess) return e;
    c->m_pos = reinterpret_cast<float *>(m + L.pos);
    c->m_ub = reinterpret_cast<float *>(m + L.ub);
    c->m_area = reinterpret_cast<float *>(m + L.area);
    c->m_gain = reinterpret_cast<float *>(m + L.gain);
    c->m_slot = reinterpret_cast<int32_t *>(m + L.slot);
    c->m_cell = cell;
    c->m_perm = perm;
    c->tile_mask = reinterpret_cast<uint64_t *>(m + L.tile_mask);
    c->tile_start = reinterpret_cast<int32_t *>(m + L.tile_start);
    c->band_cell = reinterpret_cast<int32_t *>(m + L.band_cell);
    c->band_ru = m + L.band_ru;
    c->band_force = m + L.band_force;
    c->ib_part = reinterpret_cast<double *>(m + L.ib_part);
    hipLaunchKernelGGL(k_mk_gather, grid_for(n), dim3(256), 0, st, n, perm, xyz, ub, area, gain, c->m_pos, c->m_ub,
                       c->m_area, c->m_gain);
    if ((e = launch_zero(c, c->tile_mask, (size_t)c->g.W * 8)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_mk_mark, grid_for(n), dim3(256), 0, st, mg, n, c->m_pos,
                       reinterpret_cast<unsigned long long *>(c->tile_mask));
    int32_t *cnt = reinterpret_cast<int32_t *>(m + L.tile_count);
    hipLaunchKernelGGL(k_tile_count, grid_for(c->g.W), dim3(256), 0, st, c->g.W,
                       reinterpret_cast<const unsigned long long *>(c->tile_mask), cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    size_t scan_bytes = L.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(m + L.scan_tmp, scan_bytes, cnt, c->tile_start, (int)c->g.W, st);
    if (e != hipSuccess) return e;
    // band size = start[W-1] + count[W-1]
    int32_t tail[2];
    if ((e = hipMemcpyAsync(&tail[0], c->tile_start + (c->g.W - 1), 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&tail[1], cnt + (c->g.W - 1), 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    (void)nband_dev;
    c->nband = (int64_t)tail[0] + tail[1];
    hipLaunchKernelGGL(k_band_list, grid_for(c->g.W), dim3(256), 0, st, mg, c->g.W,
                       reinterpret_cast<const unsigned long long *>(c->tile_mask), c->tile_start, c->band_cell);
    hipLaunchKernelGGL(k_mk_slots, grid_for(n), dim3(256), 0, st, mg, n, c->m_pos,
                       reinterpret_cast<const unsigned long long *>(c->tile_mask), c->tile_start, c->m_slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // runs of samples with one base cell, and the run feeding each band node
    int32_t *head = reinterpret_cast<int32_t *>(m + L.run_head);
    int32_t *rid = reinterpret_cast<int32_t *>(m + L.run_id);
    c->run_start = reinterpret_cast<int32_t *>(m + L.run_start);
    c->run_sum = m + L.run_sum;
    c->band_src = reinterpret_cast<int32_t *>(m + L.band_src);
    hipLaunchKernelGGL(k_run_heads, grid_for(n), dim3(256), 0, st, n, c->m_slot, head);
    scan_bytes = L.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(m + L.scan_tmp, scan_bytes, head, rid, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_start, grid_for(n), dim3(256), 0, st, n, head, rid, c->run_start);
    if ((e = hipMemcpyAsync(&tail[0], rid + (n - 1), 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&tail[1], head + (n - 1), 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    c->nruns = (int64_t)tail[0] + tail[1];
    hipLaunchKernelGGL(k_fill_i32, grid_for(8 * c->nband), dim3(256), 0, st, c->band_src, 8 * c->nband, -1);
    hipLaunchKernelGGL(k_band_src, grid_for(c->nruns), dim3(256), 0, st, c->nruns, n, c->nband, c->run_start,
                       c->m_slot, c->band_src);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return hipStreamSynchronize(st);
}

__global__ void k_gather_gain(int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ gain,
                              float *__restrict__ gain_s)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) gain_s[k] = gain[perm[k]];
}

hipError_t launch_set_gains(lbm_ctx *c, const float *gain)
{
    hipLaunchKernelGGL(k_gather_gain, grid_for(c->nm), dim3(256), 0, c->stream, c->nm, c->m_perm, gain, c->m_gain);
    return hipGetLastError();
}

hipError_t launch_solid_maps(lbm_ctx *c, uint8_t *flags, int32_t *cell, int32_t *perm)
{
    const MarkerGeom mg = marker_geom(c);
    hipError_t e;
    if (flags) {
        if (c->nm > 0) {
            hipLaunchKernelGGL(k_flags_band, grid_for(c->N), dim3(256), 0, c->stream, mg, c->N,
                               reinterpret_cast<const unsigned long long *>(c->tile_mask), flags);
            hipLaunchKernelGGL(k_flags_base, grid_for(c->nm), dim3(256), 0, c->stream, c->nm, c->m_cell, flags);
        } else if ((e = launch_zero(c, flags, (size_t)c->N)) != hipSuccess) {
            return e;
        }
    }
    if (c->nm > 0) {
        if (cell && (e = launch_copy(c, cell, c->m_cell, (size_t)c->nm * 4)) != hipSuccess) return e;
        if (perm && (e = launch_copy(c, perm, c->m_perm, (size_t)c->nm * 4)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace lbm
