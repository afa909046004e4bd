// lbm_aux.hip -- initialisation, population I/O, macroscopic fields, FP64
// reductions, state copies and the set-up of the immersed solid samples.
#include <hipcub/hipcub.hpp>

#include <mutex>

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
// Plain copies and fills: one 16-byte element per lane over a full grid, with
// non-temporal stores (measured 6.3 TB/s on MI355X against 4.8-5.2 TB/s for a
// grid-stride loop).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy16(u32x4 *__restrict__ dst, const u32x4 *__restrict__ src, int64_t n16)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) __builtin_nontemporal_store(src[k], dst + k);
}
__global__ void k_copy1(uint8_t *__restrict__ dst, const uint8_t *__restrict__ src, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) dst[k] = src[k];
}
__global__ void __launch_bounds__(256) k_zero16(u32x4 *__restrict__ dst, int64_t n16)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n16) __builtin_nontemporal_store((u32x4){0u, 0u, 0u, 0u}, dst + k);
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

// Body copy of the caller's samples (input order); NULL ub / area / gain take
// their defaults 0 / 1 / 1.
__global__ void k_body_store(int64_t n, const float *__restrict__ xyz, const float *__restrict__ ub,
                             const float *__restrict__ area, const float *__restrict__ gain, float *__restrict__ bx,
                             float *__restrict__ bu, float *__restrict__ ba, float *__restrict__ bg)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        bx[a * n + s] = xyz[a * n + s];
        bu[a * n + s] = ub ? ub[a * n + s] : 0.0f;
    }
    ba[s] = area ? area[s] : 1.0f;
    bg[s] = gain ? gain[s] : 1.0f;
}

struct Pose {
    double R[9], o[3], v[3], w[3];  // R row-major
};

// Rigid placement (the sample update of Alg. 2 (c)): x = o + R X in FP64 with
// one rounding per operation, in the order o_a + ((R_a0 X + R_a1 Y) + R_a2 Z),
// then rounded to FP32, so the base cells do not depend on the compiler's
// choice of fused operations; u_b = R ub + v + w x (x - o) with the FP32 x.
__global__ void k_pose(int64_t n, const Pose P, const float *__restrict__ bx, const float *__restrict__ bu,
                       float *__restrict__ wx, float *__restrict__ wu)
{
#pragma clang fp contract(off)
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const double X[3] = {(double)bx[s], (double)bx[n + s], (double)bx[2 * n + s]};
    const double U[3] = {(double)bu[s], (double)bu[n + s], (double)bu[2 * n + s]};
    double r[3], ru[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = P.o[a] + ((P.R[3 * a] * X[0] + P.R[3 * a + 1] * X[1]) + P.R[3 * a + 2] * X[2]);
        const float pf = (float)p;
        wx[a * n + s] = pf;
        r[a] = (double)pf - P.o[a];
        ru[a] = (P.R[3 * a] * U[0] + P.R[3 * a + 1] * U[1]) + P.R[3 * a + 2] * U[2];
    }
    wu[s] = (float)(ru[0] + P.v[0] + (P.w[1] * r[2] - P.w[2] * r[1]));
    wu[n + s] = (float)(ru[1] + P.v[1] + (P.w[2] * r[0] - P.w[0] * r[2]));
    wu[2 * n + s] = (float)(ru[2] + P.v[2] + (P.w[0] * r[1] - P.w[1] * r[0]));
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

// Marks the 2x2x2 stencil nodes of every sample in the tile bit masks.  The
// samples are sorted, so those of one base cell are adjacent: only the first
// of them marks (the others would set the same 8 bits), which keeps the
// atomics per tile word down to a few.
__global__ void k_mk_mark(MarkerGeom mg, int64_t n, const float *__restrict__ pos, unsigned long long *__restrict__ mask)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (k > 0 && floorf(pos[k]) == floorf(pos[k - 1]) && floorf(pos[n + k]) == floorf(pos[n + k - 1]) &&
        floorf(pos[2 * n + k]) == floorf(pos[2 * n + k - 1]))
        return;
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
// A run starts where the base cell changes (slot of stencil offset 0) and at
// every multiple of 64 sorted samples (the window of one spreading wavefront).
__global__ void k_run_heads(int64_t n, const int32_t *__restrict__ slot0, int32_t *__restrict__ head)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) head[k] = ((k & 63) == 0 || slot0[k] != slot0[k - 1]) ? 1 : 0;
}

// run starts, and whether a run continues the cell of the run before it
// (cut at a window boundary only)
__global__ void k_run_start(int64_t n, const int32_t *__restrict__ head, const int32_t *__restrict__ run_id,
                            const int32_t *__restrict__ slot0, int32_t *__restrict__ run_start,
                            uint8_t *__restrict__ run_cont)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (head[k]) {
        run_start[run_id[k]] = (int32_t)k;
        run_cont[run_id[k]] = (k > 0 && slot0[k] == slot0[k - 1]) ? 1 : 0;
    }
    if (k == n - 1) run_start[run_id[k] + head[k]] = (int32_t)n;
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = v;
}

// band node t = base(run r) + d is fed by run r through offset d (one base
// per target and offset, so no two runs write the same entry)
// counts[0] = band nodes, counts[1] = runs: found on the device so that the
// set-up reads both back with one copy at its end
__global__ void k_counts(int64_t W, const int32_t *__restrict__ tile_start, const int32_t *__restrict__ tile_cnt,
                         int64_t n, const int32_t *__restrict__ run_id, const int32_t *__restrict__ head,
                         int32_t *__restrict__ counts)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counts[0] = tile_start[W - 1] + tile_cnt[W - 1];
        counts[1] = run_id[n - 1] + head[n - 1];
    }
}

// band_src = -1 over its first 8 * counts[0] entries (grid-stride)
__global__ void k_clear_band_src(int32_t *__restrict__ band_src, const int32_t *__restrict__ counts)
{
    const int64_t total = 8 * (int64_t)counts[0];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x)
        band_src[k] = -1;
}

// band_src[d][j] = the first run of the cell whose stencil offset d is band node j
__global__ void k_band_src(int64_t n, const int32_t *__restrict__ counts, const int32_t *__restrict__ run_start,
                           const uint8_t *__restrict__ run_cont, const int32_t *__restrict__ slot,
                           int32_t *__restrict__ band_src)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nband = counts[0], nruns = counts[1];
    if (r >= nruns || run_cont[r]) return;
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
// the totals into (part [red_blocks][4], flag, out [4]): the context's
// workspace for lbm_conserved, the static scratch array for
// lbm_conserved_static
template <int ST> static hipError_t conserved_st(lbm_ctx *c, double *part, int *flag, double *out)
{
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, c->stream, flag);
    hipLaunchKernelGGL((k_conserved<ST>), dim3(c->red_blocks), dim3(256), 0, c->stream, c->g,
                       static_cast<const TT<ST> *>(c->fA), c->N, part, flag);
    hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(64), 0, c->stream, part, c->red_blocks, (double)c->N, out);
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
hipError_t launch_conserved(lbm_ctx *c) { LBM_DISPATCH(conserved_st, c, c->red_part, c->red_flag, c->red_out) }

// ---------------------------------------------------------------------------
// Library-owned scratch of lbm_conserved_static, for callers that cannot
// allocate: one array per GPU, held until the process ends.  Layout: the
// per-block partials [red_blocks][4] doubles from offset 0, the non-finite
// counter at CONS_FLAG_OFF, the 4 totals at CONS_OUT_OFF.  In host code the
// name `scratch` is only a stand-in for the symbol; the device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr size_t CONS_FLAG_OFF = (size_t)MAX_RED_BLOCKS * 4 * sizeof(double);
constexpr size_t CONS_OUT_OFF = CONS_FLAG_OFF + 256;
static_assert(CONS_OUT_OFF + 4 * sizeof(double) <= STATIC_SCRATCH_BYTES, "scratch layout");

constexpr int MAX_SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[MAX_SCRATCH_DEVICES] = {};

// device address of `scratch` on `device` (looked up once per device, with
// that device current; the caller's current device is restored)
static hipError_t scratch_on(int device, unsigned char **out)
{
    if (device < 0 || device >= MAX_SCRATCH_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

// scratch bytes the reduction of this context needs (partials, counter, totals)
size_t conserved_static_need(const lbm_ctx *c)
{
    const size_t part = (size_t)c->red_blocks * 4 * sizeof(double);
    return (part <= CONS_FLAG_OFF ? CONS_FLAG_OFF : part) + 256 + 4 * sizeof(double);
}

hipError_t launch_conserved_static(lbm_ctx *c, double out[4], int *flag)
{
    if (conserved_static_need(c) > STATIC_SCRATCH_BYTES) return hipErrorInvalidValue;  // checked by the caller too
    unsigned char *base = nullptr;
    hipError_t e = scratch_on(c->device, &base);
    if (e != hipSuccess) return e;
    double *part = reinterpret_cast<double *>(base);
    int *dflag = reinterpret_cast<int *>(base + CONS_FLAG_OFF);
    double *dout = reinterpret_cast<double *>(base + CONS_OUT_OFF);
    auto run = [&]() -> hipError_t { LBM_DISPATCH(conserved_st, c, part, dflag, dout) };
    if ((e = run()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(out, dout, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(flag, dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

hipError_t launch_copy(lbm_ctx *c, void *dst, const void *src, size_t bytes)
{
    const int64_t n16 = (int64_t)(bytes / 16), tail = (int64_t)(bytes % 16);
    if (n16 > 0) {
        const int64_t nb = (n16 + 255) / 256;  // one element per lane (the kernel has no loop)
        if (nb > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_copy16, dim3((unsigned)nb), dim3(256), 0, c->stream, static_cast<u32x4 *>(dst),
                           static_cast<const u32x4 *>(src), n16);
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
        const int64_t nb = (n16 + 255) / 256;  // one element per lane (the kernel has no loop)
        if (nb > 0x7fffffff) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_zero16, dim3((unsigned)nb), dim3(256), 0, c->stream, static_cast<u32x4 *>(dst), n16);
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

// Sample sort: hipcub's stable radix sort, which at these sizes (below 2^20
// items) runs as a block sort plus merge passes.  Forcing its onesweep radix
// passes instead was measured slower on MI355X for 273k 8-byte keys (about
// 165 us against 120 us per sort).
static hipError_t sort_samples(void *tmp, size_t &tmp_bytes, const unsigned long long *keys_in,
                               unsigned long long *keys_out, const int32_t *idx_in, int32_t *idx_out, int64_t n,
                               int bits, hipStream_t st)
{
    return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, keys_in, keys_out, idx_in, idx_out, (int)n, 0, bits,
                                              st);
}

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
    hipError_t e = sort_samples(nullptr, sort_bytes, nullptr, nullptr, nullptr, nullptr, (int64_t)un, key_bits(c),
                                nullptr);
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
    L->ib_part = take(((un + 255) / 256) * 8 * 8);
    L->run_head = take(un * 4);
    L->run_id = take(un * 4);
    L->run_start = take((un + 1) * 4);
    L->run_cont = take(un);
    L->run_sum = take(8 * un * 4 * c->rsize);
    L->band_src = take(8 * nbmax * 4);
    L->cell2 = take(un * 4);
    L->body_xyz = take(3 * un * 4);
    L->body_ub = take(3 * un * 4);
    L->body_area = take(un * 4);
    L->body_gain = take(un * 4);
    L->world_xyz = take(3 * un * 4);
    L->world_ub = take(3 * un * 4);
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
    int32_t *cell = c->m_cell_next;  // the current base cells stay intact until the samples pass the checks
    int *bad = reinterpret_cast<int *>(m + L.misc);
    int32_t *counts = reinterpret_cast<int32_t *>(m + L.misc + 16);  // band nodes, runs
    hipStream_t st = c->stream;

    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, bad);
    hipLaunchKernelGGL(k_mk_keys, grid_for(n), dim3(256), 0, st, mg, n, xyz, keys_in, idx_in, cell, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (*bad) return hipSuccess;

    size_t sort_bytes = L.sort_tmp_bytes;
    e = sort_samples(m + L.sort_tmp, sort_bytes, keys_in, keys_out, idx_in, perm, n, key_bits(c), st);
    if (e != hipSuccess) return e;
    c->m_pos = reinterpret_cast<float *>(m + L.pos);
    c->m_ub = reinterpret_cast<float *>(m + L.ub);
    c->m_area = reinterpret_cast<float *>(m + L.area);
    c->m_gain = reinterpret_cast<float *>(m + L.gain);
    c->m_slot = reinterpret_cast<int32_t *>(m + L.slot);
    c->m_cell_next = c->m_cell;
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
    hipLaunchKernelGGL(k_band_list, grid_for(c->g.W), dim3(256), 0, st, mg, c->g.W,
                       reinterpret_cast<const unsigned long long *>(c->tile_mask), c->tile_start, c->band_cell);
    hipLaunchKernelGGL(k_mk_slots, grid_for(n), dim3(256), 0, st, mg, n, c->m_pos,
                       reinterpret_cast<const unsigned long long *>(c->tile_mask), c->tile_start, c->m_slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // runs of samples with one base cell, and the run feeding each band node
    int32_t *head = reinterpret_cast<int32_t *>(m + L.run_head);
    int32_t *rid = reinterpret_cast<int32_t *>(m + L.run_id);
    c->run_start = reinterpret_cast<int32_t *>(m + L.run_start);
    c->run_id = rid;
    c->run_cont = reinterpret_cast<uint8_t *>(m + L.run_cont);
    c->run_sum = m + L.run_sum;
    c->band_src = reinterpret_cast<int32_t *>(m + L.band_src);
    hipLaunchKernelGGL(k_run_heads, grid_for(n), dim3(256), 0, st, n, c->m_slot, head);
    scan_bytes = L.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(m + L.scan_tmp, scan_bytes, head, rid, (int)n, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_run_start, grid_for(n), dim3(256), 0, st, n, head, rid, c->m_slot, c->run_start, c->run_cont);
    hipLaunchKernelGGL(k_counts, dim3(1), dim3(64), 0, st, c->g.W, c->tile_start, cnt, n, rid, head, counts);
    hipLaunchKernelGGL(k_clear_band_src, dim3(1024), dim3(256), 0, st, c->band_src, counts);
    hipLaunchKernelGGL(k_band_src, grid_for(n), dim3(256), 0, st, n, counts, c->run_start, c->run_cont, c->m_slot,
                       c->band_src);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t got[2];
    if ((e = hipMemcpyAsync(got, counts, sizeof(got), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    c->nband = got[0];
    c->nruns = got[1];
    return hipSuccess;
}

hipError_t solids_store_body(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area,
                             const float *gain)
{
    SolidsLayout L;
    hipError_t e = solids_layout(c, n, &L);
    if (e != hipSuccess) return e;
    char *m = c->mws;
    c->m_cell = reinterpret_cast<int32_t *>(m + L.cell);
    c->m_cell_next = reinterpret_cast<int32_t *>(m + L.cell2);
    c->b_xyz = reinterpret_cast<float *>(m + L.body_xyz);
    c->b_ub = reinterpret_cast<float *>(m + L.body_ub);
    c->b_area = reinterpret_cast<float *>(m + L.body_area);
    c->b_gain = reinterpret_cast<float *>(m + L.body_gain);
    c->w_xyz = reinterpret_cast<float *>(m + L.world_xyz);
    c->w_ub = reinterpret_cast<float *>(m + L.world_ub);
    hipLaunchKernelGGL(k_body_store, grid_for(n), dim3(256), 0, c->stream, n, xyz, ub, area, gain, c->b_xyz, c->b_ub,
                       c->b_area, c->b_gain);
    return hipGetLastError();
}

hipError_t solids_pose(lbm_ctx *c, const double R[9], const double o[3], const double v[3], const double w[3],
                       int *bad_host)
{
    Pose P{};
    for (int k = 0; k < 9; ++k) P.R[k] = R[k];
    for (int a = 0; a < 3; ++a) {
        P.o[a] = o[a];
        P.v[a] = v[a];
        P.w[a] = w[a];
    }
    const int64_t n = c->nm;
    hipLaunchKernelGGL(k_pose, grid_for(n), dim3(256), 0, c->stream, n, P, c->b_xyz, c->b_ub, c->w_xyz, c->w_ub);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return solids_setup(c, n, c->w_xyz, c->w_ub, c->b_area, c->b_gain, bad_host);
}

__global__ void k_gather_gain(int64_t n, const int32_t *__restrict__ perm, const float *__restrict__ gain,
                              float *__restrict__ gain_s)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) gain_s[k] = gain[perm[k]];
}

hipError_t launch_set_gains(lbm_ctx *c, const float *gain)
{
    const hipError_t e = launch_copy(c, c->b_gain, gain, (size_t)c->nm * 4);
    if (e != hipSuccess) return e;
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
