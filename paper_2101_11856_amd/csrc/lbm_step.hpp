// lbm_step.hpp -- the per-step kernels of liblbm (Alg. 2 of the paper):
//   k_band      (a)+(b) on the immersed-boundary band only: pull (or the band
//               pieces the last fused kernel wrote) + rho, u
//   k_ib_run    (c) interpolation and penalty force per sample; per run of
//               samples sharing a base cell, the 8 spreading sums
//   k_ib_total  (c) FP64 total force and torque from per-block partials, in order
//   k_spread    (c) spreading completed: each band node gathers its run sums
//   k_fused     (a)+(b)+(d)+(e) for every node: pull with face rules, rho and
//               u, band force, central-moment collision, store; optionally the
//               band pieces of the next step
#pragma once

#include "lbm_ctx.hpp"

namespace lbm {

template <typename R> struct R4T;
template <> struct R4T<float> {
    using type = float4;
};
template <> struct R4T<double> {
    using type = double4;
};

template <typename R> struct R2T;
template <> struct R2T<float> {
    using type = float2;
};
template <> struct R2T<double> {
    using type = double2;
};

template <int ST> struct StepParams {
    using R = typename Store<ST>::R;
    using T = typename Store<ST>::T;
    using R4 = typename R4T<R>::type;
    using R2 = typename R2T<R>::type;
    Geom g;
    const T *__restrict__ fin;
    T *__restrict__ fout;
    Rates<R> rt;
    R body[3];
    Inlet<R> inlet;
    const uint64_t *__restrict__ tile_mask;
    const int32_t *__restrict__ tile_start;
    const R4 *__restrict__ band_force;
    // spreading finished inside the fused kernel (instead of k_spread): the
    // run sums of the cells that target each band node, gathered in k_spread's order
    int fused_spread;
    int64_t bstride, rstride;                // strides of band_src and run_sum (their capacities)
    const int32_t *__restrict__ band_src;
    const uint8_t *__restrict__ run_cont;
    const R4 *__restrict__ run_sum;
    const float *__restrict__ sc_in;
    float *__restrict__ sc_out;
    int sc_h;
    int load32;     // interior loads by 32-bit offsets from a per-wavefront base (blocked layout)
    uint32_t span;  // bytes from a row's lowest source row that cover its 9 source rows
    float one;      // 1, as a run-time value (mixed-precision FP16 sums)
    // band pieces [9][bstride] (pairs, see band_moments): written by the fused
    // kernel for the next step's band pre-pass (null: not written), read by the
    // pre-pass instead of pulling (null: it pulls)
    R2 *__restrict__ push_out;
    const R2 *__restrict__ push_in;
    const uint32_t *__restrict__ push_feeds;  // [W] bit r: tile of row r fed by wavefront w holds band nodes
};

// ---------------------------------------------------------------------------
// passive scalar: first-order upwind by the collision velocity; periodic
// wrap or zero gradient at faces; held at 1 on inlet nodes below sc_h
// ---------------------------------------------------------------------------
__device__ __forceinline__ int nb_coord(int v, int n, bool periodic)
{
    if (v < 0) return periodic ? v + n : 0;
    if (v >= n) return periodic ? v - n : n - 1;
    return v;
}

template <int ST>
__device__ __forceinline__ void scalar_update(const StepParams<ST> &P, int x, int y, int z, float ux, float uy,
                                              float uz, bool active)
{
    const Geom &g = P.g;
    auto at = [&](int xx, int yy, int zz) {
        xx = nb_coord(xx, g.nx, g.face[0] == LBM_PERIODIC);
        yy = nb_coord(yy, g.ny, g.face[2] == LBM_PERIODIC);
        zz = nb_coord(zz, g.nz, g.face[4] == LBM_PERIODIC);
        return P.sc_in[((int64_t)zz * g.ny + yy) * g.nxp + xx];
    };
    const float s0 = at(x, y, z);
    float v = s0;
    v -= ux > 0.f ? ux * (s0 - at(x - 1, y, z)) : ux * (at(x + 1, y, z) - s0);
    v -= uy > 0.f ? uy * (s0 - at(x, y - 1, z)) : uy * (at(x, y + 1, z) - s0);
    v -= uz > 0.f ? uz * (s0 - at(x, y, z - 1)) : uz * (at(x, y, z + 1) - s0);
    if (x == 0 && g.face[0] == LBM_INLET && y < P.sc_h) v = 1.f;
    if (active) P.sc_out[((int64_t)z * g.ny + y) * g.nxp + x] = v;
}

// ---------------------------------------------------------------------------
// band pieces.  At a band node away from every face (1 <= x <= nx-2, the same
// for y and z) every streamed value is a plain pull, and the sums of Eq. (2)
// are taken by source row: for the row offset (dy, dz) of the populations
// A = (+1, dy, dz), B = (0, dy, dz), C = (-1, dy, dz), whose streamed values
// come from x-1, x, x+1 of row (y-dy, z-dz), piece 0 is (A + B) + C and piece
// 1 is A - C (their x-momentum).  A is left out at the first node of a 64-node
// segment and C at the last, since they come from the neighbouring segment;
// they are added after the nine pieces.  The fused kernel of the step before
// holds A, B and C of one source row and segment in three populations of
// adjacent lanes, so it can form the pieces of the next step's band nodes
// (push_band) and the pre-pass reads 18 coalesced values per node instead of
// 27 scattered ones.  Both forms add in the same order: same bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool band_interior(const Geom &g, int x, int y, int z)
{
    return x >= 1 && x <= g.nx - 2 && y >= 1 && y <= g.ny - 2 && z >= 1 && z <= g.nz - 2;
}

template <typename R> __device__ __forceinline__ void band_piece(R A, R B, R C, int lane, R &p0, R &p1)
{
    const R a = lane != 0 ? A : (R)0, c = lane != SEG - 1 ? C : (R)0;
    p0 = (a + B) + c;
    p1 = a - c;
}

// piece of row offset (dy, dz) into the sums (piece 0 carries c_y and c_z)
template <typename R> __device__ __forceinline__ void band_add(Macro<R> &m, R p0, R p1, int dy, int dz)
{
    m.drho += p0;
    m.jx += p1;
    if (dy) m.jy += dy > 0 ? p0 : -p0;
    if (dz) m.jz += dz > 0 ? p0 : -p0;
}

// the value of population (cx, cy, cz) streamed to the interior node (x, y, z)
template <int ST>
__device__ __forceinline__ typename Store<ST>::R band_pull(const StepParams<ST> &P, int cx, int cy, int cz, int x,
                                                           int y, int z)
{
    const Geom &g = P.g;
    const int i = pop_index(cx, cy, cz);
    return Store<ST>::dec(ld_stream(P.fin + (int64_t)i * g.plane + row_off(g, y - cy, z - cz) + (x - cx)));
}

template <int ST>
__device__ __forceinline__ Macro<typename Store<ST>::R> band_moments(const StepParams<ST> &P, int64_t b, int x, int y,
                                                                     int z)
{
    using R = typename Store<ST>::R;
    const int lane = x & (SEG - 1);
    R A[9], C[9];
    Macro<R> m{0, 0, 0, 0};
    if (P.push_in) {
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const auto pp = P.push_in[r * P.bstride + b];
            band_add(m, pp.x, pp.y, r % 3 - 1, r / 3 - 1);
        }
        if (lane == 0) {
#pragma unroll
            for (int r = 0; r < 9; ++r) A[r] = band_pull<ST>(P, 1, r % 3 - 1, r / 3 - 1, x, y, z);
        }
        if (lane == SEG - 1) {
#pragma unroll
            for (int r = 0; r < 9; ++r) C[r] = band_pull<ST>(P, -1, r % 3 - 1, r / 3 - 1, x, y, z);
        }
    } else {
        R B[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            A[r] = band_pull<ST>(P, 1, r % 3 - 1, r / 3 - 1, x, y, z);
            B[r] = band_pull<ST>(P, 0, r % 3 - 1, r / 3 - 1, x, y, z);
            C[r] = band_pull<ST>(P, -1, r % 3 - 1, r / 3 - 1, x, y, z);
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            R p0, p1;
            band_piece(A[r], B[r], C[r], lane, p0, p1);
            band_add(m, p0, p1, r % 3 - 1, r / 3 - 1);
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int r = 0; r < 9; ++r) band_add(m, A[r], A[r], r % 3 - 1, r / 3 - 1);
    }
    if (lane == SEG - 1) {
#pragma unroll
        for (int r = 0; r < 9; ++r) band_add(m, C[r], -C[r], r % 3 - 1, r / 3 - 1);
    }
    return m;
}

// Tiles of the next step's band nodes that this wavefront's results feed: lane
// r < 9 loads the band mask and first slot of this segment in row (y+dy, z+dz),
// r = 3 (dz + 1) + dy + 1, when bit r of the wavefront's feeds word is set (else
// 0).  Loaded when the wavefront starts, so that they have long arrived when
// they are read, and held in three vector registers rather than 27 scalar ones
// (the kernel's scalar registers already bound its occupancy).
struct PushTiles {
    uint32_t lo, hi;
    int32_t start;
};

template <int ST>
__device__ __forceinline__ void push_tiles(const StepParams<ST> &P, uint32_t w, uint32_t feeds, int lane, PushTiles &pt)
{
    const Geom &g = P.g;
    const int dy = lane % 3 - 1, dz = lane / 3 - 1;
    pt.lo = pt.hi = 0;
    pt.start = 0;
    if (lane < 9 && ((feeds >> lane) & 1u)) {
        const int64_t t = (int64_t)w + ((int64_t)dz * g.ny + dy) * g.ntx;
        const uint64_t m = P.tile_mask[t];
        pt.lo = (uint32_t)m;
        pt.hi = (uint32_t)(m >> 32);
        pt.start = P.tile_start[t];
    }
}

// The tiles read out of the lanes into scalar registers, before the kernel's
// stores (reading them after the stores makes the compiler wait for the stores
// too, since it cannot tell the loads' wait apart from theirs).
struct PushRows {
    uint64_t mask[9];
    int32_t start[9];
};
__device__ __forceinline__ void push_rows(const PushTiles &pt, uint32_t feeds, PushRows &pr)
{
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        pr.mask[r] = 0;
        pr.start[r] = 0;
        if (!((feeds >> r) & 1u)) continue;
        pr.mask[r] = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)pt.hi, r) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane((int)pt.lo, r);
        pr.start[r] = __builtin_amdgcn_readlane(pt.start, r);
    }
}

// Lane i receives lane i-1's value (BELOW) or lane i+1's (else); lane 0,
// respectively 63, receives 0: a DPP wavefront shift by one lane.
template <bool BELOW> __device__ __forceinline__ int lane_shift(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, BELOW ? 0x138 : 0x130, 0xf, 0xf, false);  // wave_shr:1 / wave_shl:1
}
template <bool BELOW> __device__ __forceinline__ float lane_shift(float v)
{
    return __builtin_bit_cast(float, lane_shift<BELOW>(__builtin_bit_cast(int, v)));
}
template <bool BELOW> __device__ __forceinline__ double lane_shift(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)lane_shift<BELOW>((int)(uint32_t)b), hi = (uint32_t)lane_shift<BELOW>((int)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The pieces of those band nodes: lanes of the nodes store their two pieces
// at the node's band slot.  Called by all lanes of the wavefront (the shifts),
// after the kernel's own stores (issued before them, the pieces' partial-line
// stores held up the population stores: FP16 city 7.79-8.16 ms per step
// against 7.12-7.34 after them).
template <int ST>
__device__ __forceinline__ void push_band(const StepParams<ST> &P, const typename Store<ST>::R (&f)[3][3][3],
                                          uint32_t feeds, const PushRows &pr, int lane)
{
    using R = typename Store<ST>::R;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
        const int dy = r % 3 - 1, dz = r / 3 - 1;
        if (!((feeds >> r) & 1u)) continue;
        const uint64_t mask = pr.mask[r];
        // the stored values (16-bit forms round here as on store)
        const R a = Store<ST>::dec(Store<ST>::enc(f[dz + 1][dy + 1][2]));
        const R B = Store<ST>::dec(Store<ST>::enc(f[dz + 1][dy + 1][1]));
        const R c = Store<ST>::dec(Store<ST>::enc(f[dz + 1][dy + 1][0]));
        const R A = lane_shift<true>(a), C = lane_shift<false>(c);
        R p0, p1;
        band_piece(A, B, C, lane, p0, p1);
        if ((mask >> lane) & 1ull) {
            // band nodes of the tile below this lane
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
            const int64_t slot = (int64_t)pr.start[r] + below;
            typename StepParams<ST>::R2 pp;
            pp.x = p0;
            pp.y = p1;
            P.push_out[r * P.bstride + slot] = pp;
        }
    }
}

// ---------------------------------------------------------------------------
// fused step
// ---------------------------------------------------------------------------
// B32: the 27 populations of one row lie within 2^31 bytes of the row's start
// (always for the blocked layout), so the stores go through a buffer
// descriptor based at the row: population offset in a scalar register, x
// offset in one 32-bit vector register, no 64-bit vector address arithmetic.
//
// ROW: the workgroup's waves are exactly the segments of one row (segments per
// row == waves per workgroup) and x is periodic.  Rows on no y/z face then
// stage the 27 source rows in LDS with aligned, coalesced loads (one per
// population and node) and read the x-shifted values back from LDS, instead
// of 18 misaligned global loads; all waves of a workgroup share the row, so
// the barrier is uniform.
//
// COLL: the collision model (collide_as: central moments with any rates or
// with unit high-order rates, BGK, raw-moment MRT).
template <int ST, bool BAND, bool SCALAR, bool B32, bool ROW, int COLL>
__global__ void __launch_bounds__(SEG *WAVES_PER_BLOCK) k_fused(const StepParams<ST> P)
{
    using R = typename Store<ST>::R;
    using T = typename Store<ST>::T;
    const Geom &g = P.g;
    const int lane = threadIdx.x & (SEG - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / SEG);
    const uint32_t w = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (uint32_t)wv;
    if (w >= (uint32_t)g.W) return;
    int xs, y, z;
    wave_coords(w, g, xs, y, z);
    const int x = xs * SEG + lane;
    const bool active = x < g.nx;
    const int xc = active ? x : g.nx - 1;

    R Fx = P.body[0], Fy = P.body[1], Fz = P.body[2];
    // rows of the next step's band that this wavefront feeds (0: none, or no pieces)
    const uint32_t feeds = BAND && P.push_out ? P.push_feeds[w] : 0u;
    PushTiles pt;
    if (feeds) push_tiles<ST>(P, w, feeds, lane, pt);
    if (BAND) {
        const uint64_t mask = P.tile_mask[w];
        if (mask != 0 && ((mask >> lane) & 1ull)) {
            const int slot = P.tile_start[w] + __popcll(mask & ((1ull << lane) - 1ull));
            if (P.fused_spread) {
                R gx = 0, gy = 0, gz = 0;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    int64_t src = P.band_src[(int64_t)d * P.bstride + slot];
                    if (src >= 0) {
                        for (;;) {
                            const auto v = P.run_sum[(int64_t)d * P.rstride + src];
                            gx += v.x;
                            gy += v.y;
                            gz += v.z;
                            if (!P.run_cont[src + 1]) break;  // the entry after the last run is 0
                            ++src;
                        }
                    }
                }
                Fx += gx;
                Fy += gy;
                Fz += gz;
            } else {
                const auto F = P.band_force[slot];
                Fx += F.x;
                Fy += F.y;
                Fz += F.z;
            }
        }
    }
    R f[3][3][3];
    R rho, ux, uy, uz;
    // FP16 deviations, central moments at unit high-order rates, interior
    // rows: the halves go straight into the mixed-precision first stage
    constexpr bool MIX = ST == LBM_F16DEV && COLL == COLL_CM_UNIT_HIGH && B32 && !ROW;
    bool collided = false;
    if constexpr (MIX) {
        const bool yz = (y == 0 && g.face[2] != LBM_PERIODIC) || (y == g.ny - 1 && g.face[3] != LBM_PERIODIC) ||
                        (z == 0 && g.face[4] != LBM_PERIODIC) || (z == g.nz - 1 && g.face[5] != LBM_PERIODIC);
        const bool xf = (xs == 0 && g.face[0] != LBM_PERIODIC) || (xs == g.ntx - 1 && g.face[1] != LBM_PERIODIC);
        const bool wrap = y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
        if (P.load32 && !yz && !xf && !wrap) {
            _Float16 h[3][3][3];
            pull_interior32_f16(h, P.fin, xc, y, z, g, P.span);
            unit_high_from_low(low_moments_f16(h, P.one), f, Fx, Fy, Fz, P.rt, rho, ux, uy, uz);
            collided = true;
        }
    }
    if (!collided) {
    if constexpr (ROW) {
        __shared__ T row[Q][SEG * WAVES_PER_BLOCK];
        const bool yz = (y == 0 && g.face[2] != LBM_PERIODIC) || (y == g.ny - 1 && g.face[3] != LBM_PERIODIC) ||
                        (z == 0 && g.face[4] != LBM_PERIODIC) || (z == g.nz - 1 && g.face[5] != LBM_PERIODIC);
        if (yz) {
            pull_general<ST>(f, P.fin, xc, y, z, g, P.inlet);
        } else {
            const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
            const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
            const int ysrc[3] = {yp, y, ym};
            const int zsrc[3] = {zp, z, zm};
            if (active) {
                if (P.load32 && y > 0 && y < g.ny - 1 && z > 0 && z < g.nz - 1) {
                    // 32-bit offsets from the lowest source row (see pull_interior32)
                    const int row0 = (z - 1) * g.ny + (y - 1);
                    const BufRsrc rs = make_rsrc(P.fin + row_off(g, row0), P.span);
                    const int lr = g.lr, rmask = (int)g.rmask, hi0 = row0 >> lr, lo0 = row0 & rmask;
                    uint32_t rb[3][3];
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            const int rw = row0 + (2 - a) * g.ny + (2 - b);
                            const int el = ((rw >> lr) - hi0) * (int)g.bstride + ((rw & rmask) - lo0) * g.nxp;
                            rb[a][b] = (uint32_t)el * (uint32_t)sizeof(T);
                        }
                    const uint32_t plane_b = (uint32_t)g.plane * (uint32_t)sizeof(T), xb = (uint32_t)(x * sizeof(T));
#pragma unroll
                    for (int i = 0; i < Q; ++i) row[i][x] = buf_ld<T>(rs, xb, rb[CZ[i] + 1][CY[i] + 1] + (uint32_t)i * plane_b);
                } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                        row[i][x] = P.fin[(int64_t)i * g.plane + row_off(g, ysrc[CY[i] + 1], zsrc[CZ[i] + 1]) + x];
                }
            }
            __syncthreads();
            const int xm = xc == 0 ? g.nx - 1 : xc - 1, xp = xc == g.nx - 1 ? 0 : xc + 1;
            const int xsrc[3] = {xp, xc, xm};
#pragma unroll
            for (int i = 0; i < Q; ++i) f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = Store<ST>::dec(row[i][xsrc[CX[i] + 1]]);
        }
    } else if (B32 && P.load32) {
        pull_wave32<ST>(f, P.fin, xs, xc, y, z, g, P.inlet, P.span);
    } else {
        pull_wave<ST>(f, P.fin, xs, xc, y, z, g, P.inlet);
    }
    collide_as<COLL>(f, Fx, Fy, Fz, P.rt, rho, ux, uy, uz);
    }
    PushRows pr;
    if (feeds) push_rows(pt, feeds, pr);
    if (active) {
        if constexpr (B32 && LBM_BUF_STORES) {
            const BufRsrc rout = make_rsrc(P.fout + row_off(g, y, z), (uint32_t)(Q * g.plane * (int64_t)sizeof(T)));
            const uint32_t xb = (uint32_t)(x * sizeof(T));
#pragma unroll
            for (int i = 0; i < Q; ++i)
                buf_st_nt<T>(Store<ST>::enc(f[CZ[i] + 1][CY[i] + 1][CX[i] + 1]), rout, xb,
                             (uint32_t)i * (uint32_t)(g.plane * (int64_t)sizeof(T)));
        } else {
            const int64_t base = row_off(g, y, z) + x;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                __builtin_nontemporal_store(Store<ST>::enc(f[CZ[i] + 1][CY[i] + 1][CX[i] + 1]),
                                            P.fout + (int64_t)i * g.plane + base);
        }
    }
    if (feeds) push_band<ST>(P, f, feeds, pr, lane);
    if (SCALAR) scalar_update<ST>(P, xc, y, z, (float)ux, (float)uy, (float)uz, active);
    // lanes in the row's x padding (nx <= x < nxp, last segment only) store
    // zeros, so that every byte of a state this kernel writes is defined (a
    // state written straight into a tape slot equals a copy of the same state)
    if (xs == g.ntx - 1 && !active && x < g.nxp) {
        const int64_t base = row_off(g, y, z) + x;
#pragma unroll
        for (int i = 0; i < Q; ++i) P.fout[(int64_t)i * g.plane + base] = (T)0;
        if (SCALAR) P.sc_out[((int64_t)z * g.ny + y) * g.nxp + x] = 0.f;
    }
}

// ---------------------------------------------------------------------------
// band pre-pass: streamed rho and u0 = j/rho of every band node
// ---------------------------------------------------------------------------
template <int ST>
__device__ __forceinline__ void band_node(const StepParams<ST> &P, const int32_t *__restrict__ band_cell, int64_t b,
                                          typename StepParams<ST>::R4 *__restrict__ band_ru)
{
    using R = typename Store<ST>::R;
    const Geom &g = P.g;
    const int64_t cell = band_cell[b];
    const int x = (int)(cell % g.nx);
    const int64_t r = cell / g.nx;
    const int y = (int)(r % g.ny), z = (int)(r / g.ny);
    const Macro<R> m = band_interior(g, x, y, z) ? band_moments<ST>(P, b, x, y, z)
                                                 : node_moments<ST>(P.fin, x, y, z, g, P.inlet);
    const R rho = (R)1 + m.drho, inv = (R)1 / rho;
    typename StepParams<ST>::R4 v;
    v.x = rho;
    v.y = m.jx * inv;
    v.z = m.jy * inv;
    v.w = m.jz * inv;
    band_ru[b] = v;
}

// LOOP = false: one lane per band node, the count `known` from the host.
// LOOP = true: the count is read on the device (the set-up of a moving solid
// does not wait for it) and the lanes loop over it.  Two variants, because
// the loop keeps the kernel arguments live across iterations (about 100 more
// scalar registers spilled).
template <int ST, bool LOOP>
__global__ void __launch_bounds__(256)
    k_band(const StepParams<ST> P, const int32_t *__restrict__ band_cell, int64_t known, const int32_t *__restrict__ counts,
           typename StepParams<ST>::R4 *__restrict__ band_ru)
{
    const int64_t b0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (LOOP) {
        const int64_t nband = counts[0];
        for (int64_t b = b0; b < nband; b += (int64_t)gridDim.x * blockDim.x) band_node<ST>(P, band_cell, b, band_ru);
    } else {
        if (b0 < known) band_node<ST>(P, band_cell, b0, band_ru);
    }
}

// ---------------------------------------------------------------------------
// immersed boundary (Eqs. 6-8), spreading in two deterministic phases.  The
// samples of one base cell are contiguous in the sorted order (Sec. 4.2.2);
// a "run" is such a group cut at every multiple of 64 sorted samples, so
// that no run leaves the 64-sample window of one wavefront.  A cell whose
// samples straddle a window boundary has two runs; the second is marked as
// continuing the first (run_cont).
//   k_ib_seg (default): one lane per sample.  Each lane interpolates (Eq. 6),
//     forms its penalty force (Eq. 7) and its 24 spreading terms
//     a_s K_d g_s (8 offsets d x 3 components); a segmented inclusive scan
//     across the wavefront sums them per run (the wavefront-level reduction
//     that replaces the paper's atomics), and the last lane of each run
//     stores the run's 8 sums.  Work per lane is the same for every sample,
//     however the samples are spread over cells (Sec. 4.3, Table 1).
//   k_ib_run: one lane per run, looping over the run's samples with the 8
//     stencil nodes loaded once (the lane's time grows with its run length).
//   k_spread: one lane per band node gathers, per offset, the sums of the
//     run(s) of the cell that targets it, in a fixed order.
// No floating-point atomics anywhere: the step is bit-reproducible.
// ---------------------------------------------------------------------------
constexpr int64_t IB_SEG_MAX_BLOCKS = 4096;  // grid of k_ib_seg (FP64 partials summed by k_ib_total)

template <typename R> struct IbParams {
    using R4 = typename R4T<R>::type;
    int64_t n, rstride;                     // samples; stride of run_sum (its capacity)
    const int32_t *__restrict__ counts;     // device {band nodes, runs}
    const int32_t *__restrict__ run_start;  // [nruns + 1]
    const int32_t *__restrict__ run_id;     // [n] run of each sorted sample
    const float *__restrict__ pos;          // [3][n] sorted
    const float *__restrict__ ub;           // [3][n]
    const float *__restrict__ area;         // [n]
    const float *__restrict__ gain;         // [n]
    const int32_t *__restrict__ slot;       // [8][n]
    const R4 *__restrict__ band_ru;
    R4 *__restrict__ run_sum;               // [8][rstride]
    double *__restrict__ part;              // [gridDim.x][8] per-block force and torque totals
    double ox, oy, oz;                      // reference point of the torque
};

// FP64 force and torque of the block's lanes into one partial per block
// (wave reduction, then the block's waves in order; no same-address atomics)
__device__ __forceinline__ void block_partial6(double (&tot)[6], double *__restrict__ part)
{
    __shared__ double wsum[4][6];
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 6; ++a) tot[a] += __shfl_down(tot[a], off, 64);
    if (lane == 0)
#pragma unroll
        for (int a = 0; a < 6; ++a) wsum[threadIdx.x >> 6][a] = tot[a];
    __syncthreads();
    if (threadIdx.x < 6)
        part[8 * blockIdx.x + threadIdx.x] =
            wsum[0][threadIdx.x] + wsum[1][threadIdx.x] + wsum[2][threadIdx.x] + wsum[3][threadIdx.x];
}

template <typename R>
__global__ void __launch_bounds__(256) k_ib_run(const IbParams<R> P)
{
    using R4 = typename R4T<R>::type;
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = P.n;
    double tot[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // force, then torque about (ox, oy, oz)
    if (r < P.counts[1]) {
        const int64_t k0 = P.run_start[r], k1 = P.run_start[r + 1];
        R4 node[8];
#pragma unroll
        for (int d = 0; d < 8; ++d) node[d] = P.band_ru[P.slot[(int64_t)d * n + k0]];
        R acc[8][3];
#pragma unroll
        for (int d = 0; d < 8; ++d) acc[d][0] = acc[d][1] = acc[d][2] = (R)0;
        for (int64_t k = k0; k < k1; ++k) {
            R t[3];
            float p[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p[a] = P.pos[a * n + k];
                t[a] = (R)(p[a] - floorf(p[a]));
            }
            R K[8], rs = 0, us[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                K[d] = ((d & 1) ? t[0] : (R)1 - t[0]) * ((d & 2) ? t[1] : (R)1 - t[1]) * ((d & 4) ? t[2] : (R)1 - t[2]);
                rs += K[d] * node[d].x;
                us[0] += K[d] * node[d].y;
                us[1] += K[d] * node[d].z;
                us[2] += K[d] * node[d].w;
            }
            // Eq. (7) with the sample's gain; Eq. (8) carries the area weight
            const R ag = (R)P.area[k] * (R)P.gain[k] * rs;
            R aG[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                aG[a] = ag * ((R)P.ub[a * n + k] - us[a]);
                tot[a] += (double)aG[a];
            }
            // Alg. 2 (c) torque: (x_s - o) x (a_s g_s), lever arm in FP64
            const double rx = (double)p[0] - P.ox, ry = (double)p[1] - P.oy, rz = (double)p[2] - P.oz;
            tot[3] += ry * (double)aG[2] - rz * (double)aG[1];
            tot[4] += rz * (double)aG[0] - rx * (double)aG[2];
            tot[5] += rx * (double)aG[1] - ry * (double)aG[0];
#pragma unroll
            for (int d = 0; d < 8; ++d)
#pragma unroll
                for (int a = 0; a < 3; ++a) acc[d][a] += K[d] * aG[a];
        }
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            R4 v;
            v.x = acc[d][0];
            v.y = acc[d][1];
            v.z = acc[d][2];
            v.w = (R)0;
            P.run_sum[(int64_t)d * P.rstride + r] = v;
        }
    }
    block_partial6(tot, P.part);
}

template <typename R>
__global__ void __launch_bounds__(256) k_ib_seg(const IbParams<R> P)
{
    using R4 = typename R4T<R>::type;
    const int64_t n = P.n;
    const int lane = threadIdx.x & 63;  // == k mod 64: runs restart at every window
    double tot[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // force, then torque about (ox, oy, oz)
    // grid-stride over 256-sample chunks (a bounded grid keeps the number of
    // FP64 block partials small); every lane of a wave runs the same trips
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k - lane < n;
         k += (int64_t)gridDim.x * blockDim.x) {
        const bool valid = k < n;
        const int32_t c0 = valid ? P.slot[k] : -1;  // band slot of the base cell (offset 0) names the cell
        const int32_t cprev = __shfl_up(c0, 1, 64);
        const bool head = valid && (lane == 0 || c0 != cprev);
        const uint64_t heads = __ballot(head);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const uint64_t hle = heads & upto;
        const int first = hle ? 63 - __clzll(hle) : lane;  // first lane of this lane's run
        const int dist = valid ? lane - first : 0;
        const bool last = valid && (lane == 63 || k + 1 == n || ((heads >> (lane + 1)) & 1ull));

        R v[8][3];
#pragma unroll
        for (int d = 0; d < 8; ++d) v[d][0] = v[d][1] = v[d][2] = (R)0;
        if (valid) {
            R t[3];
            float p[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p[a] = P.pos[a * n + k];
                t[a] = (R)(p[a] - floorf(p[a]));
            }
            R K[8], rs = 0, us[3] = {0, 0, 0};
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const R4 node = P.band_ru[P.slot[(int64_t)d * n + k]];
                K[d] = ((d & 1) ? t[0] : (R)1 - t[0]) * ((d & 2) ? t[1] : (R)1 - t[1]) * ((d & 4) ? t[2] : (R)1 - t[2]);
                rs += K[d] * node.x;
                us[0] += K[d] * node.y;
                us[1] += K[d] * node.z;
                us[2] += K[d] * node.w;
            }
            // Eq. (7) with the sample's gain; Eq. (8) carries the area weight
            const R ag = (R)P.area[k] * (R)P.gain[k] * rs;
            R aG[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                aG[a] = ag * ((R)P.ub[a * n + k] - us[a]);
                tot[a] += (double)aG[a];
            }
            // Alg. 2 (c) torque: (x_s - o) x (a_s g_s), lever arm in FP64
            const double rx = (double)p[0] - P.ox, ry = (double)p[1] - P.oy, rz = (double)p[2] - P.oz;
            tot[3] += ry * (double)aG[2] - rz * (double)aG[1];
            tot[4] += rz * (double)aG[0] - rx * (double)aG[2];
            tot[5] += rx * (double)aG[1] - ry * (double)aG[0];
#pragma unroll
            for (int d = 0; d < 8; ++d)
#pragma unroll
                for (int a = 0; a < 3; ++a) v[d][a] = K[d] * aG[a];
        }
        // segmented inclusive scan: after the steps with offsets 1, 2, 4, ...
        // up to the longest run, the last lane of a run holds the run's sums
        // (a fixed tree order, so repeated runs give the same bits)
        int span = dist;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) span = max(span, __shfl_xor(span, off, 64));
        span = __builtin_amdgcn_readfirstlane(span);
        for (int off = 1; off <= span; off <<= 1) {
#pragma unroll
            for (int d = 0; d < 8; ++d)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R up = __shfl_up(v[d][a], off, 64);
                    if (dist >= off) v[d][a] += up;
                }
        }
        if (last) {
            const int64_t r = (int64_t)P.run_id[k - lane] + (int64_t)__popcll(hle) - 1;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                R4 w;
                w.x = v[d][0];
                w.y = v[d][1];
                w.z = v[d][2];
                w.w = (R)0;
                P.run_sum[(int64_t)d * P.rstride + r] = w;
            }
        }
    }
    block_partial6(tot, P.part);
}

template <typename R>
__global__ void __launch_bounds__(256) k_spread(int64_t known, const int32_t *__restrict__ counts, int64_t bstride,
                                                int64_t rstride,
                                                const int32_t *__restrict__ band_src,
                                                const uint8_t *__restrict__ run_cont,
                                                const typename R4T<R>::type *__restrict__ run_sum,
                                                typename R4T<R>::type *__restrict__ band_force)
{
    const int64_t nband = known >= 0 ? known : counts[0];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nband; j += (int64_t)gridDim.x * blockDim.x) {
        typename R4T<R>::type g;
        g.x = g.y = g.z = g.w = (R)0;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            int64_t src = band_src[(int64_t)d * bstride + j];
            if (src >= 0) {
                // the first run of the cell, then any runs continuing it (the
                // entry after the last run is 0)
                for (;;) {
                    const auto v = run_sum[(int64_t)d * rstride + src];
                    g.x += v.x;
                    g.y += v.y;
                    g.z += v.z;
                    if (!run_cont[src + 1]) break;
                    ++src;
                }
            }
        }
        band_force[j] = g;
    }
}

// ordered sum of the per-block force and torque partials (deterministic FP64 totals);
// a template so that every storage's translation unit may hold its copy
template <int UNUSED = 0>
__global__ void __launch_bounds__(256) k_ib_total(const double *__restrict__ part, int nblk, double *__restrict__ ftot)
{
    __shared__ double sh[6][256];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
        for (int a = 0; a < 6; ++a) acc[a] += part[8 * b + a];
#pragma unroll
    for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int a = 0; a < 6; ++a) sh[a][threadIdx.x] += sh[a][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 6) ftot[threadIdx.x] = sh[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <int ST> StepParams<ST> make_params(lbm_ctx *c)
{
    using R = typename Store<ST>::R;
    using T = typename Store<ST>::T;
    StepParams<ST> P{};
    P.g = c->g;
    P.fin = static_cast<const T *>(c->fA);
    P.fout = static_cast<T *>(c->fB);
    P.rt = {(R)c->s_nu, (R)c->s_b, (R)c->s_h[0], (R)c->s_h[1], (R)c->s_h[2], (R)c->s_h[3]};
    for (int a = 0; a < 3; ++a) {
        P.body[a] = (R)c->p.body_force[a];
        P.inlet.u[a] = (R)c->p.u_in[a];
    }
    P.inlet.prof = static_cast<const R *>(c->p.inlet_profile);
    P.tile_mask = c->tile_mask;
    P.tile_start = c->tile_start;
    P.band_force = static_cast<const typename StepParams<ST>::R4 *>(c->band_force);
    P.fused_spread = fused_spread(c) ? 1 : 0;
    P.bstride = c->nbcap;
    P.rstride = c->nm;
    P.band_src = c->band_src;
    P.run_cont = c->run_cont;
    P.run_sum = static_cast<const typename StepParams<ST>::R4 *>(c->run_sum);
    P.sc_in = c->scA;
    P.sc_out = c->scB;
    P.sc_h = c->p.scalar_inlet_height;
    P.load32 = c->load32 ? 1 : 0;
    P.span = c->span32;
    P.one = 1.0f;
    P.push_out = nullptr;
    P.push_in = nullptr;
    P.push_feeds = c->push_feeds;
    return P;
}

static inline unsigned blocks_for_items(int64_t W) { return (unsigned)((W + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK); }

template <int ST, bool B32, int COLL> static void fused_launch(lbm_ctx *c, const StepParams<ST> &P)
{
    const bool band = c->nm > 0, scalar = c->p.passive_scalar != 0;
    const dim3 grid(blocks_for_items(c->g.W)), block(SEG * WAVES_PER_BLOCK);
    if (band && scalar) hipLaunchKernelGGL((k_fused<ST, true, true, B32, false, COLL>), grid, block, 0, c->stream, P);
    else if (band) hipLaunchKernelGGL((k_fused<ST, true, false, B32, false, COLL>), grid, block, 0, c->stream, P);
    else if (scalar) hipLaunchKernelGGL((k_fused<ST, false, true, B32, false, COLL>), grid, block, 0, c->stream, P);
    else if (B32 && c->row_stage)
        hipLaunchKernelGGL((k_fused<ST, false, false, B32, B32, COLL>), grid, block, 0, c->stream, P);
    else hipLaunchKernelGGL((k_fused<ST, false, false, B32, false, COLL>), grid, block, 0, c->stream, P);
}

// the fused step of one storage form and one collision model
template <int ST, int COLL> hipError_t fused_st(lbm_ctx *c)
{
    StepParams<ST> P = make_params<ST>(c);
    if (band_push_on(c)) P.push_out = static_cast<typename StepParams<ST>::R2 *>(c->band_push);
    if constexpr (ST != LBM_F64) {
        if (c->buffer_path) fused_launch<ST, true, COLL>(c, P);
        else fused_launch<ST, false, COLL>(c, P);
    } else {
        fused_launch<ST, false, COLL>(c, P);
    }
    return hipGetLastError();
}

// Grid of the per-band-node kernels, which loop over the device's band count:
// one lane per node when the count is known, else room for a quarter more
// than the last count read (a moving solid's band changes little per step).
inline unsigned band_blocks(const lbm_ctx *c)
{
    int64_t want = c->nband;
    if (!c->counts_exact) want = std::min<int64_t>(c->nbcap, c->nband + c->nband / 4 + 4096);
    const int64_t nb = (want + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(nb, 1 << 20));
}

template <int ST> hipError_t band_ib_st(lbm_ctx *c, const void *state, double *ftot, bool spread, bool pieces)
{
    using R = typename Store<ST>::R;
    using R4 = typename StepParams<ST>::R4;
    StepParams<ST> P = make_params<ST>(c);
    P.fin = static_cast<const typename Store<ST>::T *>(state);
    if (pieces) P.push_in = static_cast<const typename StepParams<ST>::R2 *>(c->band_push);
    const unsigned nb = band_blocks(c);
    const int64_t known = c->counts_exact ? c->nband : -1;
    if (known >= 0)
        hipLaunchKernelGGL((k_band<ST, false>), dim3(nb), dim3(256), 0, c->stream, P, c->band_cell, known, c->dcounts,
                           static_cast<R4 *>(c->band_ru));
    else
        hipLaunchKernelGGL((k_band<ST, true>), dim3(nb), dim3(256), 0, c->stream, P, c->band_cell, known, c->dcounts,
                           static_cast<R4 *>(c->band_ru));
    IbParams<R> Q{};
    Q.n = c->nm;
    Q.rstride = c->nm;
    Q.counts = c->dcounts;
    Q.run_start = c->run_start;
    Q.run_id = c->run_id;
    Q.pos = c->m_pos;
    Q.ub = c->m_ub;
    Q.area = c->m_area;
    Q.gain = c->m_gain;
    Q.slot = c->m_slot;
    Q.band_ru = static_cast<const R4 *>(c->band_ru);
    Q.run_sum = static_cast<R4 *>(c->run_sum);
    Q.part = c->ib_part;
    Q.ox = c->pose_o[0];
    Q.oy = c->pose_o[1];
    Q.oz = c->pose_o[2];
    // lane per run: the run count is on the device, at most one run per sample
    const int nblk = c->ib_lane_per_run ? (int)((c->nm + 255) / 256)
                                        : (int)std::min<int64_t>(IB_SEG_MAX_BLOCKS, (c->nm + 255) / 256);
    if (c->ib_lane_per_run) hipLaunchKernelGGL((k_ib_run<R>), dim3((unsigned)nblk), dim3(256), 0, c->stream, Q);
    else hipLaunchKernelGGL((k_ib_seg<R>), dim3((unsigned)nblk), dim3(256), 0, c->stream, Q);
    hipLaunchKernelGGL(k_ib_total<>, dim3(1), dim3(256), 0, c->stream, c->ib_part, nblk, ftot);
    if (spread)
        hipLaunchKernelGGL((k_spread<R>), dim3(nb), dim3(256), 0, c->stream, known, c->dcounts, c->nbcap, c->nm,
                           c->band_src, c->run_cont, static_cast<const R4 *>(c->run_sum),
                           static_cast<R4 *>(c->band_force));
    return hipGetLastError();
}

}  // namespace lbm
