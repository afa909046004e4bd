// lbm_internal.hpp -- device building blocks shared by the liblbm kernels.
//
// Populations are held as deviations d_i = f_i - w_i from the lattice weights
// in every storage form.  The collision (Sec. 3, Eqs. 4-5) is written in the
// factorised form the paper's Sec. 4.4.2 argues for (shared monomials
// u_x^p u_y^q u_z^r computed once): a separable raw-moment transform along x,
// y and z, a separable binomial shift to central moments about u, relaxation,
// and the inverse path.  All of it stays in registers; the deviation form keeps
// every intermediate small, which is what lets FP32 track the FP64 reference.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "lbm.h"

namespace lbm {

constexpr int Q = 27;

// Lattice order (see lbm.h): rest, faces, edges (xy, xz, yz), corners; sign
// patterns with x fastest inside each group.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1};

constexpr int pop_index(int cx, int cy, int cz)
{
    for (int i = 0; i < Q; ++i)
        if (CX[i] == cx && CY[i] == cy && CZ[i] == cz) return i;
    return -1;
}
constexpr int opp(int i) { return pop_index(-CX[i], -CY[i], -CZ[i]); }
constexpr double weight(int i)
{
    return (CX[i] ? 1.0 / 6.0 : 2.0 / 3.0) * (CY[i] ? 1.0 / 6.0 : 2.0 / 3.0) * (CZ[i] ? 1.0 / 6.0 : 2.0 / 3.0);
}

// population index by (cx+1) + 3 (cy+1) + 9 (cz+1), for run-time lookups
__device__ __constant__ const int8_t POP_OF[27] = {
    pop_index(-1, -1, -1), pop_index(0, -1, -1), pop_index(1, -1, -1), pop_index(-1, 0, -1), pop_index(0, 0, -1),
    pop_index(1, 0, -1),   pop_index(-1, 1, -1), pop_index(0, 1, -1),  pop_index(1, 1, -1),  pop_index(-1, -1, 0),
    pop_index(0, -1, 0),   pop_index(1, -1, 0),  pop_index(-1, 0, 0),  pop_index(0, 0, 0),   pop_index(1, 0, 0),
    pop_index(-1, 1, 0),   pop_index(0, 1, 0),   pop_index(1, 1, 0),   pop_index(-1, -1, 1), pop_index(0, -1, 1),
    pop_index(1, -1, 1),   pop_index(-1, 0, 1),  pop_index(0, 0, 1),   pop_index(1, 0, 1),   pop_index(-1, 1, 1),
    pop_index(0, 1, 1),    pop_index(1, 1, 1)};

// ---------------------------------------------------------------------------
// storage codecs
// ---------------------------------------------------------------------------

template <int ST> struct Store;
template <> struct Store<LBM_F32> {
    using T = float;
    using R = float;
    __device__ static R dec(T v) { return v; }
    __device__ static T enc(R v) { return v; }
};
template <> struct Store<LBM_F64> {
    using T = double;
    using R = double;
    __device__ static R dec(T v) { return v; }
    __device__ static T enc(R v) { return v; }
};
template <> struct Store<LBM_F16DEV> {
    using T = uint16_t;
    using R = float;
    __device__ static R dec(T v) { return __half2float(__ushort_as_half(v)); }
    __device__ static T enc(R v) { return __half_as_ushort(__float2half_rn(v)); }
};
template <> struct Store<LBM_BF16DEV> {
    using T = uint16_t;
    using R = float;
    __device__ static R dec(T v) { return __uint_as_float(((uint32_t)v) << 16); }
    // round to nearest even (gfx950 converts natively: v_cvt_pk_bf16_f32)
    __device__ static T enc(R v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
};

// ---------------------------------------------------------------------------
// geometry shared by every kernel
// ---------------------------------------------------------------------------

// Build-time tuning switches (values chosen by measurement on MI355X).
#ifndef LBM_NT_LOADS
#define LBM_NT_LOADS 0      // population reads with the non-temporal (streaming) hint
#endif
#ifndef LBM_WAVES
#define LBM_WAVES 4         // wavefronts per workgroup of the fused kernel
#endif
#ifndef LBM_XCD_REMAP
#define LBM_XCD_REMAP 0     // contiguous logical blocks per XCD (off: all XCDs share one moving front)
#endif
#ifndef LBM_BUF_STORES
#define LBM_BUF_STORES 1    // fused-kernel stores through a per-row buffer descriptor
#endif

// Work item = one x-segment of 64 nodes of one (y, z) row; a wavefront owns
// one work item, a workgroup LBM_WAVES consecutive ones.
constexpr int SEG = 64;
constexpr int WAVES_PER_BLOCK = LBM_WAVES;

// base + 32-bit byte offset: with a wave-uniform base this selects the
// scalar-base / 32-bit vector-offset memory form (no 64-bit address math)
template <typename T> __device__ __forceinline__ const T *at_bytes(const T *base, uint32_t byte_off)
{
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T> __device__ __forceinline__ T *at_bytes(T *base, uint32_t byte_off)
{
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}

// streaming read of a population (used once per step, except the one-element
// overlap of neighbouring segments, which the L2 still catches)
template <typename T> __device__ __forceinline__ T ld_stream(const T *p)
{
#if LBM_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// Population layout.  Rows (row = z*ny + y) are grouped into blocks of
// R = 2^lr rows stored as [block][27][R][nxp]: population i of node (x, row)
// sits at (row >> lr) * bstride + i * plane + (row & rmask) * nxp + x, with
// plane = R*nxp and bstride = 27*R*nxp.  Each block is one contiguous region,
// so a wave's 27 loads (and 27 stores) fall in a few nearby DRAM pages instead
// of 27 distant planes.  lr = 31 is the plain plane-major layout [27][rows][nxp]
// (one block; plane = padded rows*nxp).
// Division by an invariant divisor d (1 <= d < 2^31) of numerators n < 2^31:
// q = (n * m) >> (31 + l) with l = ceil(log2 d) and m = ceil(2^(31+l) / d).
// m = (2^(31+l) + e) / d with 0 <= e < d <= 2^l, so n*m / 2^(31+l) exceeds n/d
// by less than n*e / (d 2^(31+l)) < 1/d: the floor is exact (the round-up
// method for invariant divisors).  m <= 2^32 + 1, so n*m fits in 64 bits.
struct Divisor {
    uint64_t m;
    int sh;
};
inline Divisor make_divisor(uint32_t d)
{
    int l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t p = uint64_t(1) << (31 + l);
    return {p / d + (p % d != 0), 31 + l};
}
__host__ __device__ __forceinline__ uint32_t divide(uint32_t n, const Divisor &d)
{
    return (uint32_t)(((uint64_t)n * d.m) >> d.sh);
}

struct Geom {
    int nx, ny, nz;
    int nxp;         // row pitch (elements), multiple of 32
    int ntx;         // segments per row
    int lr;          // log2 of the rows per block
    int64_t rmask;   // rows per block - 1
    int64_t plane;   // stride between populations inside a block (elements)
    int64_t bstride; // stride between blocks (elements)
    int64_t total;   // elements of one population copy
    int64_t W;       // number of work items (< 2^31)
    Divisor dntx, dny;
    int face[6];
};

// work item w -> (segment, y, z); all three are wave-uniform
__device__ __forceinline__ void wave_coords(uint32_t w, const Geom &g, int &xs, int &y, int &z)
{
    const uint32_t row = divide(w, g.dntx);
    xs = (int)(w - row * (uint32_t)g.ntx);
    const uint32_t zz = divide(row, g.dny);
    y = (int)(row - zz * (uint32_t)g.ny);
    z = (int)zz;
}

__host__ __device__ __forceinline__ int64_t row_off(const Geom &g, int64_t row)
{
    return (row >> g.lr) * g.bstride + (row & g.rmask) * g.nxp;
}
__host__ __device__ __forceinline__ int64_t row_off(const Geom &g, int y, int z)
{
    return row_off(g, (int64_t)z * g.ny + y);
}

// Face-layer nodes, enumerated densely (one lane each): part A = every node
// of the rows on a non-periodic y or z face (y faces first: y = 0, ny-1 for
// each z; then z = 0, nz-1 for the y not on a y face); part B = the two x-face
// nodes (x = 0, nx-1) of every other row, when the x faces are non-periodic.
struct FaceSet {
    int yf, zf, xf;     // axes with non-periodic faces
    int ry, rz;         // rows of part A on y faces / on z faces
    int y0, ny1, z0;    // part B rows: y in [y0, y0 + ny1), z from z0
    int64_t na, nb;     // node counts of parts A and B
};
__host__ __device__ inline FaceSet face_set(const Geom &g)
{
    FaceSet F{};
    F.yf = g.face[2] != LBM_PERIODIC;
    F.zf = g.face[4] != LBM_PERIODIC;
    F.xf = g.face[0] != LBM_PERIODIC;
    F.ry = F.yf ? 2 * g.nz : 0;
    F.y0 = F.yf ? 1 : 0;
    F.ny1 = g.ny - 2 * F.y0;
    F.rz = F.zf ? 2 * F.ny1 : 0;
    F.z0 = F.zf ? 1 : 0;
    F.na = (int64_t)(F.ry + F.rz) * g.nx;
    const int64_t other = (int64_t)F.ny1 * (g.nz - 2 * F.z0);
    F.nb = F.xf ? 2 * other : 0;
    return F;
}
__host__ __device__ __forceinline__ void face_node(int64_t k, const Geom &g, const FaceSet &F, int &x, int &y, int &z)
{
    if (k < F.na) {
        const int r = (int)(k / g.nx);
        x = (int)(k - (int64_t)r * g.nx);
        if (r < F.ry) {
            y = (r & 1) ? g.ny - 1 : 0;
            z = r >> 1;
        } else {
            const int q = r - F.ry;
            z = (q & 1) ? g.nz - 1 : 0;
            y = F.y0 + (q >> 1);
        }
    } else {
        const int64_t b = k - F.na;
        x = (b & 1) ? g.nx - 1 : 0;
        const int64_t r = b >> 1;
        y = F.y0 + (int)(r % F.ny1);
        z = F.z0 + (int)(r / F.ny1);
    }
}

// Raw buffer access: the descriptor holds a wave-uniform 64-bit base, the
// uniform part of an offset goes in a scalar register (soffset) and the
// per-lane part in a 32-bit vector register, so an access costs no vector
// address arithmetic.  Descriptor word 3 is the gfx9 raw-buffer format.
using BufRsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ BufRsrc make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_ld(BufRsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float buf_ld<float>(BufRsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ uint16_t buf_ld<uint16_t>(BufRsrc r, uint32_t voff, uint32_t soff)
{
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
// non-temporal store (aux bit 1 = nt)
template <typename T> __device__ __forceinline__ void buf_st_nt(T v, BufRsrc r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ void buf_st_nt<float>(float v, BufRsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 2);
}
template <> __device__ __forceinline__ void buf_st_nt<uint16_t>(uint16_t v, BufRsrc r, uint32_t voff, uint32_t soff)
{
    __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)voff, (int)soff, 2);
}

// Workgroups are dispatched round-robin over the 8 XCDs.  The remap gives each
// XCD a contiguous range of logical blocks, so that x-neighbouring segments
// (which share cache lines at their edges) land in the same L2.  Measured on
// MI355X it is slower (23.1 vs 25.8 GLUPS at 256^3 FP32): with plain dispatch
// order all XCDs stream through one narrow front of the domain, which keeps
// DRAM pages open, and the shared edge lines are caught by the Infinity Cache.
__device__ __forceinline__ int xcd_remap(int bid, int nb)
{
#if !LBM_XCD_REMAP
    return bid;
#endif
    const int xcd = bid & 7, local = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + local;
}

__device__ __forceinline__ int face_rank(int f)
{
    return f == LBM_NOSLIP ? 4 : f == LBM_INLET ? 3 : f == LBM_OUTFLOW ? 2 : f == LBM_FREESLIP ? 1 : 0;
}

// Source of the streamed population f*_i at node (x, y, z) under the face
// rules: plane `pl` at node (sx, sy, sz); `inlet` = add the wall-velocity term
// of the inlet at row (sy, sz).  At most one inward move (outflow) happens.
struct PullSrc {
    int pl, sx, sy, sz, inlet;
};

__device__ __forceinline__ PullSrc resolve(int i, int x, int y, int z, const Geom &g)
{
    const int cx = CX[i], cy = CY[i], cz = CZ[i];
    int px = x, py = y, pz = z;
    for (int pass = 0; pass < 2; ++pass) {
        int sx = px - cx, sy = py - cy, sz = pz - cz;
        int crossed = 0, best = LBM_PERIODIC, bestrank = 0, baxis = 0, bside = 0;
        // one axis at a time; every index below is a named scalar (no local arrays)
        auto axis = [&](int a, int &sv, int n, int fm, int fp) {
            int side = -1;
            if (sv < 0) side = 0;
            else if (sv >= n) side = 1;
            if (side < 0) return;
            const int fc = side ? fp : fm;
            if (fc == LBM_PERIODIC) {
                sv += side ? -n : n;
                return;
            }
            crossed |= 1 << a;
            const int r = face_rank(fc);
            if (r > bestrank) {
                bestrank = r;
                best = fc;
                baxis = a;
                bside = side;
            }
        };
        axis(0, sx, g.nx, g.face[0], g.face[1]);
        axis(1, sy, g.ny, g.face[2], g.face[3]);
        axis(2, sz, g.nz, g.face[4], g.face[5]);
        if (best == LBM_PERIODIC) return {i, sx, sy, sz, 0};
        if (best == LBM_NOSLIP) return {opp(i), px, py, pz, 0};
        if (best == LBM_INLET) return {opp(i), px, py, pz, 1};
        if (best == LBM_OUTFLOW) {
            const int d = bside ? -1 : 1;
            if (baxis == 0) px += d;
            else if (baxis == 1) py += d;
            else pz += d;
            continue;
        }
        // free slip: reflect the crossed components, stay on the node's layer
        int rx = cx, ry = cy, rz = cz;
        if (crossed & 1) {
            rx = -rx;
            sx = px;
        }
        if (crossed & 2) {
            ry = -ry;
            sy = py;
        }
        if (crossed & 4) {
            rz = -rz;
            sz = pz;
        }
        return {POP_OF[(rx + 1) + 3 * (ry + 1) + 9 * (rz + 1)], sx, sy, sz, 0};
    }
    return {i, px, py, pz, 0};  // not reached for valid geometry
}

// Inlet velocity at row (y, z): profile [3][nz][ny] or uniform.
template <typename R> struct Inlet {
    const R *prof;
    R u[3];
    __device__ R at(int a, int y, int z, int ny, int nz) const
    {
        return prof ? prof[((int64_t)a * nz + z) * ny + y] : u[a];
    }
};

// One streamed deviation of node (x, y, z), general face-aware path.
template <int ST, typename R>
__device__ __forceinline__ R pull_one(int i, const typename Store<ST>::T *__restrict__ in, int x, int y, int z,
                                      const Geom &g, const Inlet<R> &inl)
{
    const PullSrc s = resolve(i, x, y, z, g);
    const int64_t idx = (int64_t)s.pl * g.plane + row_off(g, s.sy, s.sz) + s.sx;
    R v = Store<ST>::dec(ld_stream(in + idx));
    if (s.inlet) {
        const R cu = (R)CX[i] * inl.at(0, s.sy, s.sz, g.ny, g.nz) + (R)CY[i] * inl.at(1, s.sy, s.sz, g.ny, g.nz) +
                     (R)CZ[i] * inl.at(2, s.sy, s.sz, g.ny, g.nz);
        v += (R)(6.0 * weight(i)) * cu;
    }
    return v;
}

template <int ST, typename R, int... I>
__device__ __forceinline__ void pull_general_seq(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x,
                                                 int y, int z, const Geom &g, const Inlet<R> &inl,
                                                 std::integer_sequence<int, I...>)
{
    ((f[CZ[I] + 1][CY[I] + 1][CX[I] + 1] = pull_one<ST, R>(I, in, x, y, z, g, inl)), ...);
}

// Pull the 27 deviations of node (x, y, z) into f[cz+1][cy+1][cx+1] with the
// face rules (population index expanded at compile time).
template <int ST, typename R>
__device__ __forceinline__ void pull_general(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x,
                                             int y, int z, const Geom &g, const Inlet<R> &inl)
{
    pull_general_seq<ST, R>(f, in, x, y, z, g, inl, std::make_integer_sequence<int, Q>{});
}

// Fast path for a wave away from non-periodic faces: pure pull with periodic
// wrap; row offsets are wave-uniform.
template <int ST, typename R>
__device__ __forceinline__ void pull_interior(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x,
                                              int y, int z, const Geom &g)
{
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const int xs[3] = {xp, x, xm};  // source x for c_x = -1, 0, +1
    const int ys[3] = {yp, y, ym};
    const int zs[3] = {zp, z, zm};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int64_t row = row_off(g, ys[CY[i] + 1], zs[CZ[i] + 1]);
        const typename Store<ST>::T *pl = in + (int64_t)i * g.plane + row;
        f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = Store<ST>::dec(ld_stream(pl + xs[CX[i] + 1]));
    }
}

// Interior pull with 32-bit offsets, for a row (y, z) away from every y and
// z face or wrap (1 <= y <= ny-2, 1 <= z <= nz-2): one buffer descriptor per
// wavefront based at its lowest source row (z-1, y-1), spanning `span`
// bytes; the (population, source row) part of each offset in a scalar
// register and the lane's source x in one of three vector registers (x - 1,
// x, x + 1, wrapped), so the 27 loads need no 64-bit address arithmetic,
// scalar or vector.  The host guarantees that the 9 source rows of any such
// row lie within `span` < 2^31 bytes of the base (blocked layout only).
template <int ST, typename R>
__device__ __forceinline__ void pull_interior32(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x,
                                                int y, int z, const Geom &g, uint32_t span)
{
    using T = typename Store<ST>::T;
    const int row0 = (z - 1) * g.ny + (y - 1);
    const BufRsrc rs = make_rsrc(in + row_off(g, row0), span);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const uint32_t xb[3] = {(uint32_t)(xp * (int)sizeof(T)), (uint32_t)(x * (int)sizeof(T)),
                            (uint32_t)(xm * (int)sizeof(T))};  // source x for c_x = -1, 0, +1
    const int lr = g.lr, rmask = (int)g.rmask, nxp = g.nxp, bstride = (int)g.bstride;
    const int hi0 = row0 >> lr, lo0 = row0 & rmask;
    const uint32_t plane_b = (uint32_t)g.plane * (uint32_t)sizeof(T);
    uint32_t rb[3][3];  // byte offset of source row (y + 1 - b, z + 1 - a) from the base
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int row = row0 + (2 - a) * g.ny + (2 - b);
            const int el = ((row >> lr) - hi0) * bstride + ((row & rmask) - lo0) * nxp;
            rb[a][b] = (uint32_t)el * (uint32_t)sizeof(T);
        }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] =
            Store<ST>::dec(buf_ld<T>(rs, xb[CX[i] + 1], rb[CZ[i] + 1][CY[i] + 1] + (uint32_t)i * plane_b));
}

// pull_interior32 for FP16 deviations, handing the raw halves on (for
// low_moments_f16)
__device__ __forceinline__ void pull_interior32_f16(_Float16 (&h)[3][3][3], const uint16_t *__restrict__ in, int x,
                                                    int y, int z, const Geom &g, uint32_t span)
{
    const int row0 = (z - 1) * g.ny + (y - 1);
    const BufRsrc rs = make_rsrc(in + row_off(g, row0), span);
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const uint32_t xb[3] = {(uint32_t)(xp * 2), (uint32_t)(x * 2), (uint32_t)(xm * 2)};
    const int lr = g.lr, rmask = (int)g.rmask, nxp = g.nxp, bstride = (int)g.bstride;
    const int hi0 = row0 >> lr, lo0 = row0 & rmask;
    const uint32_t plane_b = (uint32_t)g.plane * 2u;
    uint32_t rb[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int row = row0 + (2 - a) * g.ny + (2 - b);
            rb[a][b] = (uint32_t)(((row >> lr) - hi0) * bstride + ((row & rmask) - lo0) * nxp) * 2u;
        }
#pragma unroll
    for (int i = 0; i < Q; ++i)
        h[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = __builtin_bit_cast(
            _Float16, buf_ld<uint16_t>(rs, xb[CX[i] + 1], rb[CZ[i] + 1][CY[i] + 1] + (uint32_t)i * plane_b));
}

// Pull for a wave that touches a non-periodic x face but no y or z face (an
// x-segment at either end of a row).  Directions with c_x = 0 read as in the
// interior.  The others select per lane between the plain source and the face
// rule's source (lanes at x = 0 for c_x = +1, x = nx-1 for c_x = -1), so each
// population is still one load: no-slip / inlet read the opposite population
// at the node itself (the inlet adds 2 w_i (c_i.u_in)/cs^2), free slip reads
// the x-reflected population across y, z, outflow reads the last layer.
template <int ST, typename R>
__device__ __forceinline__ void pull_xface(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x, int y,
                                           int z, const Geom &g, const Inlet<R> &inl)
{
    using T = typename Store<ST>::T;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const int ys[3] = {yp, y, ym};
    const int zs[3] = {zp, z, zm};
    const int64_t row_own = row_off(g, y, z);
    const int F0 = g.face[0], F1 = g.face[1];
    const bool lo = x == 0, hi = x == g.nx - 1;
    const R uin[3] = {inl.at(0, y, z, g.ny, g.nz), inl.at(1, y, z, g.ny, g.nz), inl.at(2, y, z, g.ny, g.nz)};
    const uint32_t xb = (uint32_t)(x * sizeof(T));
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int cx = CX[i];
        const int64_t row_src = row_off(g, ys[CY[i] + 1], zs[CZ[i] + 1]);
        const T *nb = in + ((int64_t)i * g.plane + row_src);
        R v;
        if (cx == 0) {
            v = Store<ST>::dec(ld_stream(at_bytes(nb, xb)));
        } else {
            const bool cross = cx > 0 ? lo : hi;
            const int Fc = cx > 0 ? F0 : F1;
            const int rx = pop_index(-CX[i], CY[i], CZ[i]);
            const T *ab = Fc == LBM_FREESLIP ? in + ((int64_t)rx * g.plane + row_src)
                          : Fc == LBM_OUTFLOW ? nb
                                              : in + ((int64_t)opp(i) * g.plane + row_own);
            const uint32_t axb = Fc == LBM_OUTFLOW ? (uint32_t)((g.nx - 1) * sizeof(T)) : xb;
            const uint32_t nxb = (uint32_t)((x - cx) * sizeof(T));
            const T *p = cross ? at_bytes(ab, axb) : at_bytes(nb, nxb);
            v = Store<ST>::dec(ld_stream(p));
            if (cx > 0 && Fc == LBM_INLET && cross)
                v += (R)(6.0 * weight(i)) * ((R)CX[i] * uin[0] + (R)CY[i] * uin[1] + (R)CZ[i] * uin[2]);
        }
        f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = v;
    }
}

// Wave-level choice of the pull (all lanes of a wave share y, z and the
// segment): the face-aware general form only for rows on a y or z face.
template <int ST, typename R>
__device__ __forceinline__ void pull_wave(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int xs, int x,
                                          int y, int z, const Geom &g, const Inlet<R> &inl)
{
    const bool yz = (y == 0 && g.face[2] != LBM_PERIODIC) || (y == g.ny - 1 && g.face[3] != LBM_PERIODIC) ||
                    (z == 0 && g.face[4] != LBM_PERIODIC) || (z == g.nz - 1 && g.face[5] != LBM_PERIODIC);
    const bool xf = (xs == 0 && g.face[0] != LBM_PERIODIC) || (xs == g.ntx - 1 && g.face[1] != LBM_PERIODIC);
    if (yz) pull_general<ST>(f, in, x, y, z, g, inl);
    else if (xf) pull_xface<ST>(f, in, x, y, z, g, inl);
    else pull_interior<ST>(f, in, x, y, z, g);
}
// the same with the 32-bit interior pull on rows away from y and z faces and wraps
template <int ST, typename R>
__device__ __forceinline__ void pull_wave32(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int xs,
                                            int x, int y, int z, const Geom &g, const Inlet<R> &inl, uint32_t span)
{
    const bool yz = (y == 0 && g.face[2] != LBM_PERIODIC) || (y == g.ny - 1 && g.face[3] != LBM_PERIODIC) ||
                    (z == 0 && g.face[4] != LBM_PERIODIC) || (z == g.nz - 1 && g.face[5] != LBM_PERIODIC);
    const bool xf = (xs == 0 && g.face[0] != LBM_PERIODIC) || (xs == g.ntx - 1 && g.face[1] != LBM_PERIODIC);
    const bool wrap = y == 0 || y == g.ny - 1 || z == 0 || z == g.nz - 1;
    if (yz) pull_general<ST>(f, in, x, y, z, g, inl);
    else if (xf) pull_xface<ST>(f, in, x, y, z, g, inl);
    else if (wrap) pull_interior<ST>(f, in, x, y, z, g);
    else pull_interior32<ST>(f, in, x, y, z, g, span);
}


// ---------------------------------------------------------------------------
// collision (Eqs. 4-5) in deviation form
// ---------------------------------------------------------------------------

template <typename R> struct Rates {
    R s_nu, s_b, s3, s4, s5, s6;
};

// Raw moments along one axis of the line (v(-1), v(0), v(+1)) -> (m0, m1, m2).
template <typename R> __host__ __device__ __forceinline__ void raw3(R &a, R &b, R &c)
{
    const R s = c + a, t = c - a;
    a = s + b;
    b = t;
    c = s;
}
// Central shift along one axis: (m0, m1, m2) -> (k0, k1, k2) about u.
template <typename R> __host__ __device__ __forceinline__ void shift3(R &m0, R &m1, R &m2, R u)
{
    const R k1 = m1 - u * m0;
    m2 = m2 - u * (m1 + k1);
    m1 = k1;
}
// Inverse shift: (k0, k1, k2) -> (m0, m1, m2).
template <typename R> __host__ __device__ __forceinline__ void unshift3(R &k0, R &k1, R &k2, R u)
{
    const R m1 = k1 + u * k0;
    k2 = k2 + u * (k1 + m1);
    k1 = m1;
}
// Inverse raw transform: (m0, m1, m2) -> (v(-1), v(0), v(+1)).
template <typename R> __host__ __device__ __forceinline__ void iraw3(R &a, R &b, R &c)
{
    const R h = (R)0.5 * c;
    const R m0 = a, m1 = b, m2 = c;
    a = h - (R)0.5 * m1;
    c = h + (R)0.5 * m1;
    b = m0 - m2;
}

// Apply a 3-point line operation to the 9 lines of f[z][y][x] along x, y or z.
template <typename R, typename Op> __host__ __device__ __forceinline__ void lines_x(R (&f)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(f[a][b][0], f[a][b][1], f[a][b][2]);
}
template <typename R, typename Op> __host__ __device__ __forceinline__ void lines_y(R (&f)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(f[a][0][b], f[a][1][b], f[a][2][b]);
}
template <typename R, typename Op> __host__ __device__ __forceinline__ void lines_z(R (&f)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(f[0][a][b], f[1][a][b], f[2][a][b]);
}

// Macroscopic values of a pulled node: rho = 1 + sum d, j = sum c d (Eq. 2).
template <typename R> struct Macro {
    R drho, jx, jy, jz;
};

// Relaxation of the central moments of d (index [c][b][a] = exponents
// (a,b,c)) at density 1 + drho, half-force velocity u and force F:
// kappa'(d) = kappa(d) - S (kappa(d) + Delta) + (I - S/2) kappa_F, where
// Delta = kappa(w; u) - kappa_eq(rho) is written out so that no large terms
// cancel (kappa - kappa_eq = kappa(d) + Delta).
template <typename R>
__host__ __device__ __forceinline__ void relax(R (&f)[3][3][3], R ux, R uy, R uz, R drho, R Fx, R Fy, R Fz, const Rates<R> &rt)
{
    const R third = (R)(1.0 / 3.0), ninth = (R)(1.0 / 9.0), t27 = (R)(1.0 / 27.0);
    const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    const R px = third + x2, py = third + y2, pz = third + z2;
    const R dr3 = drho * third, dr9 = drho * ninth;
    // order 1: conserved (rate 0), forcing adds F
    f[0][0][1] += Fx;
    f[0][1][0] += Fy;
    f[1][0][0] += Fz;
    // order 2, off-diagonal: shear rate
    f[0][1][1] -= rt.s_nu * (f[0][1][1] + ux * uy);
    f[1][0][1] -= rt.s_nu * (f[1][0][1] + ux * uz);
    f[1][1][0] -= rt.s_nu * (f[1][1][0] + uy * uz);
    // order 2, diagonal: deviator at s_nu, trace at s_b
    {
        const R nxx = f[0][0][2] + x2 - dr3, nyy = f[0][2][0] + y2 - dr3, nzz = f[2][0][0] + z2 - dr3;
        const R tr = (rt.s_b - rt.s_nu) * third * (nxx + nyy + nzz);
        f[0][0][2] -= rt.s_nu * nxx + tr;
        f[0][2][0] -= rt.s_nu * nyy + tr;
        f[2][0][0] -= rt.s_nu * nzz + tr;
    }
    // order 3 (forcing term F cs^2 on the (1,2,0) family)
    {
        const R s = rt.s3, h = (R)1 - (R)0.5 * s;
        f[0][2][1] += -s * (f[0][2][1] - ux * py) + h * third * Fx;  // (1,2,0)
        f[2][0][1] += -s * (f[2][0][1] - ux * pz) + h * third * Fx;  // (1,0,2)
        f[0][1][2] += -s * (f[0][1][2] - uy * px) + h * third * Fy;  // (2,1,0)
        f[2][1][0] += -s * (f[2][1][0] - uy * pz) + h * third * Fy;  // (0,1,2)
        f[1][0][2] += -s * (f[1][0][2] - uz * px) + h * third * Fz;  // (2,0,1)
        f[1][2][0] += -s * (f[1][2][0] - uz * py) + h * third * Fz;  // (0,2,1)
        f[1][1][1] -= s * (f[1][1][1] - ux * uy * uz);               // (1,1,1)
    }
    // order 4
    {
        const R s = rt.s4;
        f[0][2][2] -= s * (f[0][2][2] + (x2 + y2) * third + x2 * y2 - dr9);  // (2,2,0)
        f[2][0][2] -= s * (f[2][0][2] + (x2 + z2) * third + x2 * z2 - dr9);  // (2,0,2)
        f[2][2][0] -= s * (f[2][2][0] + (y2 + z2) * third + y2 * z2 - dr9);  // (0,2,2)
        f[1][1][2] -= s * (f[1][1][2] + px * uy * uz);                       // (2,1,1)
        f[1][2][1] -= s * (f[1][2][1] + py * ux * uz);                       // (1,2,1)
        f[2][1][1] -= s * (f[2][1][1] + pz * ux * uy);                       // (1,1,2)
    }
    // order 5 (forcing term F cs^4 on the (1,2,2) family)
    {
        const R s = rt.s5, h = (R)1 - (R)0.5 * s;
        f[2][2][1] += -s * (f[2][2][1] - ux * py * pz) + h * ninth * Fx;  // (1,2,2)
        f[2][1][2] += -s * (f[2][1][2] - uy * px * pz) + h * ninth * Fy;  // (2,1,2)
        f[1][2][2] += -s * (f[1][2][2] - uz * px * py) + h * ninth * Fz;  // (2,2,1)
    }
    // order 6
    {
        const R d6 = (x2 * y2 + x2 * z2 + y2 * z2) * third + (x2 + y2 + z2) * ninth + x2 * y2 * z2 - drho * t27;
        f[2][2][2] -= rt.s6 * (f[2][2][2] + d6);
    }
}

template <typename R> __host__ __device__ __forceinline__ void raw_all(R (&f)[3][3][3])
{
    auto raw = [](R &a, R &b, R &c) { raw3(a, b, c); };
    lines_x(f, raw);
    lines_y(f, raw);
    lines_z(f, raw);
}

// Half-force velocity and density from raw moments of d.
template <typename R>
__host__ __device__ __forceinline__ void velocity(const R (&m)[3][3][3], R Fx, R Fy, R Fz, R &drho, R &ux, R &uy, R &uz)
{
    drho = m[0][0][0];
    const R inv = (R)1 / ((R)1 + drho);
    ux = (m[0][0][1] + (R)0.5 * Fx) * inv;
    uy = (m[0][1][0] + (R)0.5 * Fy) * inv;
    uz = (m[1][0][0] + (R)0.5 * Fz) * inv;
}

// Inverse path shared by the central-moment forms: central moments of d about
// u -> raw moments -> populations (deviations).
template <typename R> __host__ __device__ __forceinline__ void central_to_populations(R (&f)[3][3][3], R ux, R uy, R uz)
{
    lines_z(f, [uz](R &a, R &b, R &c) { unshift3(a, b, c, uz); });
    lines_y(f, [uy](R &a, R &b, R &c) { unshift3(a, b, c, uy); });
    lines_x(f, [ux](R &a, R &b, R &c) { unshift3(a, b, c, ux); });
    auto iraw = [](R &a, R &b, R &c) { iraw3(a, b, c); };
    lines_z(f, iraw);
    lines_y(f, iraw);
    lines_x(f, iraw);
}

// f holds the pulled deviations; on return f holds the post-collision
// deviations and (rho, u) the density and half-force velocity used.
template <typename R>
__host__ __device__ __forceinline__ void collide(R (&f)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt, R &rho_o, R &ux_o,
                                        R &uy_o, R &uz_o)
{
    raw_all(f);  // raw moments of d (index [mz][my][mx])
    R drho, ux, uy, uz;
    velocity(f, Fx, Fy, Fz, drho, ux, uy, uz);
    rho_o = (R)1 + drho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
    // central moments of d about u
    lines_x(f, [ux](R &a, R &b, R &c) { shift3(a, b, c, ux); });
    lines_y(f, [uy](R &a, R &b, R &c) { shift3(a, b, c, uy); });
    lines_z(f, [uz](R &a, R &b, R &c) { shift3(a, b, c, uz); });
    relax(f, ux, uy, uz, drho, Fx, Fy, Fz, rt);
    // back to raw moments, then to populations
    central_to_populations(f, ux, uy, uz);
}

// Raw moments of d up to second order (exponents (a,b,c) with a+b+c <= 2),
// taken separably: x-pass on all 9 lines, then only the y and z sums that
// feed a moment of order <= 2 (66 additions instead of the 81 of the full
// transform).  m[c][b][a] = sum d c_x^a c_y^b c_z^c.
template <typename R> struct Low {
    R m000, m100, m010, m001, m200, m020, m002, m110, m101, m011;
};
// Raw moments of orders 0-2 from the x-line moments X0, X1, X2 (the y and z
// stages of low_moments).
template <typename R>
__host__ __device__ __forceinline__ Low<R> low_moments_yz(const R (&X0)[3][3], const R (&X1)[3][3], const R (&X2)[3][3])
{
    R Y00[3], Y01[3], Y02[3], Y10[3], Y11[3], Y20[3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
        const R s0 = X0[z][2] + X0[z][0];
        Y00[z] = s0 + X0[z][1];
        Y01[z] = X0[z][2] - X0[z][0];
        Y02[z] = s0;
        Y10[z] = (X1[z][2] + X1[z][0]) + X1[z][1];
        Y11[z] = X1[z][2] - X1[z][0];
        Y20[z] = (X2[z][2] + X2[z][0]) + X2[z][1];
    }
    Low<R> L;
    const R s00 = Y00[2] + Y00[0];
    L.m000 = s00 + Y00[1];
    L.m001 = Y00[2] - Y00[0];
    L.m002 = s00;
    L.m010 = (Y01[2] + Y01[0]) + Y01[1];
    L.m011 = Y01[2] - Y01[0];
    L.m020 = (Y02[2] + Y02[0]) + Y02[1];
    L.m100 = (Y10[2] + Y10[0]) + Y10[1];
    L.m101 = Y10[2] - Y10[0];
    L.m110 = (Y11[2] + Y11[0]) + Y11[1];
    L.m200 = (Y20[2] + Y20[0]) + Y20[1];
    return L;
}
template <typename R> __host__ __device__ __forceinline__ Low<R> low_moments(const R (&f)[3][3][3])
{
    R X0[3][3], X1[3][3], X2[3][3];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const R s = f[z][y][2] + f[z][y][0];
            X1[z][y] = f[z][y][2] - f[z][y][0];
            X0[z][y] = s + f[z][y][1];
            X2[z][y] = s;
        }
    return low_moments_yz(X0, X1, X2);
}
// The same from FP16 deviations: the x stage widens and adds in one mixed
// precision instruction (v_fma_mix_f32: a*one + b with either operand in
// FP16), so no separate conversions.  `one` is 1 at run time (a known
// constant would be folded back into plain adds of converted values).  The
// widening is exact, so every sum equals convert-then-add bit for bit.
__device__ __forceinline__ Low<float> low_moments_f16(const _Float16 (&h)[3][3][3], float one)
{
    float X0[3][3], X1[3][3], X2[3][3];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const float s = __builtin_fmaf((float)h[z][y][2], one, (float)h[z][y][0]);
            X1[z][y] = __builtin_fmaf((float)h[z][y][0], -one, (float)h[z][y][2]);
            X0[z][y] = __builtin_fmaf((float)h[z][y][1], one, s);
            X2[z][y] = s;
        }
    return low_moments_yz(X0, X1, X2);
}

// collide() for unit rates of orders 3 to 6 (the default): those central
// moments relax fully, kappa' = kappa_eq + kappa_F / 2, so they depend on
// rho, u and F only and the forward transform is needed up to order 2.  Same
// post-collision state as collide() up to rounding.
// The post-collision central moments kappa' of collide_unit_high (into k),
// from the raw moments of orders 0-2; also rho and the half-force velocity.
template <typename R>
__host__ __device__ __forceinline__ void unit_high_kappa(const Low<R> &L, R (&f)[3][3][3], R Fx, R Fy, R Fz,
                                                         const Rates<R> &rt, R &rho_o, R &ux_o, R &uy_o, R &uz_o)
{
    const R drho = L.m000;
    const R inv = (R)1 / ((R)1 + drho);
    const R ux = (L.m100 + (R)0.5 * Fx) * inv, uy = (L.m010 + (R)0.5 * Fy) * inv, uz = (L.m001 + (R)0.5 * Fz) * inv;
    rho_o = (R)1 + drho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
    // central moments of d about u, orders 1 and 2
    const R k100 = L.m100 - ux * drho, k010 = L.m010 - uy * drho, k001 = L.m001 - uz * drho;
    const R k200 = L.m200 - ux * (L.m100 + k100);
    const R k020 = L.m020 - uy * (L.m010 + k010);
    const R k002 = L.m002 - uz * (L.m001 + k001);
    const R k110 = L.m110 - ux * L.m010 - uy * k100;
    const R k101 = L.m101 - ux * L.m001 - uz * k100;
    const R k011 = L.m011 - uy * L.m001 - uz * k010;
    const R third = (R)(1.0 / 3.0), ninth = (R)(1.0 / 9.0), t27 = (R)(1.0 / 27.0);
    const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    const R px = third + x2, py = third + y2, pz = third + z2;
    const R dr3 = drho * third, dr9 = drho * ninth;
    // orders 0 and 1 (force added to the momentum)
    f[0][0][0] = drho;
    f[0][0][1] = k100 + Fx;
    f[0][1][0] = k010 + Fy;
    f[1][0][0] = k001 + Fz;
    // order 2 as in relax(): shear rate on the off-diagonal and deviatoric
    // parts, bulk rate on the trace
    f[0][1][1] = k110 - rt.s_nu * (k110 + ux * uy);
    f[1][0][1] = k101 - rt.s_nu * (k101 + ux * uz);
    f[1][1][0] = k011 - rt.s_nu * (k011 + uy * uz);
    {
        const R nxx = k200 + x2 - dr3, nyy = k020 + y2 - dr3, nzz = k002 + z2 - dr3;
        const R tr = (rt.s_b - rt.s_nu) * third * (nxx + nyy + nzz);
        f[0][0][2] = k200 - (rt.s_nu * nxx + tr);
        f[0][2][0] = k020 - (rt.s_nu * nyy + tr);
        f[2][0][0] = k002 - (rt.s_nu * nzz + tr);
    }
    // orders 3 to 6 at rate 1: -Delta (the equilibrium in deviation form) plus
    // half the force moments (F cs^2 on the (1,2,0) family, F cs^4 on (1,2,2))
    const R f3 = (R)(1.0 / 6.0), f5 = (R)(1.0 / 18.0);
    f[0][2][1] = ux * py + f3 * Fx;  // (1,2,0)
    f[2][0][1] = ux * pz + f3 * Fx;  // (1,0,2)
    f[0][1][2] = uy * px + f3 * Fy;  // (2,1,0)
    f[2][1][0] = uy * pz + f3 * Fy;  // (0,1,2)
    f[1][0][2] = uz * px + f3 * Fz;  // (2,0,1)
    f[1][2][0] = uz * py + f3 * Fz;  // (0,2,1)
    f[1][1][1] = ux * uy * uz;       // (1,1,1)
    f[0][2][2] = dr9 - ((x2 + y2) * third + x2 * y2);  // (2,2,0)
    f[2][0][2] = dr9 - ((x2 + z2) * third + x2 * z2);  // (2,0,2)
    f[2][2][0] = dr9 - ((y2 + z2) * third + y2 * z2);  // (0,2,2)
    f[1][1][2] = -(px * uy * uz);                      // (2,1,1)
    f[1][2][1] = -(py * ux * uz);                      // (1,2,1)
    f[2][1][1] = -(pz * ux * uy);                      // (1,1,2)
    f[2][2][1] = ux * py * pz + f5 * Fx;               // (1,2,2)
    f[2][1][2] = uy * px * pz + f5 * Fy;               // (2,1,2)
    f[1][2][2] = uz * px * py + f5 * Fz;               // (2,2,1)
    f[2][2][2] = drho * t27 - ((x2 * y2 + x2 * z2 + y2 * z2) * third + (x2 + y2 + z2) * ninth + x2 * y2 * z2);
}
template <typename R>
__host__ __device__ __forceinline__ void unit_high_from_low(const Low<R> &L, R (&f)[3][3][3], R Fx, R Fy, R Fz,
                                                            const Rates<R> &rt, R &rho_o, R &ux_o, R &uy_o, R &uz_o)
{
    unit_high_kappa(L, f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
    central_to_populations(f, ux_o, uy_o, uz_o);
}
template <typename R>
__host__ __device__ __forceinline__ void collide_unit_high(R (&f)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt,
                                                           R &rho_o, R &ux_o, R &uy_o, R &uz_o)
{
    unit_high_from_low(low_moments(f), f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
}

// ---------------------------------------------------------------------------
// comparison collision models (Sec. 5.1 and its collision-cost figure): the
// paper prints neither; both take the product-form equilibrium, half-force
// velocity and Guo forcing of the central-moment model (reading), so they
// differ from it only in where relaxation happens
// ---------------------------------------------------------------------------

// rho - 1 and j of pulled deviations from the x-line sums (53 additions).
template <typename R> __host__ __device__ __forceinline__ void mass_momentum(const R (&f)[3][3][3], R &drho, R &jx, R &jy, R &jz)
{
    R X0[3][3], X1[3][3];
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            X1[z][y] = f[z][y][2] - f[z][y][0];
            X0[z][y] = (f[z][y][2] + f[z][y][0]) + f[z][y][1];
        }
    R Z0[3], Y1[3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
        Z0[z] = (X0[z][2] + X0[z][0]) + X0[z][1];
        Y1[z] = X0[z][2] - X0[z][0];
    }
    drho = (Z0[2] + Z0[0]) + Z0[1];
    jz = Z0[2] - Z0[0];
    jy = (Y1[2] + Y1[0]) + Y1[1];
    jx = ((X1[0][0] + X1[0][1]) + (X1[0][2] + X1[1][0])) + ((X1[1][1] + X1[1][2]) + (X1[2][0] + (X1[2][1] + X1[2][2])));
}

// Lattice BGK at rate omega = s_nu: f' = f - omega (f - f_eq(rho, u)) +
// (1 - omega/2) G with the product-form f_eq = rho Phi(u), Phi =
// phi(u_x) phi(u_y) phi(u_z), and G = F . dPhi/du.  In deviations
// (d = f - w, w = Phi(0)):
//   d' = (1 - omega) d + omega [(Phi - Phi0) + drho Phi] + h G,  h = 1 - omega/2,
// evaluated as a sum of three tensor products grouped by the x factor,
//   omega[...] + h G = A_x (omega drho B + h E) + (omega Q_x + h F_x D_x) B + omega P_x C,
// with per-axis vectors P = phi(0), Q = phi(u) - phi(0), A = phi(u),
// D = dphi/du and per-(y,z) products B = A_y A_z, C = Q_y A_z + P_y Q_z,
// E = F_y D_y A_z + A_y F_z D_z.  No O(1) terms cancel.
template <typename R>
__host__ __device__ __forceinline__ void collide_bgk(R (&f)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt, R &rho_o,
                                                     R &ux_o, R &uy_o, R &uz_o)
{
    R drho, jx, jy, jz;
    mass_momentum(f, drho, jx, jy, jz);
    const R inv = (R)1 / ((R)1 + drho);
    const R u[3] = {(jx + (R)0.5 * Fx) * inv, (jy + (R)0.5 * Fy) * inv, (jz + (R)0.5 * Fz) * inv};
    rho_o = (R)1 + drho;
    ux_o = u[0];
    uy_o = u[1];
    uz_o = u[2];
    const R om = rt.s_nu, h = (R)1 - (R)0.5 * rt.s_nu;
    const R P[3] = {(R)(1.0 / 6.0), (R)(2.0 / 3.0), (R)(1.0 / 6.0)};  // index c + 1
    R Q[3][3], A[3][3], D[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R v = u[a], v2 = v * v;
        Q[a][0] = (R)0.5 * (v2 - v);
        Q[a][1] = -v2;
        Q[a][2] = (R)0.5 * (v2 + v);
        D[a][0] = v - (R)0.5;
        D[a][1] = (R)-2 * v;
        D[a][2] = v + (R)0.5;
#pragma unroll
        for (int c = 0; c < 3; ++c) A[a][c] = P[c] + Q[a][c];
    }
    const R omd = om * drho, hFx = h * Fx;
    R V2[3], V3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        V2[c] = om * Q[0][c] + hFx * D[0][c];
        V3[c] = om * P[c];
    }
    const R keep = (R)1 - om;
#pragma unroll
    for (int z = 0; z < 3; ++z) {
        const R FzDz = Fz * D[2][z];
#pragma unroll
        for (int y = 0; y < 3; ++y) {
            const R B = A[1][y] * A[2][z];
            const R C = Q[1][y] * A[2][z] + P[y] * Q[2][z];
            const R E = (Fy * D[1][y]) * A[2][z] + A[1][y] * FzDz;
            const R M1 = omd * B + h * E;
#pragma unroll
            for (int x = 0; x < 3; ++x) f[z][y][x] = keep * f[z][y][x] + (A[0][x] * M1 + (V2[x] * B + V3[x] * C));
        }
    }
}

// Raw-moment MRT: the combination basis of the central-moment model taken
// about zero velocity.  Raw moments of d; equilibrium raw moments of the
// product form, rho prod_a r_e(u_a) with r_0 = 1, r_1 = u, r_2 = 1/3 + u^2,
// in deviations drho prod r(u) + (prod r(u) - prod r(0)) expanded per axis;
// force moments sum_a F_a d/du_a prod r(u); relaxation per group as in
// relax() (deviator / trace split of the second-order diagonal), then the
// inverse raw transform.
template <typename R>
__host__ __device__ __forceinline__ void collide_rm(R (&f)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt, R &rho_o,
                                                    R &ux_o, R &uy_o, R &uz_o)
{
    raw_all(f);  // raw moments of d, index [c][b][a]
    R drho, ux, uy, uz;
    velocity(f, Fx, Fy, Fz, drho, ux, uy, uz);
    rho_o = (R)1 + drho;
    ux_o = ux;
    uy_o = uy;
    uz_o = uz;
    const R u[3] = {ux, uy, uz};
    const R F[3] = {Fx, Fy, Fz};
    const R third = (R)(1.0 / 3.0);
    R r[3][3], q[3][3], dr[3][3];  // [axis][exponent]: r(u), r(u) - r(0), dr/du
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const R v = u[a], v2 = v * v;
        r[a][0] = (R)1;
        r[a][1] = v;
        r[a][2] = third + v2;
        q[a][0] = (R)0;
        q[a][1] = v;
        q[a][2] = v2;
        dr[a][0] = (R)0;
        dr[a][1] = (R)1;
        dr[a][2] = (R)2 * v;
    }
    const R r0[3] = {(R)1, (R)0, third};
    R neq[3][3][3], mF[3][3][3];  // m - m_eq and the force moments
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R ryz = r[1][b] * r[2][c];
                const R Rabc = r[0][a] * ryz;
                const R dev = q[0][a] * ryz + r0[a] * (q[1][b] * r[2][c] + r0[b] * q[2][c]);
                neq[c][b][a] = f[c][b][a] - (drho * Rabc + dev);
                mF[c][b][a] = F[0] * dr[0][a] * ryz + r[0][a] * (F[1] * dr[1][b] * r[2][c] + r[1][b] * F[2] * dr[2][c]);
            }
    // relaxation: m' = m - S (m - m_eq) + (I - S/2) m_F; orders 0 and 1 keep
    // their moments and gain the force
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int n = a + b + c;
                const bool diag2 = n == 2 && (a == 2 || b == 2 || c == 2);
                if (n < 2) {
                    f[c][b][a] += mF[c][b][a];
                } else if (!diag2) {
                    const R s = n == 2 ? rt.s_nu : n == 3 ? rt.s3 : n == 4 ? rt.s4 : n == 5 ? rt.s5 : rt.s6;
                    f[c][b][a] += -s * neq[c][b][a] + ((R)1 - (R)0.5 * s) * mF[c][b][a];
                }
            }
    {
        const R tn = (rt.s_b - rt.s_nu) * third * (neq[0][0][2] + neq[0][2][0] + neq[2][0][0]);
        const R tf = (rt.s_b - rt.s_nu) * third * (mF[0][0][2] + mF[0][2][0] + mF[2][0][0]);
        f[0][0][2] += -(rt.s_nu * neq[0][0][2] + tn) + mF[0][0][2] - (R)0.5 * (rt.s_nu * mF[0][0][2] + tf);
        f[0][2][0] += -(rt.s_nu * neq[0][2][0] + tn) + mF[0][2][0] - (R)0.5 * (rt.s_nu * mF[0][2][0] + tf);
        f[2][0][0] += -(rt.s_nu * neq[2][0][0] + tn) + mF[2][0][0] - (R)0.5 * (rt.s_nu * mF[2][0][0] + tf);
    }
    auto iraw = [](R &a, R &b, R &c) { iraw3(a, b, c); };
    lines_z(f, iraw);
    lines_y(f, iraw);
    lines_x(f, iraw);
}

// Collision by model: 0 central moments (any rates), 1 central moments with
// unit rates of orders 3 to 6, 2 BGK, 3 raw-moment MRT.
enum : int { COLL_CM = 0, COLL_CM_UNIT_HIGH = 1, COLL_BGK = 2, COLL_RM = 3 };
template <int COLL, typename R>
__host__ __device__ __forceinline__ void collide_as(R (&f)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt, R &rho_o,
                                                    R &ux_o, R &uy_o, R &uz_o)
{
    if constexpr (COLL == COLL_CM_UNIT_HIGH) collide_unit_high(f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
    else if constexpr (COLL == COLL_BGK) collide_bgk(f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
    else if constexpr (COLL == COLL_RM) collide_rm(f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
    else collide(f, Fx, Fy, Fz, rt, rho_o, ux_o, uy_o, uz_o);
}

// rho - 1 and j of pulled deviations (no transform of the rest).
template <typename R> __device__ __forceinline__ Macro<R> moments01(const R (&f)[3][3][3])
{
    Macro<R> m{0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R v = f[CZ[i] + 1][CY[i] + 1][CX[i] + 1];
        m.drho += v;
        if (CX[i]) m.jx += CX[i] > 0 ? v : -v;
        if (CY[i]) m.jy += CY[i] > 0 ? v : -v;
        if (CZ[i]) m.jz += CZ[i] > 0 ? v : -v;
    }
    return m;
}

// Eq. (2) moments (drho = rho - 1, j) of the streamed deviations at one node,
// for kernels whose lanes hold unrelated nodes (band nodes, dense macros):
// the plain periodic pull when no source crosses a non-periodic face, the
// face-aware one otherwise.  Both are unrolled so that the 27 loads are in
// flight together (a compact loop over the face rules waits for each load in
// turn and measured slower).
// Pull of a node that touches exactly one non-periodic face, a no-slip wall
// on axis `ax` at side `hi` (0 = low, 1 = high), and no other: the sources
// that cross the wall bounce back to the node's own opposite population,
// every other source is the plain pull (with periodic wrap on the remaining
// axes).  The same values as pull_general, without its per-population face
// search (the common case of band nodes at a wall).
template <int ST, typename R>
__device__ __forceinline__ void pull_wall(R (&f)[3][3][3], const typename Store<ST>::T *__restrict__ in, int x, int y,
                                          int z, const Geom &g, int ax, int hi)
{
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const int xs[3] = {xp, x, xm};  // source for c = -1, 0, +1
    const int ys[3] = {yp, y, ym};
    const int zs[3] = {zp, z, zm};
    const int inward = hi ? -1 : 1;  // c along ax whose source lies beyond the wall
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int ca = ax == 0 ? CX[i] : ax == 1 ? CY[i] : CZ[i];
        const bool back = ca == inward;
        const int sx = back ? x : xs[CX[i] + 1], sy = back ? y : ys[CY[i] + 1], sz = back ? z : zs[CZ[i] + 1];
        const int pl = back ? opp(i) : i;
        const int64_t idx = (int64_t)pl * g.plane + row_off(g, sy, sz) + sx;
        f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = Store<ST>::dec(ld_stream(in + idx));
    }
}

template <int ST, typename R>
__device__ __forceinline__ Macro<R> node_moments(const typename Store<ST>::T *__restrict__ in, int x, int y, int z,
                                                 const Geom &g, const Inlet<R> &inl)
{
    const bool t0 = x == 0 && g.face[0] != LBM_PERIODIC, t1 = x == g.nx - 1 && g.face[1] != LBM_PERIODIC;
    const bool t2 = y == 0 && g.face[2] != LBM_PERIODIC, t3 = y == g.ny - 1 && g.face[3] != LBM_PERIODIC;
    const bool t4 = z == 0 && g.face[4] != LBM_PERIODIC, t5 = z == g.nz - 1 && g.face[5] != LBM_PERIODIC;
    const int touched = (int)t0 + (int)t1 + (int)t2 + (int)t3 + (int)t4 + (int)t5;
    const int k = t0 ? 0 : t1 ? 1 : t2 ? 2 : t3 ? 3 : t4 ? 4 : 5;  // the touched face when touched == 1
    R f[3][3][3];
    if (touched == 0) pull_interior<ST>(f, in, x, y, z, g);
    else if (touched == 1 && g.face[k] == LBM_NOSLIP) pull_wall<ST>(f, in, x, y, z, g, k >> 1, k & 1);
    else pull_general<ST>(f, in, x, y, z, g, inl);
    return moments01(f);
}

// ---------------------------------------------------------------------------
// rigid placement of a solid sample (the sample update of Alg. 2 (c))
// ---------------------------------------------------------------------------
// Coordinate a of x = o + R X (R row-major) in FP64 with one rounding per
// operation, in the order o_a + ((R_a0 X + R_a1 Y) + R_a2 Z), then rounded to
// FP32, so that the base cells do not depend on the compiler's choice of fused
// operations (the same function on the host and the device).
__host__ __device__ inline float place_coord(const double R[9], const double o[3], int a, double X, double Y, double Z)
{
#pragma clang fp contract(off)
    const double p = o[a] + ((R[3 * a] * X + R[3 * a + 1] * Y) + R[3 * a + 2] * Z);
    return (float)p;
}

// Whether every sample of a body whose body-frame coordinates lie in the box
// [lo, hi] is placed by place_coord inside [0, top_a) on every axis: interval
// bounds of o_a + sum_b R_ab X_b over the box, widened by (|o_a| +
// sum_b max|R_ab X_b| + 1) 2^-20, which is far above the rounding of the
// FP64 placement (a few units of 2^-53 of that magnitude) and of its FP32
// result (2^-24).  False when that cannot be shown.
inline bool pose_inside_box(const double R[9], const double o[3], const double lo[3], const double hi[3],
                            const double top[3])
{
    for (int a = 0; a < 3; ++a) {
        double l = o[a], h = o[a], mag = o[a] < 0 ? -o[a] : o[a];
        for (int b = 0; b < 3; ++b) {
            const double p = R[3 * a + b] * lo[b], q = R[3 * a + b] * hi[b];
            l += p < q ? p : q;
            h += p < q ? q : p;
            const double ap = p < 0 ? -p : p, aq = q < 0 ? -q : q;
            mag += ap > aq ? ap : aq;
        }
        const double margin = (mag + 1.0) * 0x1p-20;
        if (!(l - margin >= 0.0) || !(h + margin < top[a])) return false;
    }
    return true;
}

}  // namespace lbm
