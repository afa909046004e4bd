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
// solid samples (Sec. 4.2.2): keys, sort, band tiles, slots, runs
//
// The sort orders the samples by (l^3 block in x-y-z order, Morton order of
// the quantised position inside the block, input index).  It runs as a
// bucket sort with one bucket per block: a histogram of the blocks (integer
// atomics), an exclusive scan of it, a scatter of the samples into their
// bucket's range (in any order), then every bucket ordered on its own by the
// unique key (Morton code, index).  Buckets of at most RANK_MAX samples take
// counting ranks, one lane per sample; larger ones a bitonic network run by
// one workgroup.  The result does not depend on the scatter's order.
// ---------------------------------------------------------------------------
constexpr int ELL = 4;
constexpr int RANK_MAX = 2048;
constexpr int BIG_SORT_BLOCKS = 16;

struct MarkerGeom {
    int nx, ny, nz, nbx, nby, ntx;
    int periodic[3];
};

__device__ __forceinline__ float domain_top(const MarkerGeom &mg, int a)
{
    const int n = a == 0 ? mg.nx : a == 1 ? mg.ny : mg.nz;
    return mg.periodic[a] ? (float)n : (float)(n - 1);
}

// Integer atomic add of `delta` per lane to p[key], one atomic per distinct
// key of the wavefront's active lanes (their leader adds the group's total):
// samples in input order tend to share blocks, and same-address atomics
// serialise.  Returns the value before the group's add, minus `delta` times
// the number of lower lanes in the group, i.e. a slot of the lane's own.
__device__ __forceinline__ int32_t wave_grouped_add(int32_t *p, int32_t key, int32_t delta)
{
    const int lane = (int)(threadIdx.x & 63);
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t todo = __ballot(1);
    int32_t mine = 0;
    while (todo) {
        const int leader = __ffsll((long long)todo) - 1;
        const int32_t kl = __shfl(key, leader, 64);
        const uint64_t same = __ballot(key == kl);
        int32_t old = 0;
        if (lane == leader) old = atomicAdd(p + kl, delta * (int32_t)__popcll(same));
        old = __shfl(old, leader, 64);
        if (key == kl) mine = old + delta * (int32_t)__popcll(same & below);
        todo &= ~same;
    }
    return mine;
}

struct Pose {
    double R[9], o[3], v[3], w[3];  // R row-major
};

// Rigid placement of sample s (the sample update of Alg. 2 (c)): x = o + R X
// by place_coord (FP64, one rounding per operation, then FP32); u_b = R ub + v
// + w x (x - o) with the FP32 x.  A coordinate outside the domain is clamped
// into it (so that the set-up after the placement stays in range whether or
// not the host waits for the count of such samples); returns whether one was.
__device__ __forceinline__ bool place_sample(const MarkerGeom &mg, int64_t n, int64_t s, const Pose &P,
                                             const float *__restrict__ bx, const float *__restrict__ bu,
                                             float *__restrict__ wx, float *__restrict__ wu, float (&x)[3])
{
#pragma clang fp contract(off)
    const double X[3] = {(double)bx[s], (double)bx[n + s], (double)bx[2 * n + s]};
    const double U[3] = {(double)bu[s], (double)bu[n + s], (double)bu[2 * n + s]};
    double r[3], ru[3];
    bool out = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float pf = place_coord(P.R, P.o, a, X[0], X[1], X[2]);
        const float top = domain_top(mg, a);
        if (!(pf >= 0.0f) || !(pf < top)) {
            out = true;
            pf = top > 0.0f ? fminf(fmaxf(pf, 0.0f), __int_as_float(__float_as_int(top) - 1)) : 0.0f;
        }
        x[a] = pf;
        wx[a * n + s] = pf;
        r[a] = (double)pf - P.o[a];
        ru[a] = (P.R[3 * a] * U[0] + P.R[3 * a + 1] * U[1]) + P.R[3 * a + 2] * U[2];
    }
    wu[s] = (float)(ru[0] + P.v[0] + (P.w[1] * r[2] - P.w[2] * r[1]));
    wu[n + s] = (float)(ru[1] + P.v[1] + (P.w[2] * r[0] - P.w[0] * r[2]));
    wu[2 * n + s] = (float)(ru[2] + P.v[2] + (P.w[0] * r[1] - P.w[1] * r[0]));
    return out;
}

// Checks, base cell and sort key of each sample (input order), and the
// histogram of the blocks.  POSED: the sample is first placed at the pose
// (body coordinates bx, bu in, placed wx, wu out) and counted in `bad` if it
// had to be clamped; otherwise xyz holds the positions and a sample outside
// the domain is counted.  Also clears the base-cell bit map and the count
// of large buckets, which later launches fill.
template <bool POSED>
__global__ void k_mk_keys(MarkerGeom mg, int64_t n, const float *__restrict__ xyz, unsigned long long *__restrict__ keys,
                          int32_t *__restrict__ cell, int32_t *__restrict__ bcount, int *__restrict__ bad,
                          unsigned long long *__restrict__ occ, int64_t W, int32_t *__restrict__ nbig, const Pose P,
                          const float *__restrict__ bx, const float *__restrict__ bu, float *__restrict__ wx,
                          float *__restrict__ wu)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t w = s; w < W; w += (int64_t)gridDim.x * blockDim.x) occ[w] = 0ull;
    if (s == 0) *nbig = 0;
    if (s >= n) return;
    float pos[3];
    if constexpr (POSED) {
        if (place_sample(mg, n, s, P, bx, bu, wx, wu, pos)) atomicAdd(bad, 1);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) pos[a] = xyz[a * n + s];
    }
    int b[3], B[3];
    unsigned q[3];
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float p = pos[a];
        if (!(p >= 0.0f) || !(p < domain_top(mg, a))) ok = false;
        b[a] = ok ? (int)floorf(p) : 0;
        B[a] = b[a] / ELL;
        // (x - l B) * (1024 / l): exact in FP32
        float r = floorf((p - (float)(ELL * B[a])) * (float)(1024 / ELL));
        r = fminf(fmaxf(r, 0.0f), 1023.0f);
        q[a] = ok ? (unsigned)r : 0u;
    }
    unsigned long long morton = 0;
#pragma unroll
    for (int bit = 0; bit < 10; ++bit)
#pragma unroll
        for (int a = 0; a < 3; ++a) morton |= (unsigned long long)((q[a] >> bit) & 1u) << (3 * bit + a);
    const unsigned long long block =
        (unsigned long long)B[0] + (unsigned long long)mg.nbx * ((unsigned long long)B[1] + (unsigned long long)mg.nby * B[2]);
    // a sample outside the domain stops the set-up before the scatter; the
    // caller then clears the histogram again
    if (ok) wave_grouped_add(bcount, (int32_t)block, 1);
    else atomicAdd(bad, 1);
    keys[s] = (block << 30) | morton;
    cell[s] = (int32_t)((int64_t)b[0] + (int64_t)mg.nx * ((int64_t)b[1] + (int64_t)mg.ny * b[2]));
}

// Each sample into its block's range, at the position its atomic decrement of
// the block's count returns (so the counts are zero again afterwards); the
// bucket-local key is (Morton code, input index).
__global__ void k_scatter(int64_t n, const unsigned long long *__restrict__ keys, const int32_t *__restrict__ bstart,
                          int32_t *__restrict__ bcount, uint32_t *__restrict__ tb, unsigned long long *__restrict__ tkk)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const unsigned long long key = keys[s];
    const uint32_t b = (uint32_t)(key >> 30);
    const int32_t p = bstart[b] + wave_grouped_add(bcount, (int32_t)b, -1) - 1;
    tb[p] = b;
    tkk[p] = ((key & ((1ull << 30) - 1ull)) << 31) | (unsigned long long)s;
}

// Counting ranks inside a bucket: the sample of rank r (number of smaller
// keys; the keys are unique) goes to the bucket's position r.  Buckets above
// RANK_MAX are listed for k_bucket_big.
__global__ void k_bucket_rank(int64_t n, const int32_t *__restrict__ bstart, const uint32_t *__restrict__ tb,
                              const unsigned long long *__restrict__ tkk, int32_t *__restrict__ perm,
                              int32_t *__restrict__ big, int32_t *__restrict__ nbig)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint32_t b = tb[k];
    const int32_t lo = bstart[b], hi = bstart[b + 1];
    if (hi - lo > RANK_MAX) {
        if (k == lo) big[atomicAdd(nbig, 1)] = (int32_t)b;
        return;
    }
    const unsigned long long kk = tkk[k];
    int32_t r = 0, j = lo;
    for (; j + 8 <= hi; j += 8) {  // eight loads in flight
        unsigned long long v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = tkk[j + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) r += v[u] < kk ? 1 : 0;
    }
    for (; j < hi; ++j) r += tkk[j] < kk ? 1 : 0;
    perm[lo + r] = (int32_t)(kk & 0x7fffffffull);
}

// Buckets above RANK_MAX: a bitonic network over the bucket in place (every
// comparator ascending, the first of each merge against the mirrored
// partner, so that the virtual +inf padding up to a power of two never
// moves), one workgroup per listed bucket.  Exits at once when none is
// listed.
__global__ void __launch_bounds__(256) k_bucket_big(const int32_t *__restrict__ bstart, const int32_t *__restrict__ big,
                                                     const int32_t *__restrict__ nbig,
                                                     unsigned long long *__restrict__ tkk, int32_t *__restrict__ perm)
{
    const int32_t m = *nbig;
    for (int32_t e = blockIdx.x; e < m; e += gridDim.x) {
        const uint32_t b = (uint32_t)big[e];
        const int32_t lo = bstart[b], c = bstart[b + 1] - lo;
        unsigned long long *a = tkk + lo;
        int64_t P = 1;  // 64-bit: c may exceed 2^30
        while (P < c) P <<= 1;
        for (int64_t k = 2; k <= P; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1) {
                for (int32_t i = threadIdx.x; i < c; i += blockDim.x) {
                    const int64_t l = j == (k >> 1) ? (i ^ (k - 1)) : (i ^ j);
                    if (l > i && l < c) {
                        const unsigned long long u = a[i], v = a[l];
                        if (u > v) {
                            a[i] = v;
                            a[l] = u;
                        }
                    }
                }
                __syncthreads();
            }
        for (int32_t i = threadIdx.x; i < c; i += blockDim.x) perm[lo + i] = (int32_t)(a[i] & 0x7fffffffull);
        __syncthreads();
    }
}

// Sorted copies of the sample data; run heads (a new base cell, or every
// 64th sorted sample: the window of one spreading wavefront); the bit of each
// base cell in the base-cell map (set by the first sample of the cell).
__global__ void k_mk_gather(MarkerGeom mg, int64_t n, const int32_t *__restrict__ perm, const int32_t *__restrict__ cell,
                            const float *__restrict__ xyz, const float *__restrict__ ub, const float *__restrict__ area,
                            const float *__restrict__ gain, float *__restrict__ pos_s, float *__restrict__ ub_s,
                            float *__restrict__ area_s, float *__restrict__ gain_s, int32_t *__restrict__ head,
                            unsigned long long *__restrict__ occ)
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
    const int32_t ck = cell[s];
    const bool first = k == 0 || cell[perm[k - 1]] != ck;
    head[k] = (first || (k & 63) == 0) ? 1 : 0;
    if (first) {
        const int x = ck % mg.nx;
        const int64_t row = ck / mg.nx;
        atomicOr(occ + row * mg.ntx + x / SEG, 1ull << (x % SEG));
    }
}

// Band tiles: node (x, y, z) receives force when one of the base cells
// (x, y, z) - d, d in {0, 1}^3, holds a sample (the 2x2x2 stencil, wrapped on
// periodic axes), i.e. the base-cell map dilated by one node towards +x, +y,
// +z.  One lane per 64-node word; also the word's node count.
__global__ void k_dilate(MarkerGeom mg, int64_t W, const unsigned long long *__restrict__ occ,
                         unsigned long long *__restrict__ mask, int32_t *__restrict__ cnt)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const int xs = (int)(w % mg.ntx);
    const int64_t row = w / mg.ntx;
    const int y = (int)(row % mg.ny), z = (int)(row / mg.ny);
    unsigned long long m = 0;
    for (int dz = 0; dz < 2; ++dz) {
        int zz = z - dz;
        if (zz < 0) {
            if (!mg.periodic[2]) continue;
            zz += mg.nz;
        }
        for (int dy = 0; dy < 2; ++dy) {
            int yy = y - dy;
            if (yy < 0) {
                if (!mg.periodic[1]) continue;
                yy += mg.ny;
            }
            const int64_t rb = ((int64_t)zz * mg.ny + yy) * mg.ntx;
            const unsigned long long o = occ[rb + xs];
            m |= o | (o << 1);
            if (xs > 0) {
                m |= occ[rb + xs - 1] >> 63;
            } else if (mg.periodic[0]) {
                const int xl = mg.nx - 1;
                m |= (occ[rb + xl / SEG] >> (xl % SEG)) & 1ull;
            }
        }
    }
    // the shift of a base cell at x = nx - 1 (periodic x) lands past the row
    // end; its node x = 0 was taken above
    const int valid = mg.nx - xs * SEG;
    if (valid < SEG) m &= (1ull << valid) - 1ull;
    mask[w] = m;
    cnt[w] = __popcll(m);
}

// Band list (node index of each band slot, in node order), with the 8 run
// entries of each band node cleared; the tile starts corrected for the run
// heads that precede the tile counts in the shared scan; the last lane also
// stores the band and run counts.
__global__ void k_band_list(MarkerGeom mg, int64_t W, const unsigned long long *__restrict__ mask,
                            int32_t *__restrict__ start, int32_t *__restrict__ band_cell,
                            int32_t *__restrict__ band_src, int64_t bstride, int64_t n,
                            const int32_t *__restrict__ rid, const int32_t *__restrict__ head,
                            int32_t *__restrict__ counts)
{
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    unsigned long long m = mask[w];
    const int32_t nruns = rid[n - 1] + head[n - 1];
    const int32_t s0 = start[w] - nruns;  // the scan ran over the run heads first
    start[w] = s0;
    if (w == W - 1) {
        counts[0] = s0 + __popcll(m);
        counts[1] = nruns;
    }
    if (!m) return;
    const int xs = (int)(w % mg.ntx);
    const int64_t row = w / mg.ntx;
    int r = s0;
    while (m) {
        const int bit = __ffsll((long long)m) - 1;
        m &= m - 1;
        band_cell[r] = (int32_t)(row * mg.nx + xs * SEG + bit);
#pragma unroll
        for (int d = 0; d < 8; ++d) band_src[(int64_t)d * bstride + r] = -1;
        ++r;
    }
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

// Band slots of the 8 stencil nodes of each sorted sample; at a run head the
// run's start, whether it continues the cell of the run before it (a cut at a
// window boundary only), and, for the first run of a cell, the run feeding
// each of the cell's stencil nodes (band_src[d][slot]).  The run after the
// last gets start n and continuation 0, which ends the readers' loops.
__global__ void k_mk_slots(MarkerGeom mg, int64_t n, const float *__restrict__ pos,
                           const unsigned long long *__restrict__ mask, const int32_t *__restrict__ start,
                           const int32_t *__restrict__ head, const int32_t *__restrict__ rid, int32_t *__restrict__ slot,
                           int32_t *__restrict__ run_start, uint8_t *__restrict__ run_cont,
                           int32_t *__restrict__ band_src, int64_t bstride)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t sl[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        int x, y, z;
        stencil_node(mg, pos, n, k, d, x, y, z);
        const int64_t w = ((int64_t)z * mg.ny + y) * mg.ntx + x / SEG;
        const int bit = x % SEG;
        sl[d] = start[w] + __popcll(mask[w] & ((1ull << bit) - 1ull));
        slot[(int64_t)d * n + k] = sl[d];
    }
    if (head[k]) {
        const int32_t r = rid[k];
        const bool cont = k > 0 && floorf(pos[k]) == floorf(pos[k - 1]) &&
                          floorf(pos[n + k]) == floorf(pos[n + k - 1]) &&
                          floorf(pos[2 * n + k]) == floorf(pos[2 * n + k - 1]);
        run_start[r] = (int32_t)k;
        run_cont[r] = cont ? 1 : 0;
        if (!cont)
#pragma unroll
            for (int d = 0; d < 8; ++d) band_src[(int64_t)d * bstride + sl[d]] = r;
    }
    if (k == n - 1) {
        const int32_t nr = rid[k] + head[k];
        run_start[nr] = (int32_t)n;
        run_cont[nr] = 0;
    }
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

// Body-frame bounding box of the samples (one workgroup): lo[3], hi[3], and
// a flag for a non-finite coordinate.
__global__ void __launch_bounds__(256) k_body_bounds(int64_t n, const float *__restrict__ X, float *__restrict__ out)
{
    __shared__ float sh[6][256];
    __shared__ int nonfinite;
    if (threadIdx.x == 0) nonfinite = 0;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool bad = false;
    __syncthreads();
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = X[a * n + s];
            if (!isfinite(v)) bad = true;
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    if (bad) atomicOr(&nonfinite, 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        sh[a][threadIdx.x] = lo[a];
        sh[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sh[a][threadIdx.x] = fminf(sh[a][threadIdx.x], sh[a][threadIdx.x + h]);
                sh[3 + a][threadIdx.x] = fmaxf(sh[3 + a][threadIdx.x], sh[3 + a][threadIdx.x + h]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = sh[threadIdx.x][0];
    if (threadIdx.x == 6) out[6] = nonfinite ? 1.0f : 0.0f;
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

static int64_t block_count(const lbm_ctx *c)
{
    return (int64_t)((c->g.nx + ELL - 1) / ELL) * ((c->g.ny + ELL - 1) / ELL) * ((c->g.nz + ELL - 1) / ELL);
}

int64_t band_capacity(const lbm_ctx *c, int64_t n) { return std::min<int64_t>(8 * std::max<int64_t>(n, 1), c->N); }

hipError_t solids_layout(const lbm_ctx *c, int64_t n, SolidsLayout *L)
{
    const size_t un = (size_t)(n > 0 ? n : 1);
    const size_t W = (size_t)c->g.W;
    const size_t nb = (size_t)block_count(c);
    if (nb >= (size_t(1) << 31)) return hipErrorInvalidValue;  // block index of the sort key
    const size_t nbmax = (size_t)band_capacity(c, n);
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
    L->cell2 = take(un * 4);
    L->perm = take(un * 4);
    L->keys = take(un * 8);
    L->tkk = take(un * 8);
    L->tb = take(un * 4);
    L->bcount = take((nb + 1) * 4);
    L->bstart = take((nb + 1) * 4);
    L->big = take((un / RANK_MAX + 1) * 4);
    L->occ = take(W * 8);
    L->tile_mask = take(W * 8);
    // run heads followed by the tile counts, and their one exclusive scan:
    // run ids followed by the tile starts (offset by the run count until
    // k_band_list subtracts it)
    L->run_head = take((un + W) * 4);
    L->tile_count = L->run_head + un * 4;
    L->run_id = take((un + W) * 4);
    L->tile_start = L->run_id + un * 4;
    size_t scan_bytes = 0;
    hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (int32_t *)nullptr, (int32_t *)nullptr,
                                                    (int)std::max<size_t>(un + W, nb + 1));
    if (e != hipSuccess) return e;
    L->scan_tmp_bytes = scan_bytes;
    L->scan_tmp = take(scan_bytes);
    L->band_cell = take(nbmax * 4);
    L->band_ru = take(nbmax * 4 * c->rsize);
    L->band_force = take(nbmax * 4 * c->rsize);
    L->ib_part = take(((un + 255) / 256) * 8 * 8);
    L->run_start = take((un + 1) * 4);
    L->run_cont = take(un + 1);
    L->run_sum = take(8 * un * 4 * c->rsize);
    L->band_src = take(8 * nbmax * 4);
    L->band_push = take(18 * nbmax * c->rsize);
    L->push_feeds = take(W * 4);
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

// misc block: [0] out-of-domain count, [16] band and run counts, [32] count
// of buckets above RANK_MAX, [64] body box (7 floats)
static int *misc_bad(lbm_ctx *c, const SolidsLayout &L) { return reinterpret_cast<int *>(c->mws + L.misc); }

// pose == NULL: xyz and ub are the positions; else they are the staging
// arrays that the key kernel fills from the body copy at the pose
static hipError_t setup_impl(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area,
                             const float *gain, const Pose *pose, bool wait, int *bad_host)
{
    SolidsLayout L;
    hipError_t e = solids_layout(c, n, &L);
    if (e != hipSuccess) return e;
    char *m = c->mws;
    const MarkerGeom mg = marker_geom(c);
    const int64_t W = c->g.W, nb = block_count(c);
    auto I32 = [&](size_t off) { return reinterpret_cast<int32_t *>(m + off); };
    auto *keys = reinterpret_cast<unsigned long long *>(m + L.keys);
    auto *tkk = reinterpret_cast<unsigned long long *>(m + L.tkk);
    auto *tb = reinterpret_cast<uint32_t *>(m + L.tb);
    auto *occ = reinterpret_cast<unsigned long long *>(m + L.occ);
    int32_t *bcount = I32(L.bcount), *bstart = I32(L.bstart), *big = I32(L.big), *perm = I32(L.perm);
    int32_t *cell = c->m_cell_next;  // the current base cells stay intact until the samples pass the checks
    int *bad = misc_bad(c, L);
    int32_t *counts = I32(L.misc + 16), *nbig = I32(L.misc + 32);
    hipStream_t st = c->stream;

    // the count of samples outside starts at zero, except for a placement that
    // does not wait: its count adds up until a synchronising call reads it
    if (!pose || wait) hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, bad);
    if (pose)
        hipLaunchKernelGGL(k_mk_keys<true>, grid_for(n), dim3(256), 0, st, mg, n, xyz, keys, cell, bcount, bad, occ, W,
                           nbig, *pose, c->b_xyz, c->b_ub, c->w_xyz, c->w_ub);
    else
        hipLaunchKernelGGL(k_mk_keys<false>, grid_for(n), dim3(256), 0, st, mg, n, xyz, keys, cell, bcount, bad, occ,
                           W, nbig, Pose{}, nullptr, nullptr, nullptr, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    *bad_host = 0;
    if (wait) {
        if ((e = hipMemcpyAsync(bad_host, bad, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (*bad_host) return launch_zero(c, bcount, (size_t)(nb + 1) * 4);  // the histogram holds the others
    }
    // bucket sort (one bucket per l^3 block)
    size_t scan_bytes = L.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(m + L.scan_tmp, scan_bytes, bcount, bstart, (int)(nb + 1), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter, grid_for(n), dim3(256), 0, st, n, keys, bstart, bcount, tb, tkk);
    hipLaunchKernelGGL(k_bucket_rank, grid_for(n), dim3(256), 0, st, n, bstart, tb, tkk, perm, big, nbig);
    hipLaunchKernelGGL(k_bucket_big, dim3(BIG_SORT_BLOCKS), dim3(256), 0, st, bstart, big, nbig, tkk, perm);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    c->m_pos = reinterpret_cast<float *>(m + L.pos);
    c->m_ub = reinterpret_cast<float *>(m + L.ub);
    c->m_area = reinterpret_cast<float *>(m + L.area);
    c->m_gain = reinterpret_cast<float *>(m + L.gain);
    c->m_slot = I32(L.slot);
    c->m_cell_next = c->m_cell;
    c->m_cell = cell;
    c->m_perm = perm;
    c->tile_mask = reinterpret_cast<uint64_t *>(m + L.tile_mask);
    c->tile_start = I32(L.tile_start);
    c->band_cell = I32(L.band_cell);
    c->band_ru = m + L.band_ru;
    c->band_force = m + L.band_force;
    c->ib_part = reinterpret_cast<double *>(m + L.ib_part);
    c->run_start = I32(L.run_start);
    c->run_id = I32(L.run_id);
    c->run_cont = reinterpret_cast<uint8_t *>(m + L.run_cont);
    c->run_sum = m + L.run_sum;
    c->band_src = I32(L.band_src);
    c->band_push = m + L.band_push;
    c->push_feeds = reinterpret_cast<uint32_t *>(m + L.push_feeds);
    c->push_valid = false;  // a new band: no pieces for it yet
    c->feeds_valid = false;
    c->nbcap = band_capacity(c, n);
    c->dcounts = counts;
    c->dbad = bad;
    auto *mask = reinterpret_cast<unsigned long long *>(c->tile_mask);
    int32_t *head = I32(L.run_head), *cnt = I32(L.tile_count);

    hipLaunchKernelGGL(k_mk_gather, grid_for(n), dim3(256), 0, st, mg, n, perm, cell, xyz, ub, area, gain, c->m_pos,
                       c->m_ub, c->m_area, c->m_gain, head, occ);
    hipLaunchKernelGGL(k_dilate, grid_for(W), dim3(256), 0, st, mg, W, occ, mask, cnt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    scan_bytes = L.scan_tmp_bytes;
    e = hipcub::DeviceScan::ExclusiveSum(m + L.scan_tmp, scan_bytes, head, c->run_id, (int)(n + W), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_list, grid_for(W), dim3(256), 0, st, mg, W, mask, c->tile_start, c->band_cell,
                       c->band_src, c->nbcap, n, c->run_id, head, counts);
    hipLaunchKernelGGL(k_mk_slots, grid_for(n), dim3(256), 0, st, mg, n, c->m_pos, mask, c->tile_start, head,
                       c->run_id, c->m_slot, c->run_start, c->run_cont, c->band_src, c->nbcap);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!wait) {
        c->counts_exact = false;  // the counts stay on the device; nband / nruns keep the last read values
        return hipSuccess;
    }
    return read_counts(c);
}

hipError_t solids_setup(lbm_ctx *c, int64_t n, const float *xyz, const float *ub, const float *area, const float *gain,
                        bool wait, int *bad_host)
{
    return setup_impl(c, n, xyz, ub, area, gain, nullptr, wait, bad_host);
}

hipError_t read_counts(lbm_ctx *c)
{
    int32_t got[2];
    hipError_t e = hipMemcpyAsync(got, c->dcounts, sizeof(got), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    c->nband = got[0];
    c->nruns = got[1];
    c->counts_exact = true;
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
    c->dbad = misc_bad(c, L);
    c->box_state = 0;
    // the block histogram starts at zero; every set-up leaves it at zero
    if ((e = launch_zero(c, m + L.bcount, (size_t)(block_count(c) + 1) * 4)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_body_store, grid_for(n), dim3(256), 0, c->stream, n, xyz, ub, area, gain, c->b_xyz, c->b_ub,
                       c->b_area, c->b_gain);
    return hipGetLastError();
}

hipError_t body_box(lbm_ctx *c)
{
    SolidsLayout L;
    hipError_t e = solids_layout(c, c->nm, &L);
    if (e != hipSuccess) return e;
    float *out = reinterpret_cast<float *>(c->mws + L.misc + 64);
    hipLaunchKernelGGL(k_body_bounds, dim3(1), dim3(256), 0, c->stream, c->nm, c->b_xyz, out);
    float box[7];
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(box, out, sizeof(box), hipMemcpyDeviceToHost, c->stream)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return e;
    for (int a = 0; a < 3; ++a) {
        c->box_lo[a] = box[a];
        c->box_hi[a] = box[3 + a];
    }
    c->box_state = box[6] == 0.0f ? 1 : -1;
    return hipSuccess;
}

hipError_t solids_pose(lbm_ctx *c, const double R[9], const double o[3], const double v[3], const double w[3],
                       bool wait, int *bad_host)
{
    Pose P{};
    for (int k = 0; k < 9; ++k) P.R[k] = R[k];
    for (int a = 0; a < 3; ++a) {
        P.o[a] = o[a];
        P.v[a] = v[a];
        P.w[a] = w[a];
    }
    return setup_impl(c, c->nm, c->w_xyz, c->w_ub, c->b_area, c->b_gain, &P, wait, bad_host);
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
