// Host checks of the index arithmetic shared by the kernels (compiled and run
// by test_host_index.py): the invariant-divisor division and the population
// layout offsets.  Prints one line per failure and "OK" at the end.
#include "lbm_internal.hpp"

#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

using namespace lbm;

static int check_divisor(uint32_t d, std::mt19937_64 &rng)
{
    const Divisor D = make_divisor(d);
    int bad = 0;
    auto one = [&](uint32_t n) {
        if (divide(n, D) != n / d) {
            if (bad++ < 5) std::printf("divide(%u, %u) = %u, expected %u\n", n, d, divide(n, D), n / d);
        }
    };
    for (uint32_t n = 0; n < (1u << 20); ++n) one(n);                 // every small numerator
    for (uint64_t k = 1; k * d < (1ull << 31); k = k * 3 + 1)         // around multiples of d
        for (int e = -2; e <= 2; ++e) {
            const int64_t n = (int64_t)(k * d) + e;
            if (n >= 0 && n < (1ll << 31)) one((uint32_t)n);
        }
    for (int t = 0; t < 200000; ++t) one((uint32_t)(rng() & 0x7fffffffu));
    one(0x7fffffffu);
    return bad;
}

static int check_layout(int nx, int ny, int nz, int lr)
{
    Geom g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.nxp = (nx + 31) / 32 * 32;
    const int64_t rows = (int64_t)ny * nz;
    if (lr == 31) {
        g.lr = 31;
        g.rmask = 0x7fffffff;
        g.plane = (rows * g.nxp + 63) / 64 * 64;
        g.bstride = 0;
        g.total = 27 * g.plane;
    } else {
        const int64_t R = int64_t(1) << lr;
        g.lr = lr;
        g.rmask = R - 1;
        g.plane = R * g.nxp;
        g.bstride = 27 * g.plane;
        g.total = ((rows + R - 1) >> lr) * g.bstride;
    }
    std::vector<unsigned char> hit((size_t)g.total, 0);
    int bad = 0;
    for (int i = 0; i < 27; ++i)
        for (int64_t r = 0; r < rows; ++r)
            for (int x = 0; x < g.nxp; ++x) {
                const int64_t a = (int64_t)i * g.plane + row_off(g, r) + x;
                if (a < 0 || a >= g.total || hit[(size_t)a]++) {
                    if (bad++ < 5) std::printf("layout %dx%dx%d lr=%d: bad offset for i=%d row=%lld x=%d\n", nx, ny, nz,
                                               lr, i, (long long)r, x);
                }
            }
    return bad;
}

// every node on a non-periodic face layer exactly once, nothing else
static int check_faces(int nx, int ny, int nz, int xf, int yf, int zf)
{
    Geom g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    const int P = LBM_PERIODIC, N = LBM_NOSLIP;
    const int fc[6] = {xf ? LBM_INLET : P, xf ? LBM_OUTFLOW : P, yf ? N : P, yf ? N : P, zf ? N : P, zf ? N : P};
    for (int k = 0; k < 6; ++k) g.face[k] = fc[k];
    const FaceSet F = face_set(g);
    std::vector<int> hit((size_t)nx * ny * nz, 0);
    int bad = 0;
    for (int64_t k = 0; k < F.na + F.nb; ++k) {
        int x, y, z;
        face_node(k, g, F, x, y, z);
        if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz) {
            if (bad++ < 5) std::printf("faces %dx%dx%d: k=%lld out of range\n", nx, ny, nz, (long long)k);
            continue;
        }
        hit[(size_t)x + (size_t)nx * (y + (size_t)ny * z)]++;
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const bool face = (xf && (x == 0 || x == nx - 1)) || (yf && (y == 0 || y == ny - 1)) ||
                                  (zf && (z == 0 || z == nz - 1));
                const int h = hit[(size_t)x + (size_t)nx * (y + (size_t)ny * z)];
                if (h != (face ? 1 : 0)) {
                    if (bad++ < 5) std::printf("faces %dx%dx%d (%d%d%d): node (%d,%d,%d) hit %d times\n", nx, ny, nz, xf, yf, zf, x, y, z, h);
                }
            }
    return bad;
}

int main()
{
    std::mt19937_64 rng(2101);
    int bad = 0;
    const uint32_t ds[] = {1, 2, 3, 4, 5, 7, 12, 19, 64, 100, 250, 256, 840, 1000, 4093, 65536, 1u << 20, 123457,
                           (1u << 30) + 1, 0x7fffffffu};
    for (uint32_t d : ds) bad += check_divisor(d, rng);
    const int dims[][3] = {{16, 8, 8}, {24, 12, 12}, {70, 18, 15}, {33, 7, 3}, {1200, 5, 3}, {64, 1, 1}, {100, 9, 1}};
    for (auto &d : dims)
        for (int lr : {0, 1, 2, 3, 4, 31})
            if (lr == 31 || (int64_t(1) << lr) <= (int64_t)d[1] * d[2]) bad += check_layout(d[0], d[1], d[2], lr);
    const int fd[][3] = {{7, 5, 4}, {2, 2, 2}, {2, 3, 2}, {5, 2, 3}, {64, 9, 6}, {70, 18, 15}, {3, 1, 4}};
    for (auto &d : fd)
        for (int m = 0; m < 8; ++m)
            if ((!(m & 2) || d[1] >= 2) && (!(m & 4) || d[2] >= 2)) bad += check_faces(d[0], d[1], d[2], m & 1, (m >> 1) & 1, (m >> 2) & 1);
    std::printf(bad ? "FAIL %d\n" : "OK\n", bad);
    return bad != 0;
}
