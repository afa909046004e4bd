// Host check of the hand-written reverse modes of the per-node collision
// (collide_vjp, and collide_unit_high_vjp for unit rates of orders 3 to 6, in
// lbm_adjoint.hpp) against central differences of the forward collisions
// (collide, collide_unit_high in lbm_internal.hpp), all compiled for the CPU
// in FP64.  For random pulled deviations, forces, relaxation rates and output
// adjoints g, J = <g, collide(d, F)> is differentiated numerically in each of
// the 27 deviations and 3 force components and compared with the VJP.
// Prints one line per failure, the worst relative error, and "OK" at the end.
#include "lbm_adjoint.hpp"

#include <cmath>
#include <cstdio>
#include <random>

using namespace lbm;
using R = double;

static R objective(const R (&d)[3][3][3], const R F[3], const Rates<R> &rt, const R (&g)[3][3][3], bool unit)
{
    R f[3][3][3];
    copy27(f, d);
    R rho, ux, uy, uz;
    if (unit) collide_unit_high(f, F[0], F[1], F[2], rt, rho, ux, uy, uz);
    else collide(f, F[0], F[1], F[2], rt, rho, ux, uy, uz);
    R J = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) J += g[a][b][c] * f[a][b][c];
    return J;
}

int main()
{
    std::mt19937_64 rng(20240611);
    std::normal_distribution<R> N(0.0, 1.0);
    std::uniform_real_distribution<R> U(0.05, 1.95);
    int bad = 0;
    R worst = 0;
    // cases 0-39: collide_vjp against collide (any rates); cases 40-79:
    // collide_unit_high_vjp against collide_unit_high (orders 3-6 at rate 1)
    for (int t = 0; t < 80; ++t) {
        const bool unit = t >= 40;
        // deviations of a near-equilibrium node: scale 0.01 (velocities ~0.05)
        R d[3][3][3], g[3][3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c) {
                    d[a][b][c] = 0.01 * N(rng);
                    g[a][b][c] = N(rng);
                }
        R F[3] = {1e-3 * N(rng), 1e-3 * N(rng), 1e-3 * N(rng)};
        Rates<R> rt{U(rng), U(rng), U(rng), U(rng), U(rng), U(rng)};
        if (t % 4 == 0) rt = {1.99, 1.0, 1.0, 1.0, 1.0, 1.0};  // the default high-order rates
        if (unit) rt.s3 = rt.s4 = rt.s5 = rt.s6 = 1.0;
        // reverse mode
        R gv[3][3][3];
        copy27(gv, g);
        R Fb[3] = {0, 0, 0};
        if (unit) collide_unit_high_vjp(d, F[0], F[1], F[2], rt, gv, Fb[0], Fb[1], Fb[2]);
        else collide_vjp(d, F[0], F[1], F[2], rt, gv, Fb[0], Fb[1], Fb[2]);
        // central differences, step h, error O(h^2) + round-off O(eps/h)
        const R h = 1e-6;
        R num[30], ana[30];
        int k = 0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int c = 0; c < 3; ++c, ++k) {
                    R dp[3][3][3], dm[3][3][3];
                    copy27(dp, d);
                    copy27(dm, d);
                    dp[a][b][c] += h;
                    dm[a][b][c] -= h;
                    num[k] = (objective(dp, F, rt, g, unit) - objective(dm, F, rt, g, unit)) / (2 * h);
                    ana[k] = gv[a][b][c];
                }
        for (int e = 0; e < 3; ++e, ++k) {
            R Fp[3] = {F[0], F[1], F[2]}, Fm[3] = {F[0], F[1], F[2]};
            Fp[e] += h;
            Fm[e] -= h;
            num[k] = (objective(d, Fp, rt, g, unit) - objective(d, Fm, rt, g, unit)) / (2 * h);
            ana[k] = Fb[e];
        }
        R nn = 0, ne = 0;
        for (int j = 0; j < 30; ++j) {
            nn += num[j] * num[j];
            ne += (num[j] - ana[j]) * (num[j] - ana[j]);
        }
        const R rel = std::sqrt(ne / nn);
        if (rel > worst) worst = rel;
        if (!(rel <= 1e-7)) {
            if (bad++ < 5) std::printf("case %d: relative error %.3e\n", t, rel);
        }
    }
    std::printf("worst relative error %.3e\n", worst);
    std::printf(bad ? "FAIL\n" : "OK\n");
    return bad ? 1 : 0;
}
