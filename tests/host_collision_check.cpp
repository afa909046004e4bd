// Host build of the fused kernel's collision functions (lbm_internal.hpp) in
// FP64, driven by test_host_collision.py: reads cases from stdin, one per
// line -- model (0 central moments, 1 central moments with unit high-order
// rates, 2 BGK, 3 raw-moment MRT), the six rates s_nu s_b s3 s4 s5 s6, the
// force F, then the 27 pulled deviations in population order -- and prints
// the 27 post-collision deviations per case.
#include "lbm_internal.hpp"

#include <cstdio>

using namespace lbm;
using R = double;

int main()
{
    int model;
    while (std::scanf("%d", &model) == 1) {
        Rates<R> rt;
        R F[3], d[27];
        if (std::scanf("%lf %lf %lf %lf %lf %lf", &rt.s_nu, &rt.s_b, &rt.s3, &rt.s4, &rt.s5, &rt.s6) != 6) return 1;
        if (std::scanf("%lf %lf %lf", &F[0], &F[1], &F[2]) != 3) return 1;
        for (int i = 0; i < 27; ++i)
            if (std::scanf("%lf", &d[i]) != 1) return 1;
        R f[3][3][3];
        for (int i = 0; i < 27; ++i) f[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = d[i];
        R rho, ux, uy, uz;
        switch (model) {
        case 0: collide_as<COLL_CM>(f, F[0], F[1], F[2], rt, rho, ux, uy, uz); break;
        case 1: collide_as<COLL_CM_UNIT_HIGH>(f, F[0], F[1], F[2], rt, rho, ux, uy, uz); break;
        case 2: collide_as<COLL_BGK>(f, F[0], F[1], F[2], rt, rho, ux, uy, uz); break;
        case 3: collide_as<COLL_RM>(f, F[0], F[1], F[2], rt, rho, ux, uy, uz); break;
        default: return 1;
        }
        for (int i = 0; i < 27; ++i) std::printf("%.17g%c", f[CZ[i] + 1][CY[i] + 1][CX[i] + 1], i == 26 ? '\n' : ' ');
    }
    return 0;
}
