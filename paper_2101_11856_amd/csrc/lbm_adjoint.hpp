// lbm_adjoint.hpp -- hand-written reverse mode of the per-node collision
// (Eqs. 4-5 in the deviation-moment form of lbm_internal.hpp).
//
// Given the pulled deviations d* and force F of a node, and the adjoint g of
// its post-collision deviations, collide_vjp returns the adjoint of d* (in g)
// and of F.  The forward pieces are recomputed from d* with the very same
// functions the step uses; the reverse sweep transposes each stage in turn:
// inverse raw transform, inverse shift, relaxation, shift, velocity, raw
// transform.
#pragma once

#include "lbm_internal.hpp"

namespace lbm {

// ---- transposes of the 3-point line operations ---------------------------

// raw3: (a, b, c) -> (a + b + c, c - a, c + a)
template <typename R> __host__ __device__ __forceinline__ void raw3_T(R &a, R &b, R &c)
{
    const R g0 = a, g1 = b, g2 = c;
    a = g0 - g1 + g2;
    b = g0;
    c = g0 + g1 + g2;
}
// iraw3: (m0, m1, m2) -> ((m2 - m1)/2, m0 - m2, (m2 + m1)/2)
template <typename R> __host__ __device__ __forceinline__ void iraw3_T(R &a, R &b, R &c)
{
    const R gm = a, g0 = b, gp = c;
    a = g0;
    b = (R)0.5 * (gp - gm);
    c = (R)0.5 * (gm + gp) - g0;
}
// shift3 at input line (m0, m1, m2): k1 = m1 - u m0, k2 = m2 - 2u m1 + u^2 m0.
// (h0, h1, h2) adjoint of k  ->  adjoint of m; ub += d/du.
template <typename R>
__host__ __device__ __forceinline__ void shift3_T(R &h0, R &h1, R &h2, R m0, R m1, R u, R &ub)
{
    const R k1 = m1 - u * m0;
    ub += -m0 * h1 - (R)2 * k1 * h2;
    const R n0 = h0 - u * h1 + u * u * h2;
    const R n1 = h1 - (R)2 * u * h2;
    h0 = n0;
    h1 = n1;
}
// unshift3 at input line (k0, k1, k2): m1 = k1 + u k0, m2 = k2 + 2u k1 + u^2 k0.
template <typename R>
__host__ __device__ __forceinline__ void unshift3_T(R &g0, R &g1, R &g2, R k0, R k1, R u, R &ub)
{
    const R m1 = k1 + u * k0;
    ub += k0 * g1 + (R)2 * m1 * g2;
    const R n0 = g0 + u * g1 + u * u * g2;
    const R n1 = g1 + (R)2 * u * g2;
    g0 = n0;
    g1 = n1;
}

// line loops pairing the adjoint array g with the saved forward input S
template <typename R, typename Op>
__host__ __device__ __forceinline__ void lines2_x(R (&g)[3][3][3], const R (&S)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(g[a][b][0], g[a][b][1], g[a][b][2], S[a][b][0], S[a][b][1]);
}
template <typename R, typename Op>
__host__ __device__ __forceinline__ void lines2_y(R (&g)[3][3][3], const R (&S)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(g[a][0][b], g[a][1][b], g[a][2][b], S[a][0][b], S[a][1][b]);
}
template <typename R, typename Op>
__host__ __device__ __forceinline__ void lines2_z(R (&g)[3][3][3], const R (&S)[3][3][3], Op op)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) op(g[0][a][b], g[1][a][b], g[2][a][b], S[0][a][b], S[1][a][b]);
}

template <typename R> __host__ __device__ __forceinline__ void copy27(R (&d)[3][3][3], const R (&s)[3][3][3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) d[a][b][c] = s[a][b][c];
}

// Per-axis factors of Delta = prod_a P_{e_a}(u_a) - (1 + drho) prod_a E_{e_a}:
// P0 = 1, P1 = -u, P2 = 1/3 + u^2; E0 = 1, E1 = 0, E2 = 1/3.
template <typename R> __host__ __device__ __forceinline__ R Pf(int e, R u)
{
    return e == 0 ? (R)1 : e == 1 ? -u : (R)(1.0 / 3.0) + u * u;
}
template <typename R> __host__ __device__ __forceinline__ R dPf(int e, R u)
{
    return e == 0 ? (R)0 : e == 1 ? (R)-1 : (R)2 * u;
}
__host__ __device__ constexpr double Ef(int e) { return e == 0 ? 1.0 : e == 1 ? 0.0 : 1.0 / 3.0; }

// Reverse of relax(): on entry g = adjoint of kappa'(d); on exit g = adjoint
// of kappa(d); ub/drhob/Fb accumulate the adjoints of u, drho and F.
template <typename R>
__host__ __device__ __forceinline__ void relax_T(R (&g)[3][3][3], R ux, R uy, R uz, const Rates<R> &rt, R &ubx,
                                                 R &uby, R &ubz, R &drhob, R &Fbx, R &Fby, R &Fbz)
{
    R Db[3][3][3];  // adjoint of Delta
    // order 0 and 1: rate 0; order 1 carries F
    Db[0][0][0] = 0;
    Db[0][0][1] = Db[0][1][0] = Db[1][0][0] = 0;
    Fbx += g[0][0][1];
    Fby += g[0][1][0];
    Fbz += g[1][0][0];
    // order 2 diagonal (deviator s_nu, trace s_b)
    {
        const R sumg = g[0][0][2] + g[0][2][0] + g[2][0][0];
        const R t = (rt.s_b - rt.s_nu) * (R)(1.0 / 3.0) * sumg;
        const R nx = -rt.s_nu * g[0][0][2] - t, ny = -rt.s_nu * g[0][2][0] - t, nz = -rt.s_nu * g[2][0][0] - t;
        g[0][0][2] += nx;
        g[0][2][0] += ny;
        g[2][0][0] += nz;
        Db[0][0][2] = nx;
        Db[0][2][0] = ny;
        Db[2][0][0] = nz;
    }
    // all other moments of order >= 2: kappa' = kappa - s (kappa + Delta) + h kappa_F
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int n = a + b + c;
                const bool diag2 = n == 2 && (a == 2 || b == 2 || c == 2);
                if (n < 2 || diag2) continue;
                const R s = n == 2 ? rt.s_nu : n == 3 ? rt.s3 : n == 4 ? rt.s4 : n == 5 ? rt.s5 : rt.s6;
                const R gv = g[c][b][a];
                Db[c][b][a] = -s * gv;
                g[c][b][a] = ((R)1 - s) * gv;
                // forcing: exactly one exponent 1, the others 0 or 2: F_axis cs^(2 #twos)
                const int ones = (a == 1) + (b == 1) + (c == 1);
                if (ones == 1) {
                    const int twos = (a == 2) + (b == 2) + (c == 2);
                    const R w = ((R)1 - (R)0.5 * s) * (twos == 0 ? (R)1 : twos == 1 ? (R)(1.0 / 3.0) : (R)(1.0 / 9.0));
                    if (a == 1) Fbx += w * gv;
                    else if (b == 1) Fby += w * gv;
                    else Fbz += w * gv;
                }
            }
    // Delta depends on u and drho
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (a + b + c < 2) continue;
                const R d = Db[c][b][a];
                const R pa = Pf(a, ux), pb = Pf(b, uy), pc = Pf(c, uz);
                ubx += d * dPf(a, ux) * pb * pc;
                uby += d * pa * dPf(b, uy) * pc;
                ubz += d * pa * pb * dPf(c, uz);
                drhob -= d * (R)(Ef(a) * Ef(b) * Ef(c));
            }
}

// Adjoint of collide(): fs = pulled deviations (unchanged), F = force;
// g in: adjoint of post-collision deviations, out: adjoint of fs;
// Fb += adjoint of F.
template <typename R>
__host__ __device__ __forceinline__ void collide_vjp(const R (&fs)[3][3][3], R Fx, R Fy, R Fz, const Rates<R> &rt,
                                                     R (&g)[3][3][3], R &Fbx, R &Fby, R &Fbz)
{
    // forward recompute: raw moments m, velocity, relaxed central moments kp
    R m[3][3][3];
    copy27(m, fs);
    raw_all(m);
    R drho, ux, uy, uz;
    velocity(m, Fx, Fy, Fz, drho, ux, uy, uz);
    const R inv = (R)1 / ((R)1 + drho);
    R kp[3][3][3];
    copy27(kp, m);
    lines_x(kp, [ux](R &a, R &b, R &c) { shift3(a, b, c, ux); });
    lines_y(kp, [uy](R &a, R &b, R &c) { shift3(a, b, c, uy); });
    lines_z(kp, [uz](R &a, R &b, R &c) { shift3(a, b, c, uz); });
    relax(kp, ux, uy, uz, drho, Fx, Fy, Fz, rt);

    R ubx = 0, uby = 0, ubz = 0, drhob = 0;
    // inverse raw transform (forward order z, y, x)
    auto irT = [](R &a, R &b, R &c) { iraw3_T(a, b, c); };
    lines_x(g, irT);
    lines_y(g, irT);
    lines_z(g, irT);
    // inverse shift (forward order z, y, x on kp): inputs kp, C = Z(kp), D = Y(C)
    {
        R C[3][3][3], D[3][3][3];
        copy27(C, kp);
        lines_z(C, [uz](R &a, R &b, R &c) { unshift3(a, b, c, uz); });
        copy27(D, C);
        lines_y(D, [uy](R &a, R &b, R &c) { unshift3(a, b, c, uy); });
        lines2_x(g, D, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, ux, ubx); });
        lines2_y(g, C, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, uy, uby); });
    }
    {
        // kp is still the input of the z stage: recompute it (relax overwrote nothing else)
        lines2_z(g, kp, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, uz, ubz); });
    }
    // relaxation
    relax_T(g, ux, uy, uz, rt, ubx, uby, ubz, drhob, Fbx, Fby, Fbz);
    // shift (forward order x, y, z on m): inputs m, A = X(m), B = Y(A)
    {
        R A[3][3][3], B[3][3][3];
        copy27(A, m);
        lines_x(A, [ux](R &a, R &b, R &c) { shift3(a, b, c, ux); });
        copy27(B, A);
        lines_y(B, [uy](R &a, R &b, R &c) { shift3(a, b, c, uy); });
        lines2_z(g, B, [&](R &h0, R &h1, R &h2, R m0, R m1) { shift3_T(h0, h1, h2, m0, m1, uz, ubz); });
        lines2_y(g, A, [&](R &h0, R &h1, R &h2, R m0, R m1) { shift3_T(h0, h1, h2, m0, m1, uy, uby); });
    }
    lines2_x(g, m, [&](R &h0, R &h1, R &h2, R m0, R m1) { shift3_T(h0, h1, h2, m0, m1, ux, ubx); });
    // velocity u = (j + F/2) / rho, rho = 1 + drho
    g[0][0][1] += ubx * inv;
    g[0][1][0] += uby * inv;
    g[1][0][0] += ubz * inv;
    Fbx += (R)0.5 * ubx * inv;
    Fby += (R)0.5 * uby * inv;
    Fbz += (R)0.5 * ubz * inv;
    g[0][0][0] += drhob - (ubx * ux + uby * uy + ubz * uz) * inv;
    // raw transform (forward order x, y, z)
    auto rT = [](R &a, R &b, R &c) { raw3_T(a, b, c); };
    lines_z(g, rT);
    lines_y(g, rT);
    lines_x(g, rT);
}

// Adjoint of collide_unit_high() (orders 3 to 6 at unit rate, the default):
// the post-collision central moments are closed forms of rho, u, F and the
// order-2 central moments, so the reverse sweep needs only the raw moments of
// orders 0-2 of the pulled state.  Same arguments as collide_vjp.
template <typename R>
__host__ __device__ __forceinline__ void collide_unit_high_vjp(const R (&fs)[3][3][3], R Fx, R Fy, R Fz,
                                                               const Rates<R> &rt, R (&g)[3][3][3], R &Fbx, R &Fby,
                                                               R &Fbz)
{
    // forward recompute: raw moments of orders 0-2, kappa' and u
    const Low<R> L = low_moments(fs);
    R kp[3][3][3];
    R rho, ux, uy, uz;
    unit_high_kappa(L, kp, Fx, Fy, Fz, rt, rho, ux, uy, uz);
    const R drho = L.m000, inv = (R)1 / rho;
    R ubx = 0, uby = 0, ubz = 0;
    // inverse raw transform, then inverse shift (as in collide_vjp): g -> adjoint of kappa'
    auto irT = [](R &a, R &b, R &c) { iraw3_T(a, b, c); };
    lines_x(g, irT);
    lines_y(g, irT);
    lines_z(g, irT);
    {
        R C[3][3][3], D[3][3][3];
        copy27(C, kp);
        lines_z(C, [uz](R &a, R &b, R &c) { unshift3(a, b, c, uz); });
        copy27(D, C);
        lines_y(D, [uy](R &a, R &b, R &c) { unshift3(a, b, c, uy); });
        lines2_x(g, D, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, ux, ubx); });
        lines2_y(g, C, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, uy, uby); });
    }
    lines2_z(g, kp, [&](R &g0, R &g1, R &g2, R k0, R k1) { unshift3_T(g0, g1, g2, k0, k1, uz, ubz); });

    // reverse of unit_high_kappa: g[c][b][a] is the adjoint of kappa'_abc
    const R third = (R)(1.0 / 3.0), ninth = (R)(1.0 / 9.0);
    const R x2 = ux * ux, y2 = uy * uy, z2 = uz * uz;
    const R px = third + x2, py = third + y2, pz = third + z2;
    const R k100 = L.m100 - ux * drho, k010 = L.m010 - uy * drho, k001 = L.m001 - uz * drho;
    const R s = rt.s_nu;
    R drb = 0, x2b = 0, y2b = 0, z2b = 0, pxb = 0, pyb = 0, pzb = 0;
    R k100b = 0, k010b = 0, k001b = 0, k200b = 0, k020b = 0, k002b = 0, k110b = 0, k101b = 0, k011b = 0;
    // orders 0 and 1
    drb += g[0][0][0];
    k100b += g[0][0][1];
    Fbx += g[0][0][1];
    k010b += g[0][1][0];
    Fby += g[0][1][0];
    k001b += g[1][0][0];
    Fbz += g[1][0][0];
    // order 2, off-diagonal: (1 - s) k - s u_a u_b
    k110b += ((R)1 - s) * g[0][1][1];
    ubx -= s * uy * g[0][1][1];
    uby -= s * ux * g[0][1][1];
    k101b += ((R)1 - s) * g[1][0][1];
    ubx -= s * uz * g[1][0][1];
    ubz -= s * ux * g[1][0][1];
    k011b += ((R)1 - s) * g[1][1][0];
    uby -= s * uz * g[1][1][0];
    ubz -= s * uy * g[1][1][0];
    // order 2, diagonal: k - (s n + tr), n = k + u^2 - drho/3, tr = (s_b - s)/3 (n_x + n_y + n_z)
    {
        const R a = g[0][0][2], b = g[0][2][0], d = g[2][0][0];
        const R tb = (rt.s_b - s) * third * (a + b + d);
        const R nxb = -s * a - tb, nyb = -s * b - tb, nzb = -s * d - tb;
        k200b += a + nxb;
        k020b += b + nyb;
        k002b += d + nzb;
        x2b += nxb;
        y2b += nyb;
        z2b += nzb;
        drb -= third * (nxb + nyb + nzb);
    }
    // order 3
    ubx += py * g[0][2][1] + pz * g[2][0][1];
    pyb += ux * g[0][2][1];
    pzb += ux * g[2][0][1];
    Fbx += (R)(1.0 / 6.0) * (g[0][2][1] + g[2][0][1]);
    uby += px * g[0][1][2] + pz * g[2][1][0];
    pxb += uy * g[0][1][2];
    pzb += uy * g[2][1][0];
    Fby += (R)(1.0 / 6.0) * (g[0][1][2] + g[2][1][0]);
    ubz += px * g[1][0][2] + py * g[1][2][0];
    pxb += uz * g[1][0][2];
    pyb += uz * g[1][2][0];
    Fbz += (R)(1.0 / 6.0) * (g[1][0][2] + g[1][2][0]);
    ubx += uy * uz * g[1][1][1];
    uby += ux * uz * g[1][1][1];
    ubz += ux * uy * g[1][1][1];
    // order 4
    drb += ninth * (g[2][2][0] + g[2][0][2] + g[0][2][2]);
    x2b -= (third + y2) * g[0][2][2] + (third + z2) * g[2][0][2];
    y2b -= (third + x2) * g[0][2][2] + (third + z2) * g[2][2][0];
    z2b -= (third + x2) * g[2][0][2] + (third + y2) * g[2][2][0];
    pxb -= uy * uz * g[1][1][2];
    uby -= px * uz * g[1][1][2];
    ubz -= px * uy * g[1][1][2];
    pyb -= ux * uz * g[1][2][1];
    ubx -= py * uz * g[1][2][1];
    ubz -= py * ux * g[1][2][1];
    pzb -= ux * uy * g[2][1][1];
    ubx -= pz * uy * g[2][1][1];
    uby -= pz * ux * g[2][1][1];
    // order 5
    ubx += py * pz * g[2][2][1];
    pyb += ux * pz * g[2][2][1];
    pzb += ux * py * g[2][2][1];
    Fbx += (R)(1.0 / 18.0) * g[2][2][1];
    uby += px * pz * g[2][1][2];
    pxb += uy * pz * g[2][1][2];
    pzb += uy * px * g[2][1][2];
    Fby += (R)(1.0 / 18.0) * g[2][1][2];
    ubz += px * py * g[1][2][2];
    pxb += uz * py * g[1][2][2];
    pyb += uz * px * g[1][2][2];
    Fbz += (R)(1.0 / 18.0) * g[1][2][2];
    // order 6
    drb += (R)(1.0 / 27.0) * g[2][2][2];
    x2b -= ((y2 + z2) * third + ninth + y2 * z2) * g[2][2][2];
    y2b -= ((x2 + z2) * third + ninth + x2 * z2) * g[2][2][2];
    z2b -= ((x2 + y2) * third + ninth + x2 * y2) * g[2][2][2];
    // p = 1/3 + u^2, u^2
    x2b += pxb;
    y2b += pyb;
    z2b += pzb;
    ubx += (R)2 * ux * x2b;
    uby += (R)2 * uy * y2b;
    ubz += (R)2 * uz * z2b;
    // central moments of orders 1-2 from the raw moments
    R m000b = 0, m100b = 0, m010b = 0, m001b = 0, m200b = 0, m020b = 0, m002b = 0, m110b = 0, m101b = 0, m011b = 0;
    // k110 = m110 - ux m010 - uy k100, k101 = m101 - ux m001 - uz k100, k011 = m011 - uy m001 - uz k010
    m110b += k110b;
    ubx -= L.m010 * k110b;
    m010b -= ux * k110b;
    uby -= k100 * k110b;
    k100b -= uy * k110b;
    m101b += k101b;
    ubx -= L.m001 * k101b;
    m001b -= ux * k101b;
    ubz -= k100 * k101b;
    k100b -= uz * k101b;
    m011b += k011b;
    uby -= L.m001 * k011b;
    m001b -= uy * k011b;
    ubz -= k010 * k011b;
    k010b -= uz * k011b;
    // k200 = m200 - ux (m100 + k100), likewise y and z
    m200b += k200b;
    ubx -= (L.m100 + k100) * k200b;
    m100b -= ux * k200b;
    k100b -= ux * k200b;
    m020b += k020b;
    uby -= (L.m010 + k010) * k020b;
    m010b -= uy * k020b;
    k010b -= uy * k020b;
    m002b += k002b;
    ubz -= (L.m001 + k001) * k002b;
    m001b -= uz * k002b;
    k001b -= uz * k002b;
    // k100 = m100 - ux drho, likewise y and z
    m100b += k100b;
    ubx -= drho * k100b;
    drb -= ux * k100b;
    m010b += k010b;
    uby -= drho * k010b;
    drb -= uy * k010b;
    m001b += k001b;
    ubz -= drho * k001b;
    drb -= uz * k001b;
    // u = (j + F/2) / (1 + drho)
    m100b += ubx * inv;
    m010b += uby * inv;
    m001b += ubz * inv;
    Fbx += (R)0.5 * ubx * inv;
    Fby += (R)0.5 * uby * inv;
    Fbz += (R)0.5 * ubz * inv;
    drb -= (ubx * ux + uby * uy + ubz * uz) * inv;
    m000b += drb;
    // raw moments of orders 0-2 transposed: g_i = sum of c_i^(a,b,c) times the moment adjoints
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const R cx = (R)CX[i], cy = (R)CY[i], cz = (R)CZ[i];
        g[CZ[i] + 1][CY[i] + 1][CX[i] + 1] = m000b + cx * m100b + cy * m010b + cz * m001b + cx * cx * m200b +
                                             cy * cy * m020b + cz * cz * m002b + cx * cy * m110b + cx * cz * m101b +
                                             cy * cz * m011b;
    }
}

}  // namespace lbm
