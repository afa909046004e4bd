/*
 * lbm_oracle.c -- plain, slow FP64 CPU oracle for one time step of the D3Q27
 * central-moment MRT lattice Boltzmann method with immersed-boundary (IB)
 * coupling, as described in Chen, Li, Fan, Liu, "GPU Optimization for
 * High-Quality Kinetic Fluid Simulation" (arXiv:2101.11856).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is loaded by the test-suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  The product
 * library never includes, links or calls it, and it shares no code with the
 * HIP kernels.
 *
 * What it follows (section / equation / algorithm of the paper):
 *   Sec. 3, Eq. (1)   LBE update: f_i(x+c_i, t+1) - f_i(x,t) = Omega_i + G_i
 *   Sec. 3, Eq. (2)   rho = sum_i f_i, u = (1/rho) sum_i c_i f_i
 *   Sec. 3, Eq. (3)   streaming (pull): f*_i(x) = f_i(x - c_i)
 *   Sec. 3, Eq. (4)   collision with force: f(t+1) = f* + Omega + G
 *   Sec. 3, Eq. (5)   Omega = -M^{-1} D (m - m_eq), M a 27x27 moment matrix
 *   Sec. 3.1, Eq. (6) IB interpolation of u at a solid sample
 *   Sec. 3.1, Eq. (7) IB penalty force g_s = rho (u_b - u(x_s))
 *   Sec. 3.1, Eq. (8) IB spreading to fluid nodes (here in the literal
 *                     "gathering" form of Sec. 4.3.1 / Table 1)
 *   Alg. 1            bounce-back at a solid (domain) face
 *   Alg. 2            step order: stream, macros + force reset, IB, collide,
 *                     domain faces; total force and torque of the samples
 *   Sec. 4.2.2        solid-sample ordering: l^3 blocks in x-y-z order, Z-order
 *                     (Morton) inside a block
 *
 * Where the paper is silent the oracle takes these readings (the same ones the
 * GPU library documents in its header):
 *   - lattice: c_i in {-1,0,1}^3; index 0 rest, 1-6 faces, 7-18 edges
 *     (xy, xz, yz planes), 19-26 corners; inside each group the sign
 *     patterns run with x fastest, so c_26 = (-1,-1,-1).  This order
 *     reproduces the coefficients printed in the expression for Omega_26
 *     (Sec. 4.4.2) and the Omega_13 / Omega_14 rows of Table 2.
 *   - moments: central moments kappa_abc = sum_i prod_a (c_ia - u_a)^e_a f_i
 *     with exponents in {0,1,2}; the paper's basis M = C T(u) combines them
 *     (order 2: xy, xz, yz, xx-yy, xx-zz, trace; order 3: sums and
 *     differences of the (1,2,0) family; order 4: sum, partial sum and a
 *     difference of the (2,2,0) family).  Inside one relaxation group the
 *     combination does not change the result; it matters only for the
 *     order-2 split between shear rate s_nu and bulk rate s_b.
 *   - m_eq: the central moments of a Maxwellian, rho * cs^(a+b+c) for
 *     exponents all even, else 0 (cs^2 = 1/3).
 *   - rates: s_nu = 1 / (3 nu + 1/2); bulk s_b and orders 3..6 are inputs
 *     (the adaptive high-order law of the paper's Sec. 3 lives in a
 *     supplementary document that is not available: parity unpinned for it).
 *   - force: Guo-type forcing written in moment space: velocity
 *     u = (j + F/2)/rho and G = M^{-1} (I - D/2) m_F, where m_F are the
 *     central moments of the continuous forcing term.
 *   - IB kernel: tensor-product hat function (trilinear, 2x2x2 nodes), marker
 *     base cell b = floor(x_s) taken in FP32, rho at the sample interpolated
 *     with the same kernel, per-sample gain gamma_s and area a_s
 *     (g_s = gamma_s rho_s (u_b - u_s), spread a_s K g_s).
 *   - comparison collision models (Sec. 5.1, the collision-cost figure): the
 *     paper compares D3Q27 BGK and raw-moment MRT (RM-MRT) with its model but
 *     prints neither; both are taken with the same product-form equilibrium,
 *     half-force velocity and Guo forcing as the central-moment model, so the
 *     three differ only in the space where relaxation happens.  BGK relaxes
 *     every population at one rate omega = s_nu; RM-MRT relaxes the moments
 *     of the same combination basis C taken about zero velocity, M0 = C T(0),
 *     at the same per-group rates.
 *   - faces: no-slip = halfway bounce-back (Alg. 1); inlet = bounce-back with
 *     a wall velocity term 2 w_i rho_w (c_i.u_in)/cs^2, rho_w = 1; outflow =
 *     copy of the streamed value one node inward; free-slip = specular
 *     reflection of the normal component.  Precedence where a source crosses
 *     several faces: no-slip > inlet > outflow > free-slip > periodic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27
#define CS2 (1.0 / 3.0)

enum { F_PERIODIC = 0, F_NOSLIP = 1, F_FREESLIP = 2, F_INLET = 3, F_OUTFLOW = 4 };

/* ------------------------------------------------------------------------ */
/* Lattice (Fig. 1; velocity values from the readings above)                */
/* ------------------------------------------------------------------------ */

static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, 1, 0},  {1, -1, 0},  {-1, -1, 0},
    {1, 0, 1},   {-1, 0, 1},  {1, 0, -1},  {-1, 0, -1},
    {0, 1, 1},   {0, -1, 1},  {0, 1, -1},  {0, -1, -1},
    {1, 1, 1},   {-1, 1, 1},  {1, -1, 1},  {-1, -1, 1},
    {1, 1, -1},  {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};

/* exponent triples of the central moments, grouped by total order */
static const int EXPO[Q][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2},
    {1, 2, 0}, {1, 0, 2}, {2, 1, 0}, {0, 1, 2}, {2, 0, 1}, {0, 2, 1}, {1, 1, 1},
    {2, 2, 0}, {2, 0, 2}, {0, 2, 2}, {2, 1, 1}, {1, 2, 1}, {1, 1, 2},
    {1, 2, 2}, {2, 1, 2}, {2, 2, 1},
    {2, 2, 2}};

static int vel_index(int cx, int cy, int cz)
{
    for (int i = 0; i < Q; ++i)
        if (CV[i][0] == cx && CV[i][1] == cy && CV[i][2] == cz) return i;
    return -1;
}

static int opposite(int i) { return vel_index(-CV[i][0], -CV[i][1], -CV[i][2]); }

/* lattice weights: the u = 0 value of the product-form equilibrium */
static double weight(int i)
{
    double w = 1.0;
    for (int a = 0; a < 3; ++a) w *= (CV[i][a] == 0) ? 2.0 / 3.0 : 1.0 / 6.0;
    return w;
}

static int expo_index(int a, int b, int c)
{
    for (int k = 0; k < Q; ++k)
        if (EXPO[k][0] == a && EXPO[k][1] == b && EXPO[k][2] == c) return k;
    return -1;
}

void orc_lattice(int *c, double *w, int *opp, int *expo)
{
    for (int i = 0; i < Q; ++i) {
        for (int a = 0; a < 3; ++a) {
            if (c) c[3 * i + a] = CV[i][a];
            if (expo) expo[3 * i + a] = EXPO[i][a];
        }
        if (w) w[i] = weight(i);
        if (opp) opp[i] = opposite(i);
    }
}

/* ------------------------------------------------------------------------ */
/* Moment matrices (Eq. 5)                                                   */
/* ------------------------------------------------------------------------ */

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

/* T(u)[k][i] = prod_a (c_ia - u_a)^{e_ka}: raw central-moment matrix. */
void orc_central_matrix(const double u[3], double *T)
{
    for (int k = 0; k < Q; ++k)
        for (int i = 0; i < Q; ++i) {
            double v = 1.0;
            for (int a = 0; a < 3; ++a) v *= ipow((double)CV[i][a] - u[a], EXPO[k][a]);
            T[k * Q + i] = v;
        }
}

/* C: the paper's combination of central moments (row k of the basis). */
void orc_combination_matrix(double *C)
{
    memset(C, 0, sizeof(double) * Q * Q);
    for (int k = 0; k < Q; ++k) C[k * Q + k] = 1.0;
    const int k200 = expo_index(2, 0, 0), k020 = expo_index(0, 2, 0), k002 = expo_index(0, 0, 2);
    const int k120 = expo_index(1, 2, 0), k102 = expo_index(1, 0, 2), k210 = expo_index(2, 1, 0);
    const int k012 = expo_index(0, 1, 2), k201 = expo_index(2, 0, 1), k021 = expo_index(0, 2, 1);
    const int k220 = expo_index(2, 2, 0), k202 = expo_index(2, 0, 2), k022 = expo_index(0, 2, 2);
    /* rows 7..9: xx - yy, xx - zz, trace */
    for (int r = 7; r <= 9; ++r) memset(C + r * Q, 0, sizeof(double) * Q);
    C[7 * Q + k200] = 1.0;  C[7 * Q + k020] = -1.0;
    C[8 * Q + k200] = 1.0;  C[8 * Q + k002] = -1.0;
    C[9 * Q + k200] = 1.0;  C[9 * Q + k020] = 1.0;  C[9 * Q + k002] = 1.0;
    /* rows 10..15: sums then differences of the third-order pairs */
    for (int r = 10; r <= 15; ++r) memset(C + r * Q, 0, sizeof(double) * Q);
    C[10 * Q + k120] = 1.0; C[10 * Q + k102] = 1.0;
    C[11 * Q + k201] = 1.0; C[11 * Q + k021] = 1.0;
    C[12 * Q + k210] = 1.0; C[12 * Q + k012] = 1.0;
    C[13 * Q + k120] = 1.0; C[13 * Q + k102] = -1.0;
    C[14 * Q + k201] = 1.0; C[14 * Q + k021] = -1.0;
    C[15 * Q + k210] = 1.0; C[15 * Q + k012] = -1.0;
    /* rows 17..19: fourth-order diagonal family */
    for (int r = 17; r <= 19; ++r) memset(C + r * Q, 0, sizeof(double) * Q);
    C[17 * Q + k220] = 1.0; C[17 * Q + k202] = 1.0; C[17 * Q + k022] = 1.0;
    C[18 * Q + k220] = 1.0; C[18 * Q + k202] = 1.0; C[18 * Q + k022] = -2.0;
    C[19 * Q + k220] = 1.0; C[19 * Q + k202] = -1.0;
}

static void matmul(const double *A, const double *B, double *R)
{
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) {
            double s = 0.0;
            for (int k = 0; k < Q; ++k) s += A[r * Q + k] * B[k * Q + c];
            R[r * Q + c] = s;
        }
}

/* M(u) = C T(u): the moment-space projection of Eq. (5). */
void orc_basis_matrix(const double u[3], double *M)
{
    double T[Q * Q], C[Q * Q];
    orc_central_matrix(u, T);
    orc_combination_matrix(C);
    matmul(C, T, M);
}

/* Solve A x = b (n x n, row-major) by Gaussian elimination with partial
 * pivoting.  A and b are overwritten.  Returns 0, or -1 if singular. */
static int gauss_solve(double *A, double *b, int n)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        double best = fabs(A[col * n + col]);
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r * n + col]) > best) { best = fabs(A[r * n + col]); piv = r; }
        if (best == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                double t = A[col * n + c]; A[col * n + c] = A[piv * n + c]; A[piv * n + c] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = A[r * n + col] / A[col * n + col];
            if (f == 0.0) continue;
            for (int c = col; c < n; ++c) A[r * n + c] -= f * A[col * n + c];
            b[r] -= f * b[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= A[r * n + c] * b[c];
        b[r] = s / A[r * n + r];
    }
    return 0;
}

/* Inverse of an n x n matrix column by column (used by the tests). */
int orc_inverse(const double *A, double *Ainv, int n)
{
    double *W = (double *)malloc(sizeof(double) * n * n);
    double *e = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    for (int c = 0; c < n && rc == 0; ++c) {
        memcpy(W, A, sizeof(double) * n * n);
        for (int r = 0; r < n; ++r) e[r] = (r == c) ? 1.0 : 0.0;
        rc = gauss_solve(W, e, n);
        for (int r = 0; r < n; ++r) Ainv[r * n + c] = e[r];
    }
    free(W);
    free(e);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium and collision (Eqs. 2, 4, 5)                                  */
/* ------------------------------------------------------------------------ */

/* Product-form discrete equilibrium: f_i = rho prod_a phi_{c_ia}(u_a),
 * phi_0(u) = 2/3 - u^2, phi_{+-1}(u) = (1/3 +- u + u^2)/2.  Its central
 * moments are exactly those of the Maxwellian (checked by the tests). */
void orc_equilibrium(double rho, const double u[3], double *feq)
{
    for (int i = 0; i < Q; ++i) {
        double v = rho;
        for (int a = 0; a < 3; ++a) {
            const double ua = u[a];
            if (CV[i][a] == 0) v *= 2.0 / 3.0 - ua * ua;
            else v *= (1.0 / 3.0 + CV[i][a] * ua + ua * ua) * 0.5;
        }
        feq[i] = v;
    }
}

/* Maxwellian central moment of exponent triple e (density rho). */
static double kappa_eq(double rho, const int e[3])
{
    double v = rho;
    for (int a = 0; a < 3; ++a) {
        if (e[a] == 1) return 0.0;
        if (e[a] == 2) v *= CS2;
    }
    return v;
}

/* Central moment of the continuous Guo forcing term F.(xi-u)/cs^2 f_M/rho:
 * F_a cs^(2 * number of 2-exponents) when exactly one exponent is 1 (axis a)
 * and the others are 0 or 2; zero otherwise. */
static double kappa_force(const double F[3], const int e[3])
{
    int ones = 0, axis = -1, twos = 0;
    for (int a = 0; a < 3; ++a) {
        if (e[a] == 1) { ones++; axis = a; }
        if (e[a] == 2) twos++;
    }
    if (ones != 1) return 0.0;
    return F[axis] * ipow(CS2, twos);
}

/* Diagonal of D for basis row k: rates by order; the order-2 trace row uses
 * the bulk rate.  Orders 0 and 1 are conserved (rate 0). */
static double rate_of(int k, double s_nu, double s_b, const double s_high[4])
{
    const int order = EXPO[k][0] + EXPO[k][1] + EXPO[k][2];
    if (order <= 1) return 0.0;
    if (order == 2) return (k == 9) ? s_b : s_nu;
    return s_high[order - 3];
}

/* One cell of Eqs. (4)-(5): fpost = fs + Omega + G, in the moment basis
 * M = C T(u), with u the half-force velocity (j + F/2)/rho. */
int orc_collide(const double *fs, const double F[3], double s_nu, double s_b, const double s_high[4],
                double *fpost)
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += fs[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * fs[i];
    }
    double u[3];
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;

    double M[Q * Q], C[Q * Q];
    orc_basis_matrix(u, M);
    orc_combination_matrix(C);

    double m[Q], keq[Q], kF[Q], meq[Q], mF[Q], mp[Q];
    for (int k = 0; k < Q; ++k) {
        double s = 0.0;
        for (int i = 0; i < Q; ++i) s += M[k * Q + i] * fs[i];
        m[k] = s;
        keq[k] = kappa_eq(rho, EXPO[k]);
        kF[k] = kappa_force(F, EXPO[k]);
    }
    for (int k = 0; k < Q; ++k) {
        double se = 0.0, sf = 0.0;
        for (int l = 0; l < Q; ++l) {
            se += C[k * Q + l] * keq[l];
            sf += C[k * Q + l] * kF[l];
        }
        meq[k] = se;
        mF[k] = sf;
    }
    for (int k = 0; k < Q; ++k) {
        const double s = rate_of(k, s_nu, s_b, s_high);
        mp[k] = m[k] - s * (m[k] - meq[k]) + (1.0 - 0.5 * s) * mF[k];
    }
    int rc = gauss_solve(M, mp, Q);
    for (int i = 0; i < Q; ++i) fpost[i] = mp[i];
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Comparison collision models (Sec. 5.1): BGK and raw-moment MRT            */
/* ------------------------------------------------------------------------ */

/* Guo forcing shape of the product-form equilibrium: G_i = sum_a F_a
 * d Phi_i / d u_a with Phi_i(u) = prod_a phi_{c_ia}(u_a) (so f_eq = rho Phi),
 * phi_0 = 2/3 - u^2 (derivative -2u), phi_{+-1} = (1/3 +- u + u^2)/2
 * (derivative (+-1 + 2u)/2). */
void orc_forcing_shape(const double u[3], const double F[3], double *G)
{
    for (int i = 0; i < Q; ++i) {
        double phi[3], dphi[3];
        for (int a = 0; a < 3; ++a) {
            const double ua = u[a];
            if (CV[i][a] == 0) {
                phi[a] = 2.0 / 3.0 - ua * ua;
                dphi[a] = -2.0 * ua;
            } else {
                phi[a] = (1.0 / 3.0 + CV[i][a] * ua + ua * ua) * 0.5;
                dphi[a] = (CV[i][a] + 2.0 * ua) * 0.5;
            }
        }
        G[i] = F[0] * dphi[0] * phi[1] * phi[2] + F[1] * phi[0] * dphi[1] * phi[2] + F[2] * phi[0] * phi[1] * dphi[2];
    }
}

/* density, momentum and half-force velocity of pulled populations */
static double half_force_velocity(const double *fs, const double F[3], double u[3])
{
    double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < Q; ++i) {
        rho += fs[i];
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * fs[i];
    }
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + F[a] / 2.0) / rho;
    return rho;
}

/* Lattice BGK: one relaxation rate for every population,
 * fpost = fs - omega (fs - f_eq(rho, u)) + (1 - omega/2) G. */
int orc_collide_bgk(const double *fs, const double F[3], double omega, double *fpost)
{
    double u[3], feq[Q], G[Q];
    const double rho = half_force_velocity(fs, F, u);
    orc_equilibrium(rho, u, feq);
    orc_forcing_shape(u, F, G);
    for (int i = 0; i < Q; ++i) fpost[i] = fs[i] - omega * (fs[i] - feq[i]) + (1.0 - 0.5 * omega) * G[i];
    return 0;
}

/* Raw-moment MRT in the basis M0 = C T(0): m = M0 fs, m_eq = M0 f_eq(rho, u),
 * m_F = M0 G; m' = m - D (m - m_eq) + (I - D/2) m_F with the per-group rates
 * of the central-moment model; fpost solves M0 fpost = m'. */
int orc_collide_rm(const double *fs, const double F[3], double s_nu, double s_b, const double s_high[4],
                   double *fpost)
{
    double u[3], feq[Q], G[Q];
    const double rho = half_force_velocity(fs, F, u);
    orc_equilibrium(rho, u, feq);
    orc_forcing_shape(u, F, G);
    const double zero[3] = {0.0, 0.0, 0.0};
    double M0[Q * Q];
    orc_basis_matrix(zero, M0);
    double mp[Q];
    for (int k = 0; k < Q; ++k) {
        double m = 0.0, me = 0.0, mf = 0.0;
        for (int i = 0; i < Q; ++i) {
            m += M0[k * Q + i] * fs[i];
            me += M0[k * Q + i] * feq[i];
            mf += M0[k * Q + i] * G[i];
        }
        const double s = rate_of(k, s_nu, s_b, s_high);
        mp[k] = m - s * (m - me) + (1.0 - 0.5 * s) * mf;
    }
    const int rc = gauss_solve(M0, mp, Q);
    for (int i = 0; i < Q; ++i) fpost[i] = mp[i];
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Simulation state                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n[3];
    int64_t N;
    double nu, s_nu, s_b, s_high[4];
    int face[6];
    double u_in[3];
    double *inlet; /* optional [3][nz][ny] */
    double body[3];
    double *f, *fs;      /* [27][N] state and streamed state */
    double *rho, *u0, *g; /* [N], [3][N], [3][N] */
    /* markers */
    int64_t nm;
    float *mx;           /* [3][nm] positions as given (FP32) */
    double *ub, *area, *gain; /* [3][nm], [nm], [nm] */
    int32_t *base;       /* [3][nm] floor of the position */
    int64_t *bucket_start; /* [N+1] markers by base cell, ascending index */
    int64_t *bucket;
    double *Gs;          /* [3][nm] last penalty forces */
    double ftot[3];
    /* collision model: 0 central-moment MRT, 1 BGK, 2 raw-moment MRT */
    int model;
    /* passive scalar (optional) */
    int scalar, scalar_inlet_height;
    double *sc, *sc2;
} orc_sim;

static inline int64_t lin(const orc_sim *S, int x, int y, int z)
{
    return (int64_t)x + (int64_t)S->n[0] * ((int64_t)y + (int64_t)S->n[1] * z);
}

static int face_rank(int f)
{
    switch (f) {
    case F_NOSLIP: return 4;
    case F_INLET: return 3;
    case F_OUTFLOW: return 2;
    case F_FREESLIP: return 1;
    default: return 0;
    }
}

orc_sim *orc_create(int nx, int ny, int nz, double nu, const int *face, const double *u_in,
                    double s_b, const double *s_high, const double *body, int scalar)
{
    if (nx < 1 || ny < 1 || nz < 1 || !(nu > 0.0)) return NULL;
    orc_sim *S = (orc_sim *)calloc(1, sizeof(orc_sim));
    S->n[0] = nx; S->n[1] = ny; S->n[2] = nz;
    S->N = (int64_t)nx * ny * nz;
    S->nu = nu;
    S->s_nu = 1.0 / (3.0 * nu + 0.5);
    S->s_b = s_b;
    for (int k = 0; k < 4; ++k) S->s_high[k] = s_high ? s_high[k] : 1.0;
    for (int k = 0; k < 6; ++k) S->face[k] = face ? face[k] : F_PERIODIC;
    for (int a = 0; a < 3; ++a) {
        S->u_in[a] = u_in ? u_in[a] : 0.0;
        S->body[a] = body ? body[a] : 0.0;
    }
    const int64_t N = S->N;
    S->f = (double *)calloc((size_t)(Q * N), sizeof(double));
    S->fs = (double *)calloc((size_t)(Q * N), sizeof(double));
    S->rho = (double *)calloc((size_t)N, sizeof(double));
    S->u0 = (double *)calloc((size_t)(3 * N), sizeof(double));
    S->g = (double *)calloc((size_t)(3 * N), sizeof(double));
    S->scalar = scalar;
    if (scalar) {
        S->sc = (double *)calloc((size_t)N, sizeof(double));
        S->sc2 = (double *)calloc((size_t)N, sizeof(double));
    }
    if (!S->f || !S->fs || !S->rho || !S->u0 || !S->g) return NULL;
    return S;
}

static void free_markers(orc_sim *S)
{
    free(S->mx); free(S->ub); free(S->area); free(S->gain); free(S->base);
    free(S->bucket_start); free(S->bucket); free(S->Gs);
    S->mx = NULL; S->ub = S->area = S->gain = S->Gs = NULL; S->base = NULL;
    S->bucket_start = S->bucket = NULL;
    S->nm = 0;
}

void orc_destroy(orc_sim *S)
{
    if (!S) return;
    free(S->f); free(S->fs); free(S->rho); free(S->u0); free(S->g);
    free(S->inlet); free(S->sc); free(S->sc2);
    free_markers(S);
    free(S);
}

int64_t orc_num_cells(const orc_sim *S) { return S->N; }

/* collision model of the steps: 0 central-moment MRT (default), 1 BGK at
 * rate s_nu, 2 raw-moment MRT; returns -1 for an unknown code */
int orc_set_model(orc_sim *S, int model)
{
    if (model < 0 || model > 2) return -1;
    S->model = model;
    return 0;
}

void orc_set_state(orc_sim *S, const double *f) { memcpy(S->f, f, sizeof(double) * Q * S->N); }
void orc_get_state(const orc_sim *S, double *f) { memcpy(f, S->f, sizeof(double) * Q * S->N); }

void orc_set_inlet_profile(orc_sim *S, const double *prof)
{
    free(S->inlet);
    S->inlet = NULL;
    if (prof) {
        const size_t n = (size_t)3 * S->n[1] * S->n[2];
        S->inlet = (double *)malloc(sizeof(double) * n);
        memcpy(S->inlet, prof, sizeof(double) * n);
    }
}

void orc_init_equilibrium(orc_sim *S, const double *rho, const double *u)
{
    const int64_t N = S->N;
    for (int64_t k = 0; k < N; ++k) {
        double uu[3] = {u[k], u[N + k], u[2 * N + k]}, feq[Q];
        orc_equilibrium(rho[k], uu, feq);
        for (int i = 0; i < Q; ++i) S->f[i * N + k] = feq[i];
    }
}

/* ------------------------------------------------------------------------ */
/* Streaming with domain faces (Eq. 3, Alg. 1)                                */
/* ------------------------------------------------------------------------ */

static double inlet_velocity(const orc_sim *S, int a, int y, int z)
{
    if (S->inlet) return S->inlet[((int64_t)a * S->n[2] + z) * S->n[1] + y];
    return S->u_in[a];
}

/* f*_i at node p, pulled from state f, with the face rules of the readings. */
static double pull_one(const orc_sim *S, const double *f, int i, int px, int py, int pz)
{
    const int p[3] = {px, py, pz};
    int src[3], crossed[3] = {0, 0, 0};
    int best = F_PERIODIC, bestrank = 0, bestaxis = -1, bestside = 0;
    for (int a = 0; a < 3; ++a) {
        src[a] = p[a] - CV[i][a];
        int side;
        if (src[a] < 0) side = 0;
        else if (src[a] >= S->n[a]) side = 1;
        else continue;
        const int fc = S->face[2 * a + side];
        if (fc == F_PERIODIC) {
            src[a] = ((src[a] % S->n[a]) + S->n[a]) % S->n[a];
            continue;
        }
        crossed[a] = 1;
        if (face_rank(fc) > bestrank) {
            bestrank = face_rank(fc);
            best = fc;
            bestaxis = a;
            bestside = side;
        }
    }
    const int64_t N = S->N;
    switch (best) {
    case F_PERIODIC:
        return f[i * N + lin(S, src[0], src[1], src[2])];
    case F_NOSLIP:
        return f[opposite(i) * N + lin(S, px, py, pz)];
    case F_INLET: {
        double cu = 0.0;
        for (int a = 0; a < 3; ++a) cu += CV[i][a] * inlet_velocity(S, a, py, pz);
        return f[opposite(i) * N + lin(S, px, py, pz)] + 2.0 * weight(i) * cu / CS2;
    }
    case F_OUTFLOW: {
        int q[3] = {px, py, pz};
        q[bestaxis] += bestside ? -1 : 1;
        return pull_one(S, f, i, q[0], q[1], q[2]);
    }
    case F_FREESLIP: {
        int cr[3] = {CV[i][0], CV[i][1], CV[i][2]};
        for (int a = 0; a < 3; ++a)
            if (crossed[a]) {
                cr[a] = -cr[a];
                src[a] = p[a];
            }
        return f[vel_index(cr[0], cr[1], cr[2]) * N + lin(S, src[0], src[1], src[2])];
    }
    }
    return 0.0;
}

static void stream_all(orc_sim *S, const double *f, double *fs)
{
    const int nx = S->n[0], ny = S->n[1], nz = S->n[2];
    const int64_t N = S->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t k = lin(S, x, y, z);
                for (int i = 0; i < Q; ++i) fs[i * N + k] = pull_one(S, f, i, x, y, z);
            }
}

/* Eq. (2) on the streamed populations: rho and u0 = j / rho. */
static void macros_all(orc_sim *S, const double *fs)
{
    const int64_t N = S->N;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        for (int i = 0; i < Q; ++i) {
            const double v = fs[i * N + k];
            rho += v;
            for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * v;
        }
        S->rho[k] = rho;
        for (int a = 0; a < 3; ++a) S->u0[a * N + k] = j[a] / rho;
    }
}

/* ------------------------------------------------------------------------ */
/* Immersed boundary (Eqs. 6-8)                                              */
/* ------------------------------------------------------------------------ */

/* Validation shared by the set-up: positions finite, inside the domain, and
 * the 2x2x2 stencil inside any non-periodic axis.  Returns index of the
 * first bad marker, or -1. */
int64_t orc_check_markers(const orc_sim *S, int64_t n, const float *xyz)
{
    for (int64_t s = 0; s < n; ++s)
        for (int a = 0; a < 3; ++a) {
            const float v = xyz[a * n + s];
            const int periodic = S->face[2 * a] == F_PERIODIC;
            const float hi = periodic ? (float)S->n[a] : (float)(S->n[a] - 1);
            if (!(v >= 0.0f) || !(v < hi)) return s;
        }
    return -1;
}

int orc_set_markers(orc_sim *S, int64_t n, const float *xyz, const double *ub, const double *area,
                    const double *gain)
{
    free_markers(S);
    if (n <= 0) return 0;
    if (orc_check_markers(S, n, xyz) >= 0) return -1;
    S->nm = n;
    S->mx = (float *)malloc(sizeof(float) * 3 * n);
    memcpy(S->mx, xyz, sizeof(float) * 3 * n);
    S->ub = (double *)malloc(sizeof(double) * 3 * n);
    S->area = (double *)malloc(sizeof(double) * n);
    S->gain = (double *)malloc(sizeof(double) * n);
    S->Gs = (double *)calloc((size_t)(3 * n), sizeof(double));
    S->base = (int32_t *)malloc(sizeof(int32_t) * 3 * n);
    for (int64_t s = 0; s < n; ++s) {
        for (int a = 0; a < 3; ++a) {
            S->ub[a * n + s] = ub ? ub[a * n + s] : 0.0;
            S->base[a * n + s] = (int32_t)floorf(xyz[a * n + s]);
        }
        S->area[s] = area ? area[s] : 1.0;
        S->gain[s] = gain ? gain[s] : 1.0;
    }
    /* buckets of markers by base cell, each in ascending marker index */
    const int64_t N = S->N;
    S->bucket_start = (int64_t *)calloc((size_t)(N + 1), sizeof(int64_t));
    S->bucket = (int64_t *)malloc(sizeof(int64_t) * n);
    for (int64_t s = 0; s < n; ++s)
        S->bucket_start[lin(S, S->base[s], S->base[n + s], S->base[2 * n + s]) + 1]++;
    for (int64_t k = 0; k < N; ++k) S->bucket_start[k + 1] += S->bucket_start[k];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * N);
    memcpy(fill, S->bucket_start, sizeof(int64_t) * N);
    for (int64_t s = 0; s < n; ++s) {
        const int64_t b = lin(S, S->base[s], S->base[n + s], S->base[2 * n + s]);
        S->bucket[fill[b]++] = s;
    }
    free(fill);
    return 0;
}

/* kernel weight of marker s at stencil offset d (0/1 per axis): trilinear */
static double marker_weight(const orc_sim *S, int64_t s, const int d[3])
{
    const int64_t n = S->nm;
    double K = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double t = (double)S->mx[a * n + s] - (double)S->base[a * n + s];
        K *= d[a] ? t : 1.0 - t;
    }
    return K;
}

static int64_t stencil_node(const orc_sim *S, int64_t s, const int d[3])
{
    const int64_t n = S->nm;
    int q[3];
    for (int a = 0; a < 3; ++a) q[a] = (S->base[a * n + s] + d[a]) % S->n[a];
    return lin(S, q[0], q[1], q[2]);
}

/* Eqs. (6)-(7): interpolate rho and u0, penalty force per marker. */
static void ib_penalty(orc_sim *S)
{
    const int64_t n = S->nm, N = S->N;
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n; ++s) {
        double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    const int d[3] = {dx, dy, dz};
                    const double K = marker_weight(S, s, d);
                    const int64_t k = stencil_node(S, s, d);
                    rs += K * S->rho[k];
                    for (int a = 0; a < 3; ++a) us[a] += K * S->u0[a * N + k];
                }
        for (int a = 0; a < 3; ++a) S->Gs[a * n + s] = S->gain[s] * rs * (S->ub[a * n + s] - us[a]);
    }
}

static int cmp_i64(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Eq. (8) in gathering form: each fluid node sums, over the samples whose
 * 2x2x2 neighbourhood contains it, a_s K g_s, in ascending sample index. */
static void ib_gather(orc_sim *S)
{
    const int nx = S->n[0], ny = S->n[1], nz = S->n[2];
    const int64_t n = S->nm, N = S->N;
    memset(S->g, 0, sizeof(double) * 3 * N);
#pragma omp parallel
    {
        int64_t cap = 64, *ids = (int64_t *)malloc(sizeof(int64_t) * cap);
#pragma omp for schedule(dynamic, 1)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    int64_t cnt = 0;
                    const int p[3] = {x, y, z};
                    for (int dz = 0; dz < 2; ++dz)
                        for (int dy = 0; dy < 2; ++dy)
                            for (int dx = 0; dx < 2; ++dx) {
                                const int d[3] = {dx, dy, dz};
                                int b[3], ok = 1;
                                for (int a = 0; a < 3; ++a) {
                                    b[a] = p[a] - d[a];
                                    if (b[a] < 0) {
                                        if (S->face[2 * a] == F_PERIODIC) b[a] += S->n[a];
                                        else ok = 0;
                                    }
                                }
                                if (!ok) continue;
                                const int64_t bk = lin(S, b[0], b[1], b[2]);
                                for (int64_t t = S->bucket_start[bk]; t < S->bucket_start[bk + 1]; ++t) {
                                    if (cnt == cap) {
                                        cap *= 2;
                                        ids = (int64_t *)realloc(ids, sizeof(int64_t) * cap);
                                    }
                                    /* pack (marker, offset) so sorting by marker keeps offsets */
                                    ids[cnt] = S->bucket[t] * 8 + (dx + 2 * dy + 4 * dz);
                                    cnt++;
                                }
                            }
                    if (cnt == 0) continue;
                    qsort(ids, (size_t)cnt, sizeof(int64_t), cmp_i64);
                    const int64_t k = lin(S, x, y, z);
                    double acc[3] = {0.0, 0.0, 0.0};
                    for (int64_t t = 0; t < cnt; ++t) {
                        const int64_t s = ids[t] / 8;
                        const int code = (int)(ids[t] % 8);
                        const int d[3] = {code & 1, (code >> 1) & 1, (code >> 2) & 1};
                        const double K = marker_weight(S, s, d);
                        for (int a = 0; a < 3; ++a) acc[a] += S->area[s] * K * S->Gs[a * n + s];
                    }
                    for (int a = 0; a < 3; ++a) S->g[a * N + k] = acc[a];
                }
        free(ids);
    }
    for (int a = 0; a < 3; ++a) {
        double t = 0.0;
        for (int64_t s = 0; s < n; ++s) t += S->area[s] * S->Gs[a * n + s];
        S->ftot[a] = t;
    }
}

/* ------------------------------------------------------------------------ */
/* Passive scalar: first-order upwind advection by the collision velocity,   */
/* held at 1 on inlet nodes below a height, zero-gradient at other faces.    */
/* ------------------------------------------------------------------------ */

void orc_set_scalar(orc_sim *S, const double *s, int inlet_height)
{
    if (!S->scalar) return;
    memcpy(S->sc, s, sizeof(double) * S->N);
    S->scalar_inlet_height = inlet_height;
}

void orc_get_scalar(const orc_sim *S, double *s)
{
    if (S->scalar) memcpy(s, S->sc, sizeof(double) * S->N);
}

static double scalar_at(const orc_sim *S, const double *sc, int x, int y, int z)
{
    int q[3] = {x, y, z};
    for (int a = 0; a < 3; ++a) {
        if (q[a] < 0 || q[a] >= S->n[a]) {
            if (S->face[2 * a] == F_PERIODIC) q[a] = (q[a] + S->n[a]) % S->n[a];
            else q[a] = q[a] < 0 ? 0 : S->n[a] - 1;
        }
    }
    return sc[lin(S, q[0], q[1], q[2])];
}

/* ------------------------------------------------------------------------ */
/* One time step (Alg. 2)                                                    */
/* ------------------------------------------------------------------------ */

static int collide_all(orc_sim *S)
{
    const int64_t N = S->N;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t k = 0; k < N; ++k) {
        double fs[Q], fp[Q], F[3];
        for (int i = 0; i < Q; ++i) fs[i] = S->fs[i * N + k];
        for (int a = 0; a < 3; ++a) F[a] = S->g[a * N + k] + S->body[a];
        int rc;
        if (S->model == 1) rc = orc_collide_bgk(fs, F, S->s_nu, fp);
        else if (S->model == 2) rc = orc_collide_rm(fs, F, S->s_nu, S->s_b, S->s_high, fp);
        else rc = orc_collide(fs, F, S->s_nu, S->s_b, S->s_high, fp);
        if (rc != 0) bad = 1;
        for (int i = 0; i < Q; ++i) S->f[i * N + k] = fp[i];
    }
    return bad ? -1 : 0;
}

static void scalar_step(orc_sim *S)
{
    const int nx = S->n[0], ny = S->n[1], nz = S->n[2];
    const int64_t N = S->N;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int64_t k = lin(S, x, y, z);
                double u[3];
                for (int a = 0; a < 3; ++a)
                    u[a] = S->u0[a * N + k] + 0.5 * (S->g[a * N + k] + S->body[a]) / S->rho[k];
                const double c = S->sc[k];
                double v = c;
                const int p[3] = {x, y, z};
                for (int a = 0; a < 3; ++a) {
                    int qm[3] = {p[0], p[1], p[2]}, qp[3] = {p[0], p[1], p[2]};
                    qm[a] -= 1;
                    qp[a] += 1;
                    if (u[a] > 0.0) v -= u[a] * (c - scalar_at(S, S->sc, qm[0], qm[1], qm[2]));
                    else v -= u[a] * (scalar_at(S, S->sc, qp[0], qp[1], qp[2]) - c);
                }
                if (x == 0 && S->face[0] == F_INLET && y < S->scalar_inlet_height) v = 1.0;
                S->sc2[k] = v;
            }
    double *t = S->sc;
    S->sc = S->sc2;
    S->sc2 = t;
}

int orc_step(orc_sim *S, int nsteps)
{
    for (int t = 0; t < nsteps; ++t) {
        stream_all(S, S->f, S->fs);           /* (a) streaming + face rules */
        macros_all(S, S->fs);                 /* (b) rho, u; force reset     */
        memset(S->g, 0, sizeof(double) * 3 * S->N);
        if (S->nm > 0) {                      /* (c) IB                       */
            ib_penalty(S);
            ib_gather(S);
        } else {
            S->ftot[0] = S->ftot[1] = S->ftot[2] = 0.0;
        }
        if (S->scalar) scalar_step(S);
        if (collide_all(S) != 0) return -1;   /* (d) collision               */
    }
    return 0;
}

/* Virtual pull of the current state: the rho and u0 = j/rho that step (b) of
 * the next time step would see. */
void orc_macros(orc_sim *S, double *rho, double *u)
{
    stream_all(S, S->f, S->fs);
    macros_all(S, S->fs);
    memcpy(rho, S->rho, sizeof(double) * S->N);
    memcpy(u, S->u0, sizeof(double) * 3 * S->N);
}

/* Total IB force sum_s a_s g_s of the most recent step. */
void orc_last_force(const orc_sim *S, double *out) { memcpy(out, S->ftot, sizeof(double) * 3); }

/* IB force that the next step would apply, evaluated from the current state
 * without changing it. Also writes the per-marker penalty forces (if asked). */
void orc_ib_force(orc_sim *S, double *out, double *gs)
{
    stream_all(S, S->f, S->fs);
    macros_all(S, S->fs);
    const int64_t n = S->nm;
    out[0] = out[1] = out[2] = 0.0;
    if (n == 0) return;
    ib_penalty(S);
    for (int a = 0; a < 3; ++a) {
        double t = 0.0;
        for (int64_t s = 0; s < n; ++s) t += S->area[s] * S->Gs[a * n + s];
        out[a] = t;
    }
    if (gs) memcpy(gs, S->Gs, sizeof(double) * 3 * n);
}

/* Total torque, Alg. 2 (c): sum_s (x_s - o) x (a_s g_s) about the point o,
 * of the penalty forces last computed (by the last step, or by orc_ib_force
 * if that was called after it).  x_s is the stored FP32 position; the lever
 * arm and the sum are FP64, in ascending sample index. */
void orc_last_torque(const orc_sim *S, const double o[3], double *out)
{
    const int64_t n = S->nm;
    double t[3] = {0.0, 0.0, 0.0};
    for (int64_t s = 0; s < n; ++s) {
        const double r[3] = {(double)S->mx[s] - o[0], (double)S->mx[n + s] - o[1], (double)S->mx[2 * n + s] - o[2]};
        const double F[3] = {S->area[s] * S->Gs[s], S->area[s] * S->Gs[n + s], S->area[s] * S->Gs[2 * n + s]};
        t[0] += r[1] * F[2] - r[2] * F[1];
        t[1] += r[2] * F[0] - r[0] * F[2];
        t[2] += r[0] * F[1] - r[1] * F[0];
    }
    memcpy(out, t, sizeof(t));
}

/* Spread field g of the most recent step (for tests). */
void orc_get_force_field(const orc_sim *S, double *g) { memcpy(g, S->g, sizeof(double) * 3 * S->N); }

/* FP64 totals of the stored state: mass and momentum. */
void orc_conserved(const orc_sim *S, double *out)
{
    const int64_t N = S->N;
    double m = 0.0, p[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < N; ++k)
        for (int i = 0; i < Q; ++i) {
            const double v = S->f[i * N + k];
            m += v;
            for (int a = 0; a < 3; ++a) p[a] += CV[i][a] * v;
        }
    out[0] = m;
    out[1] = p[0];
    out[2] = p[1];
    out[3] = p[2];
}

/* ------------------------------------------------------------------------ */
/* Solid-sample maps (Sec. 4.2.2)                                            */
/* ------------------------------------------------------------------------ */

#define ELL 4

typedef struct {
    uint64_t key;
    int64_t idx;
} keyed;

static int cmp_keyed(const void *a, const void *b)
{
    const keyed *x = (const keyed *)a, *y = (const keyed *)b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Sort key of a sample: index of its l^3 block in x-y-z order (x fastest),
 * then the 30-bit Morton code of its position inside the block quantised to
 * 1024 steps per axis (bit 3k from x, 3k+1 from y, 3k+2 from z). */
uint64_t orc_marker_key(const orc_sim *S, const float *p)
{
    const int nb[3] = {(S->n[0] + ELL - 1) / ELL, (S->n[1] + ELL - 1) / ELL, (S->n[2] + ELL - 1) / ELL};
    int B[3];
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const int b = (int)floorf(p[a]);
        B[a] = b / ELL;
        /* (x - l B) * (1024 / l): both operations are exact in FP32 */
        double r = floor(((double)p[a] - (double)(ELL * B[a])) * (1024.0 / ELL));
        if (r < 0) r = 0;
        if (r > 1023) r = 1023;
        q[a] = (uint32_t)r;
    }
    const uint64_t block = (uint64_t)B[0] + (uint64_t)nb[0] * ((uint64_t)B[1] + (uint64_t)nb[1] * B[2]);
    uint64_t morton = 0;
    for (int bit = 0; bit < 10; ++bit)
        for (int a = 0; a < 3; ++a) morton |= (uint64_t)((q[a] >> bit) & 1u) << (3 * bit + a);
    return (block << 30) | morton;
}

/* flags[N]: bit 0 = node in some sample's 2x2x2 neighbourhood (receives IB
 * force), bit 1 = base cell of some sample.  marker_cell[n] = linear index of
 * the base cell.  marker_perm[n] = sample indices in sorted order. */
void orc_maps(const orc_sim *S, uint8_t *flags, int32_t *marker_cell, int32_t *marker_perm)
{
    const int64_t n = S->nm;
    if (flags) memset(flags, 0, (size_t)S->N);
    keyed *K = (keyed *)malloc(sizeof(keyed) * (n > 0 ? n : 1));
    for (int64_t s = 0; s < n; ++s) {
        const int64_t b = lin(S, S->base[s], S->base[n + s], S->base[2 * n + s]);
        if (marker_cell) marker_cell[s] = (int32_t)b;
        if (flags) {
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const int d[3] = {dx, dy, dz};
                        flags[stencil_node(S, s, d)] |= 1;
                    }
            flags[b] |= 2;
        }
        const float p[3] = {S->mx[s], S->mx[n + s], S->mx[2 * n + s]};
        K[s].key = orc_marker_key(S, p);
        K[s].idx = s;
    }
    qsort(K, (size_t)n, sizeof(keyed), cmp_keyed);
    if (marker_perm)
        for (int64_t s = 0; s < n; ++s) marker_perm[s] = (int32_t)K[s].idx;
    free(K);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Operator access for the tests                                             */
/* ------------------------------------------------------------------------ */

/* Streamed populations f* of the current state (Eq. 3 plus face rules). */
void orc_stream(orc_sim *S, double *out)
{
    stream_all(S, S->f, S->fs);
    memcpy(out, S->fs, sizeof(double) * Q * S->N);
}

/* Eqs. (6)-(7) on given fields rho[N], u[3][N]: penalty forces G[3][n]. */
void orc_ib_interp(orc_sim *S, const double *rho, const double *u, double *G)
{
    memcpy(S->rho, rho, sizeof(double) * S->N);
    memcpy(S->u0, u, sizeof(double) * 3 * S->N);
    if (S->nm == 0) return;
    ib_penalty(S);
    memcpy(G, S->Gs, sizeof(double) * 3 * S->nm);
}

/* Eq. (8) (gathering form) of given penalty forces G[3][n]: field g[3][N]. */
void orc_ib_spread(orc_sim *S, const double *G, double *g)
{
    if (S->nm > 0) {
        memcpy(S->Gs, G, sizeof(double) * 3 * S->nm);
        ib_gather(S);
    } else {
        memset(S->g, 0, sizeof(double) * 3 * S->N);
    }
    memcpy(g, S->g, sizeof(double) * 3 * S->N);
}
