/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of the chemical-potential multiphase
 * lattice Boltzmann step of Qin, Chen, Qin, Xu, Wen, "Spurious currents
 * suppression by accurate difference schemes in multiphase lattice Boltzmann
 * method" (arXiv 2205.09186).  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU path; every table below is built here
 * from the paper's definitions.
 *
 * Conventions (lattice units, dx = dt = c = 1, cs^2 = 1/3, Sec 2.1):
 *   - fields are stored x fastest, then y, then z; all axes periodic;
 *   - populations f[i*N + node], i the lattice direction;
 *   - the state f is the post-streaming distribution at time t.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - collision is either the SRT (BGK) reduction of Eq 1 with every
 *     s_i = 1/tau, or (D2Q9 only) the MRT form of Eq 1 with the M of Eq 3 and
 *     the rates of Sec 2.1 (s_e = 1.64, s_eps = 1.54, s_q = 1.7, s_nu = 1/tau,
 *     rate 1 on the conserved moments);
 *   - force is Eq 12 in full, F = -rho grad(mu) + cs^2 grad(rho);
 *   - k enters only through k^2 psi'(rho) (Eq 16); kappa-hat is a parameter;
 *   - Laplacian of the explicit central schemes is the matched-order central
 *     second difference per axis; of the compact schemes the composition D(D);
 *     of the isotropic schemes Eq 25b;
 *   - D3Q19 is the standard 19-velocity set (the paper only names 3D runs);
 *   - the 3D E4 weights are the D3Q19 weights divided by cs^2; the E6, E8
 *     and E10 weights (Fig 6 names these schemes but prints no weights) are
 *     the unique ones that make the weighted lattice tensors isotropic to
 *     sixth, eighth and tenth order on the shells listed with them; E10 is
 *     two-dimensional only;
 *   - OCFDS keeps the printed alpha and c; a and b come from the two
 *     fourth-order conditions so the scheme is exactly fourth order;
 *   - compact systems on a periodic line are cyclic tridiagonal, solved by the
 *     Thomas algorithm (Sec 2.3.2) with a Sherman-Morrison correction;
 *   - solid nodes (Appendix): the layers are counted through the lattice
 *     directions, as many as the central scheme's radius; their density is
 *     Eq A.1 layer by layer and their chemical potential the given mu_wall;
 *     the populations meet the wall by halfway bounce-back (the paper does not
 *     name one); only the central schemes of Eq 18-20 take walls, as the
 *     appendix describes them for those.
 *
 * Parity of every function here is pinned by the CPU tests (polynomial
 * exactness, modified wavenumber Eq 28, Table 1 constants, moment identities,
 * Gibbs-Duhem, critical point, two Maxwell formulations, mass conservation).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Parameters                                                                  */
/* ------------------------------------------------------------------------- */

enum { ORC_D2Q9 = 0, ORC_D3Q19 = 1 };
enum { ORC_CD2 = 0, ORC_CD4 = 1, ORC_CD6 = 2, ORC_E4 = 3, ORC_E8 = 4,
       ORC_OCFDS4 = 5, ORC_CFDS4 = 6, ORC_CFDS6 = 7, ORC_CFDS8 = 8,
       ORC_E6 = 9, ORC_E10 = 10, ORC_NSCHEMES = 11 };

typedef struct {
    int lattice;            /* ORC_D2Q9 or ORC_D3Q19 */
    int nx, ny, nz;         /* nz = 1 for D2Q9 */
    double tau;             /* BGK relaxation time */
    double Tr;              /* reduced temperature T / Tc */
    double k;               /* proportional coefficient of Eq 16 */
    double kappa;           /* kappa-hat of Eq 16 */
    int scheme;             /* ORC_CD2 ... */
    double a, b, R, omega;  /* Peng-Robinson constants (Sec 2.2) */
    int collision;          /* 0: SRT; 1: MRT (D2Q9, Eq 1, 3, 5) */
    double s_e, s_eps, s_q; /* MRT rates of the energy, energy-square and heat-flux
                               moments; 0 selects the values of Sec 2.1 */
    const unsigned char *solid; /* NULL: every node is fluid; else nonzero marks a
                                   solid node of the wetting boundary (Appendix) */
    double mu_wall;         /* mu_hat assigned to the solid layers (Appendix) */
} orc_params;

/* ------------------------------------------------------------------------- */
/* Velocity sets                                                               */
/* ------------------------------------------------------------------------- */

typedef struct { int q; int e[19][3]; double w[19]; } orc_lattice;

/* D2Q9 from Eq 2: e_0 = 0; e_i (i = 1..4) at angle (i-1) pi/2 with length c;
 * e_i (i = 5..8) at angle (2i-9) pi/4 with length sqrt(2) c.  Weights after
 * Eq 6: 4/9, 1/9, 1/36. */
static void lattice_d2q9(orc_lattice *L)
{
    const double pi = 3.14159265358979323846;
    memset(L, 0, sizeof(*L));
    L->q = 9;
    for (int i = 1; i <= 4; ++i) {
        double th = (i - 1) * pi / 2.0;
        L->e[i][0] = (int)lround(cos(th));
        L->e[i][1] = (int)lround(sin(th));
        L->w[i] = 1.0 / 9.0;
    }
    for (int i = 5; i <= 8; ++i) {
        double th = (2 * i - 9) * pi / 4.0;
        L->e[i][0] = (int)lround(sqrt(2.0) * cos(th));
        L->e[i][1] = (int)lround(sqrt(2.0) * sin(th));
        L->w[i] = 1.0 / 36.0;
    }
    /* rest weight 4/9, taken from the normalisation sum_i w_i = 1 (exact in
     * extended precision, then rounded) so that the nine rounded weights sum to
     * one exactly and the collision adds no systematic mass per step */
    L->w[0] = (double)(1.0L - 4.0L * L->w[1] - 4.0L * L->w[5]);
}

/* D3Q19: every integer vector with components in {-1,0,1} and |e|^2 <= 2;
 * weights 1/3 (rest), 1/18 (|e|^2 = 1), 1/36 (|e|^2 = 2). */
static void lattice_d3q19(orc_lattice *L)
{
    memset(L, 0, sizeof(*L));
    int n = 0;
    for (int s = 0; s <= 2; ++s)
        for (int z = -1; z <= 1; ++z)
            for (int y = -1; y <= 1; ++y)
                for (int x = -1; x <= 1; ++x) {
                    if (x * x + y * y + z * z != s) continue;
                    L->e[n][0] = x; L->e[n][1] = y; L->e[n][2] = z;
                    L->w[n] = (s == 0) ? 1.0 / 3.0 : (s == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                    ++n;
                }
    L->q = n; /* 19 */
    /* rest weight 1/3 from sum_i w_i = 1, as for D2Q9 */
    L->w[0] = (double)(1.0L - 6.0L * L->w[1] - 12.0L * L->w[7]);
}

static void get_lattice(int lattice, orc_lattice *L)
{
    if (lattice == ORC_D2Q9) lattice_d2q9(L); else lattice_d3q19(L);
}

static const double CS2 = 1.0 / 3.0;

/* ------------------------------------------------------------------------- */
/* Equilibrium (Eq 6), EDM forcing (Eq 8), SRT collision (Eq 1, s_i = 1/tau)   */
/* ------------------------------------------------------------------------- */

static double feq_i(const orc_lattice *L, int i, double rho, const double u[3])
{
    double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->w[i] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

void orc_feq(int lattice, double rho, double ux, double uy, double uz, double *out)
{
    orc_lattice L; get_lattice(lattice, &L);
    double u[3] = { ux, uy, uz };
    for (int i = 0; i < L.q; ++i) out[i] = feq_i(&L, i, rho, u);
}

/* Number of directions and the direction vectors, for the tests. */
int orc_lattice_info(int lattice, int *e_out, double *w_out)
{
    orc_lattice L; get_lattice(lattice, &L);
    for (int i = 0; i < L.q; ++i) {
        for (int d = 0; d < 3; ++d) if (e_out) e_out[3 * i + d] = L.e[i][d];
        if (w_out) w_out[i] = L.w[i];
    }
    return L.q;
}

/* One node: moments (Eq 7), then
 *   f*_i = f_i - (f_i - feq_i(rho,u)) / tau + [feq_i(rho,u+du) - feq_i(rho,u)]
 * with du = F / rho (Eq 8, dt = 1). */
static void collide_node(const orc_lattice *L, double tau, const double *f,
                         const double F[3], double *fout)
{
    double rho = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < L->q; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += L->e[i][d] * f[i];
    }
    double u[3], up[3];
    for (int d = 0; d < 3; ++d) { u[d] = j[d] / rho; up[d] = u[d] + F[d] / rho; }
    for (int i = 0; i < L->q; ++i) {
        double fe = feq_i(L, i, rho, u);
        double fe_shift = feq_i(L, i, rho, up);
        fout[i] = f[i] - (f[i] - fe) / tau + (fe_shift - fe);
    }
}

void orc_collide_node(int lattice, double tau, const double *f,
                      double Fx, double Fy, double Fz, double *fout)
{
    orc_lattice L; get_lattice(lattice, &L);
    double F[3] = { Fx, Fy, Fz };
    collide_node(&L, tau, f, F, fout);
}

/* ------------------------------------------------------------------------- */
/* MRT collision of Eq 1 for D2Q9                                              */
/* ------------------------------------------------------------------------- */

/* The transformation matrix of Eq 3, rows = moments (rho, e, eps, j_x, q_x,
 * j_y, q_y, p_xx, p_xy), columns = the directions of Eq 2. */
static const double MRT_M[9][9] = {
    {  1,  1,  1,  1,  1,  1,  1,  1,  1 },
    { -4, -1, -1, -1, -1,  2,  2,  2,  2 },
    {  4, -2, -2, -2, -2,  1,  1,  1,  1 },
    {  0,  1,  0, -1,  0,  1, -1, -1,  1 },
    {  0, -2,  0,  2,  0,  1, -1, -1,  1 },
    {  0,  0,  1,  0, -1,  1,  1, -1, -1 },
    {  0,  0, -2,  0,  2,  1,  1, -1, -1 },
    {  0,  1, -1,  1, -1,  0,  0,  0,  0 },
    {  0,  0,  0,  0,  0,  1, -1,  1, -1 },
};

/* M^-1 by Gauss-Jordan elimination with partial pivoting (computed once). */
static double MRT_MINV[9][9];
static int mrt_ready = 0;

static void mrt_setup(void)
{
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c) a[r][c] = c < 9 ? MRT_M[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int col = 0; col < 9; ++col) {
        int piv = col;
        for (int r = col + 1; r < 9; ++r) if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        for (int c = 0; c < 18; ++c) { double t = a[col][c]; a[col][c] = a[piv][c]; a[piv][c] = t; }
        double d = a[col][col];
        for (int c = 0; c < 18; ++c) a[col][c] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == col) continue;
            double m = a[r][col];
            for (int c = 0; c < 18; ++c) a[r][c] -= m * a[col][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) MRT_MINV[r][c] = a[r][c + 9];
    mrt_ready = 1;
}

/* The diagonal S of Eq 5 in the row order of M: s_1 = s_4 = s_6 = 1 (rho and
 * j, whose non-equilibrium parts vanish), s_2 = s_e, s_3 = s_eps,
 * s_5 = s_7 = s_q, s_8 = s_9 = 1/tau (Sec 2.1). */
static void mrt_rates(double tau, double s_e, double s_eps, double s_q, double S[9])
{
    S[0] = 1.0; S[1] = s_e; S[2] = s_eps; S[3] = 1.0; S[4] = s_q;
    S[5] = 1.0; S[6] = s_q; S[7] = 1.0 / tau; S[8] = 1.0 / tau;
}

/* One node:  m = M f,  m_eq = M f_eq(rho, u)  (Eq 4),
 *   f* = f - M^-1 S (m - m_eq) + [feq(rho, u + du) - feq(rho, u)]   (Eq 1, 8). */
static void collide_node_mrt(const orc_lattice *L, const double S[9], const double *f,
                             const double F[3], double *fout)
{
    if (!mrt_ready) mrt_setup();
    double rho = 0.0, j[3] = { 0.0, 0.0, 0.0 };
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        for (int d = 0; d < 3; ++d) j[d] += L->e[i][d] * f[i];
    }
    double u[3], up[3], fe[9], fs[9];
    for (int d = 0; d < 3; ++d) { u[d] = j[d] / rho; up[d] = u[d] + F[d] / rho; }
    for (int i = 0; i < 9; ++i) { fe[i] = feq_i(L, i, rho, u); fs[i] = feq_i(L, i, rho, up); }
    double m[9], meq[9], r[9];
    for (int k = 0; k < 9; ++k) {
        m[k] = 0.0; meq[k] = 0.0;
        for (int i = 0; i < 9; ++i) { m[k] += MRT_M[k][i] * f[i]; meq[k] += MRT_M[k][i] * fe[i]; }
        r[k] = S[k] * (m[k] - meq[k]);
    }
    for (int i = 0; i < 9; ++i) {
        double back = 0.0;
        for (int k = 0; k < 9; ++k) back += MRT_MINV[i][k] * r[k];
        fout[i] = f[i] - back + (fs[i] - fe[i]);
    }
}

void orc_collide_node_mrt(double tau, double s_e, double s_eps, double s_q, const double *f,
                          double Fx, double Fy, double Fz, double *fout)
{
    orc_lattice L; get_lattice(ORC_D2Q9, &L);
    double F[3] = { Fx, Fy, Fz }, S[9];
    mrt_rates(tau, s_e, s_eps, s_q, S);
    collide_node_mrt(&L, S, f, F, fout);
}

/* The matrix of Eq 3 and the inverse used above, for the tests. */
void orc_mrt_matrix(double *M, double *Minv)
{
    if (!mrt_ready) mrt_setup();
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) { M[9 * r + c] = MRT_M[r][c]; Minv[9 * r + c] = MRT_MINV[r][c]; }
}

/* ------------------------------------------------------------------------- */
/* Peng-Robinson equation of state (Eq 14, 15) and its critical point          */
/* ------------------------------------------------------------------------- */

/* alpha(T) of Sec 2.2 with T/Tc = Tr. */
double orc_pr_alpha(double Tr, double omega)
{
    double m = 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
    double s = 1.0 + m * (1.0 - sqrt(Tr));
    return s * s;
}

/* p0 of Eq 14 with aa = a * alpha(T). */
double orc_pr_p0(double rho, double T, double aa, double b, double R)
{
    return rho * R * T / (1.0 - b * rho) - aa * rho * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
}

/* psi'(rho) of Eq 15 (the bulk chemical potential, without the kappa term,
 * integration constant zero). */
double orc_pr_mub(double rho, double T, double aa, double b, double R)
{
    const double s2 = sqrt(2.0);
    double t1 = R * T * log(rho / (1.0 - b * rho));
    double t2 = aa / (2.0 * s2 * b) * log((s2 - 1.0 + b * rho) / (s2 + 1.0 - b * rho));
    double t3 = R * T / (1.0 - b * rho);
    double t4 = aa * rho / (1.0 + 2.0 * b * rho - b * b * rho * rho);
    return t1 - t2 + t3 - t4;
}

/* Critical point of Eq 14 with alpha = 1: dp/drho = d2p/drho2 = 0.
 * Plain Newton on (T, rho) with analytic derivatives of p. */
static void pr_derivs(double rho, double T, double a, double b, double R,
                      double *p1, double *p2, double *p1T, double *p2T, double *p3)
{
    /* p = R T rho/(1 - b rho) - a rho^2 / D, D = 1 + 2 b rho - b^2 rho^2 */
    double g = 1.0 - b * rho;
    double D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    double Dp = 2.0 * b - 2.0 * b * b * rho;
    double Dpp = -2.0 * b * b;
    /* h = rho^2 / D and its derivatives */
    double N = rho * rho, Np = 2.0 * rho, Npp = 2.0;
    double h1 = (Np * D - N * Dp) / (D * D);
    double h2 = ((Npp * D - N * Dpp) * D - 2.0 * Dp * (Np * D - N * Dp)) / (D * D * D);
    /* third derivative of h by differentiating h2 symbolically */
    double Nppp = 0.0, Dppp = 0.0;
    double A = (Npp * D - N * Dpp), Ap = (Nppp * D + Npp * Dp - Np * Dpp - N * Dppp);
    double B = (Np * D - N * Dp), Bp = (Npp * D + Np * Dp - Np * Dp - N * Dpp);
    double num = A * D - 2.0 * Dp * B;
    double nump = Ap * D + A * Dp - 2.0 * Dpp * B - 2.0 * Dp * Bp;
    double h3 = (nump * D - 3.0 * Dp * num) / (D * D * D * D);
    /* ideal part rho/(1-b rho): derivatives 1/g^2, 2b/g^3, 6b^2/g^4 */
    *p1 = R * T / (g * g) - a * h1;
    *p2 = R * T * 2.0 * b / (g * g * g) - a * h2;
    *p3 = R * T * 6.0 * b * b / (g * g * g * g) - a * h3;
    *p1T = R / (g * g);
    *p2T = R * 2.0 * b / (g * g * g);
}

int orc_pr_critical(double a, double b, double R, double *Tc, double *rhoc, double *pc)
{
    /* starting point from the van der Waals-like scale of the constants */
    double T = 0.17 * a / (b * R), rho = 0.25 / b;
    for (int it = 0; it < 100; ++it) {
        double p1, p2, p1T, p2T, p3;
        pr_derivs(rho, T, a, b, R, &p1, &p2, &p1T, &p2T, &p3);
        /* Jacobian of (p1, p2) w.r.t. (rho, T) */
        double J11 = p2, J12 = p1T, J21 = p3, J22 = p2T;
        double det = J11 * J22 - J12 * J21;
        if (det == 0.0) return -1;
        double dr = (p1 * J22 - J12 * p2) / det;
        double dT = (J11 * p2 - J21 * p1) / det;
        rho -= dr; T -= dT;
        if (fabs(dr) < 1e-15 * rho && fabs(dT) < 1e-15 * T) break;
    }
    *Tc = T; *rhoc = rho;
    *pc = orc_pr_p0(rho, T, a, b, R);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Maxwell equal-area construction, two independent formulations              */
/* ------------------------------------------------------------------------- */

static double dpdrho(double rho, double T, double aa, double b, double R)
{
    double g = 1.0 - b * rho, D = 1.0 + 2.0 * b * rho - b * b * rho * rho;
    return R * T / (g * g) - aa * (2.0 * rho + 2.0 * b * rho * rho) / (D * D);
}

/* The two spinodal densities (dp/drho = 0) below Tc, by bisection on each side
 * of the maximum of dp/drho's negative region.  Returns -1 above Tc. */
static int spinodals(double T, double aa, double b, double R, double rhoc_guess,
                     double *rs_g, double *rs_l)
{
    /* find the density of minimum dp/drho on (0, 1/b) by golden search */
    double lo = 1e-12, hi = (1.0 / b) * (1.0 - 1e-12);
    double gr = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
    double f1 = dpdrho(x1, T, aa, b, R), f2 = dpdrho(x2, T, aa, b, R);
    for (int it = 0; it < 300; ++it) {
        if (f1 < f2) { hi = x2; x2 = x1; f2 = f1; x1 = hi - gr * (hi - lo); f1 = dpdrho(x1, T, aa, b, R); }
        else { lo = x1; x1 = x2; f1 = f2; x2 = lo + gr * (hi - lo); f2 = dpdrho(x2, T, aa, b, R); }
    }
    double rmin = 0.5 * (lo + hi);
    (void)rhoc_guess;
    if (dpdrho(rmin, T, aa, b, R) >= 0.0) return -1;
    /* gas spinodal in (0, rmin): dp/drho goes + -> - */
    double a0 = 1e-300, a1 = rmin;
    for (int it = 0; it < 400; ++it) {
        double m = 0.5 * (a0 + a1);
        if (dpdrho(m, T, aa, b, R) > 0.0) a0 = m; else a1 = m;
    }
    *rs_g = 0.5 * (a0 + a1);
    /* liquid spinodal in (rmin, 1/b): - -> + */
    a0 = rmin; a1 = (1.0 / b) * (1.0 - 1e-15);
    for (int it = 0; it < 400; ++it) {
        double m = 0.5 * (a0 + a1);
        if (dpdrho(m, T, aa, b, R) < 0.0) a0 = m; else a1 = m;
    }
    *rs_l = 0.5 * (a0 + a1);
    return 0;
}

/* Formulation A: equal bulk chemical potential and equal pressure,
 * mu_b(rho_g) = mu_b(rho_l) and p0(rho_g) = p0(rho_l), by Newton on
 * (log rho_g, rho_l) from the gas-branch / liquid-branch roots at a pressure
 * inside the spinodal band. */
static double root_on_branch(double P, double lo, double hi, double T, double aa,
                             double b, double R, int increasing_from_lo)
{
    /* p is monotone on [lo, hi]; bisection in log space for the gas branch */
    for (int it = 0; it < 2000; ++it) {
        double m = (lo > 0.0 && hi / lo > 4.0) ? sqrt(lo * hi) : 0.5 * (lo + hi);
        double pm = orc_pr_p0(m, T, aa, b, R);
        int below = pm < P;
        if (below == increasing_from_lo) lo = m; else hi = m;
        if (hi - lo <= 1e-16 * hi) break;
    }
    return 0.5 * (lo + hi);
}

int orc_maxwell_mu(double Tr, double a, double b, double R, double omega,
                   double *rho_g, double *rho_l)
{
    double Tc, rhoc, pc;
    if (orc_pr_critical(a, b, R, &Tc, &rhoc, &pc)) return -1;
    if (!(Tr > 0.0 && Tr < 1.0)) return -1;
    double T = Tr * Tc, aa = a * orc_pr_alpha(Tr, omega);
    double sg, sl;
    if (spinodals(T, aa, b, R, rhoc, &sg, &sl)) return -1;
    double pmax = orc_pr_p0(sg, T, aa, b, R), pmin = orc_pr_p0(sl, T, aa, b, R);
    double lo = pmin > 0.0 ? pmin : 0.0, hi = pmax;
    /* bisection on the saturation pressure: sign of mu_l - mu_g */
    double rg = 0.0, rl = 0.0;
    for (int it = 0; it < 3000; ++it) {
        double P = (lo > 0.0 && hi / lo > 4.0) ? sqrt(lo * hi) : 0.5 * (lo + hi);
        rg = root_on_branch(P, 0.0, sg, T, aa, b, R, 1);
        rl = root_on_branch(P, sl, 1.0 / b, T, aa, b, R, 1);
        double dmu = orc_pr_mub(rl, T, aa, b, R) - orc_pr_mub(rg, T, aa, b, R);
        /* mu_l - mu_g equals the signed area int_{v_l}^{v_g} (p - P) dv, which
         * falls as P rises: a positive difference means P is still too low */
        if (dmu > 0.0) lo = P; else hi = P;
        if (hi - lo <= 4e-16 * hi) break;
    }
    /* polish with Newton on F1 = mu_l - mu_g, F2 = p_l - p_g */
    for (int it = 0; it < 50; ++it) {
        double F1 = orc_pr_mub(rl, T, aa, b, R) - orc_pr_mub(rg, T, aa, b, R);
        double F2 = orc_pr_p0(rl, T, aa, b, R) - orc_pr_p0(rg, T, aa, b, R);
        double pl = dpdrho(rl, T, aa, b, R), pg = dpdrho(rg, T, aa, b, R);
        /* d mu/d rho = p'/rho (Gibbs-Duhem) */
        double J11 = pl / rl, J12 = -pg / rg, J21 = pl, J22 = -pg;
        double det = J11 * J22 - J12 * J21;
        if (det == 0.0 || !isfinite(det)) break;
        double dl = (F1 * J22 - J12 * F2) / det;
        double dg = (J11 * F2 - J21 * F1) / det;
        if (!isfinite(dl) || !isfinite(dg)) break;
        if (fabs(dg) > 0.5 * rg) break; /* keep the gas root positive */
        rl -= dl; rg -= dg;
        if (fabs(dl) < 1e-16 * rl && fabs(dg) < 1e-16 * rg) break;
    }
    *rho_g = rg; *rho_l = rl;
    return 0;
}

/* Formulation B: equal areas in the p-v plane, v = 1/rho:
 *   int_{v_l}^{v_g} (p(v) - P) dv = 0,
 * found by bisection on P, the integral taken by composite Gauss-Legendre
 * quadrature in s = ln v (dv = v ds).  Uses only p0 of Eq 14. */
static double area_integral(double P, double rl, double rg, double T, double aa, double b, double R)
{
    static const double xg[5] = { -0.9061798459386640, -0.5384693101056831, 0.0,
                                   0.5384693101056831, 0.9061798459386640 };
    static const double wg[5] = { 0.2369268850561891, 0.4786286704993665, 0.5688888888888889,
                                   0.4786286704993665, 0.2369268850561891 };
    double s0 = log(1.0 / rl), s1 = log(1.0 / rg);
    int n = 4000;
    double h = (s1 - s0) / n, sum = 0.0;
    for (int k = 0; k < n; ++k) {
        double c = s0 + (k + 0.5) * h;
        double part = 0.0;
        for (int g = 0; g < 5; ++g) {
            double s = c + 0.5 * h * xg[g];
            double v = exp(s);
            part += wg[g] * (orc_pr_p0(1.0 / v, T, aa, b, R) - P) * v;
        }
        sum += 0.5 * h * part;
    }
    return sum;
}

int orc_maxwell_area(double Tr, double a, double b, double R, double omega,
                     double *rho_g, double *rho_l)
{
    double Tc, rhoc, pc;
    if (orc_pr_critical(a, b, R, &Tc, &rhoc, &pc)) return -1;
    if (!(Tr > 0.0 && Tr < 1.0)) return -1;
    double T = Tr * Tc, aa = a * orc_pr_alpha(Tr, omega);
    double sg, sl;
    if (spinodals(T, aa, b, R, rhoc, &sg, &sl)) return -1;
    double pmax = orc_pr_p0(sg, T, aa, b, R), pmin = orc_pr_p0(sl, T, aa, b, R);
    double lo = pmin > 0.0 ? pmin : 0.0, hi = pmax;
    double rg = 0.0, rl = 0.0;
    for (int it = 0; it < 200; ++it) {
        double P = (lo > 0.0 && hi / lo > 4.0) ? sqrt(lo * hi) : 0.5 * (lo + hi);
        rg = root_on_branch(P, 0.0, sg, T, aa, b, R, 1);
        rl = root_on_branch(P, sl, 1.0 / b, T, aa, b, R, 1);
        double A = area_integral(P, rl, rg, T, aa, b, R);
        /* A > 0: the loop above P is larger, so P must rise */
        if (A > 0.0) lo = P; else hi = P;
        if (hi - lo <= 1e-15 * hi) break;
    }
    *rho_g = rg; *rho_l = rl;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Difference operators on periodic fields (Sec 2.3)                            */
/* ------------------------------------------------------------------------- */

typedef struct { int nx, ny, nz, dim; } grid;

static inline long gidx(const grid *G, int x, int y, int z)
{
    x %= G->nx; if (x < 0) x += G->nx;
    y %= G->ny; if (y < 0) y += G->ny;
    z %= G->nz; if (z < 0) z += G->nz;
    return ((long)z * G->ny + y) * G->nx + x;
}

static inline double gat(const double *g, const grid *G, int x, int y, int z)
{
    return g[gidx(G, x, y, z)];
}

/* Explicit central first derivatives, Eq 18-20, as coefficient lists
 * c[m] for offsets m = 1..r, antisymmetric: f' = sum_m c[m](f[+m] - f[-m]). */
static int efds_first(int scheme, double c[4])
{
    memset(c, 0, 4 * sizeof(double));
    switch (scheme) {
    case ORC_CD2: c[1] = 1.0 / 2.0; return 1;                          /* Eq 18 */
    case ORC_CD4: c[1] = 8.0 / 12.0; c[2] = -1.0 / 12.0; return 2;     /* Eq 19 */
    case ORC_CD6: c[1] = 45.0 / 60.0; c[2] = -9.0 / 60.0; c[3] = 1.0 / 60.0; return 3; /* Eq 20 */
    }
    return 0;
}

/* Matched-order central second derivatives (reading of the paper's silence on
 * the Laplacian of the explicit schemes): f'' = c0 f0 + sum_m c[m](f[+m]+f[-m]). */
static int efds_second(int scheme, double *c0, double c[4])
{
    memset(c, 0, 4 * sizeof(double));
    switch (scheme) {
    case ORC_CD2: *c0 = -2.0; c[1] = 1.0; return 1;
    case ORC_CD4: *c0 = -30.0 / 12.0; c[1] = 16.0 / 12.0; c[2] = -1.0 / 12.0; return 2;
    case ORC_CD6: *c0 = -490.0 / 180.0; c[1] = 270.0 / 180.0; c[2] = -27.0 / 180.0; c[3] = 2.0 / 180.0; return 3;
    }
    return 0;
}

/* Compact tridiagonal schemes, Eq 21 with beta = 0:
 *   alpha f'_{i-1} + f'_i + alpha f'_{i+1}
 *     = a (f_{i+1}-f_{i-1})/2 + b (f_{i+2}-f_{i-2})/4 + c (f_{i+3}-f_{i-3})/6 */
static void compact_coeffs(int scheme, double *al, double *a, double *b, double *c)
{
    switch (scheme) {
    case ORC_CFDS4: *al = 0.25; *a = 1.5; *b = 0.0; *c = 0.0; break;                  /* Eq 22 */
    case ORC_CFDS6: *al = 1.0 / 3.0; *a = 14.0 / 9.0; *b = 1.0 / 9.0; *c = 0.0; break; /* Eq 23 */
    case ORC_CFDS8: *al = 3.0 / 8.0; *a = 25.0 / 16.0; *b = 1.0 / 5.0; *c = -1.0 / 80.0; break; /* Eq 24 */
    default: {
        /* OCFDS4 (Sec 3.1): printed alpha and c; b and a from the fourth-order
         * conditions a + b + c = 1 + 2 alpha and a + 4b + 9c = 6 alpha. */
        double A = 0.446776, C = -0.0541132;
        double B = (4.0 * A - 1.0 - 8.0 * C) / 3.0;
        *al = A; *c = C; *b = B; *a = 1.0 + 2.0 * A - B - C;
    }
    }
}

void orc_compact_coeffs(int scheme, double *out4)
{
    compact_coeffs(scheme, &out4[0], &out4[1], &out4[2], &out4[3]);
}

static int is_compact(int s) { return s == ORC_OCFDS4 || s == ORC_CFDS4 || s == ORC_CFDS6 || s == ORC_CFDS8; }
static int is_iso(int s) { return s == ORC_E4 || s == ORC_E6 || s == ORC_E8 || s == ORC_E10; }

/* Solve the periodic (cyclic) tridiagonal system
 *   al y_{i-1} + y_i + al y_{i+1} = d_i,  i = 0..n-1 (indices mod n),
 * by the Thomas algorithm on a modified non-periodic matrix plus a
 * Sherman-Morrison rank-one correction for the two corner entries. */
void orc_cyclic_solve(int n, double al, const double *d, double *y)
{
    if (n == 1) { y[0] = d[0] / (1.0 + 2.0 * al); return; }
    if (n == 2) {
        /* rows: y0 + 2 al y1 = d0 ; 2 al y0 + y1 = d1 */
        double det = 1.0 - 4.0 * al * al;
        y[0] = (d[0] - 2.0 * al * d[1]) / det;
        y[1] = (d[1] - 2.0 * al * d[0]) / det;
        return;
    }
    /* A = T + u v^T with u = (g, 0, .., 0, al)^T, v = (1, 0, .., 0, al/g)^T,
     * T tridiagonal with diagonal 1 except T00 = 1 - g, T(n-1)(n-1) = 1 - al^2/g. */
    double g = -1.0;
    double *diag = (double *)malloc(sizeof(double) * n);
    double *cp = (double *)malloc(sizeof(double) * n);
    double *x1 = (double *)malloc(sizeof(double) * n);
    double *x2 = (double *)malloc(sizeof(double) * n);
    double *rhs2 = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) { diag[i] = 1.0; rhs2[i] = 0.0; }
    diag[0] = 1.0 - g;
    diag[n - 1] = 1.0 - al * al / g;
    rhs2[0] = g; rhs2[n - 1] = al;
    /* Thomas forward sweep (sub- and super-diagonal al) for two right sides */
    double den = diag[0];
    cp[0] = al / den; x1[0] = d[0] / den; x2[0] = rhs2[0] / den;
    for (int i = 1; i < n; ++i) {
        den = diag[i] - al * cp[i - 1];
        cp[i] = al / den;
        x1[i] = (d[i] - al * x1[i - 1]) / den;
        x2[i] = (rhs2[i] - al * x2[i - 1]) / den;
    }
    for (int i = n - 2; i >= 0; --i) {
        x1[i] -= cp[i] * x1[i + 1];
        x2[i] -= cp[i] * x2[i + 1];
    }
    /* y = x1 - (v.x1)/(1 + v.x2) x2 */
    double vx1 = x1[0] + (al / g) * x1[n - 1];
    double vx2 = x2[0] + (al / g) * x2[n - 1];
    double fac = vx1 / (1.0 + vx2);
    for (int i = 0; i < n; ++i) y[i] = x1[i] - fac * x2[i];
    free(diag); free(cp); free(x1); free(x2); free(rhs2);
}

/* d/dx_axis of a periodic field g by scheme s (first derivative per axis). */
static void deriv_axis(const grid *G, int scheme, int axis, const double *g, double *out)
{
    int n[3] = { G->nx, G->ny, G->nz };
    if (!is_compact(scheme)) {
        double c[4];
        int r = efds_first(scheme, c);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < G->nz; ++z)
            for (int y = 0; y < G->ny; ++y)
                for (int x = 0; x < G->nx; ++x) {
                    int p[3] = { x, y, z };
                    double s = 0.0;
                    for (int m = 1; m <= r; ++m) {
                        int pp[3] = { x, y, z }, pm[3] = { x, y, z };
                        pp[axis] += m; pm[axis] -= m;
                        s += c[m] * (gat(g, G, pp[0], pp[1], pp[2]) - gat(g, G, pm[0], pm[1], pm[2]));
                    }
                    out[gidx(G, p[0], p[1], p[2])] = s;
                }
        return;
    }
    double al, a, b, c;
    compact_coeffs(scheme, &al, &a, &b, &c);
    int len = n[axis];
    int o1 = (axis + 1) % 3, o2 = (axis + 2) % 3;
    int nlines = n[o1] * n[o2];
    #pragma omp parallel for schedule(static)
    for (int line = 0; line < nlines; ++line) {
        double *dl = (double *)malloc(sizeof(double) * len);
        double *yl = (double *)malloc(sizeof(double) * len);
        int i1 = line % n[o1], i2 = line / n[o1];
        for (int i = 0; i < len; ++i) {
            int p[3];
            p[axis] = i; p[o1] = i1; p[o2] = i2;
            double f1p, f1m, f2p, f2m, f3p, f3m;
            int q[3] = { p[0], p[1], p[2] };
            q[axis] = i + 1; f1p = gat(g, G, q[0], q[1], q[2]);
            q[axis] = i - 1; f1m = gat(g, G, q[0], q[1], q[2]);
            q[axis] = i + 2; f2p = gat(g, G, q[0], q[1], q[2]);
            q[axis] = i - 2; f2m = gat(g, G, q[0], q[1], q[2]);
            q[axis] = i + 3; f3p = gat(g, G, q[0], q[1], q[2]);
            q[axis] = i - 3; f3m = gat(g, G, q[0], q[1], q[2]);
            dl[i] = a * (f1p - f1m) / 2.0 + b * (f2p - f2m) / 4.0 + c * (f3p - f3m) / 6.0;
        }
        orc_cyclic_solve(len, al, dl, yl);
        for (int i = 0; i < len; ++i) {
            int p[3];
            p[axis] = i; p[o1] = i1; p[o2] = i2;
            out[gidx(G, p[0], p[1], p[2])] = yl[i];
        }
        free(dl); free(yl);
    }
}

/* Isotropic stencils, Eq 25a/25b: weights w(|e|^2) on integer shells. */
typedef struct { int n; int e[128][3]; double w[128]; } iso_stencil;

static double iso_weight(int dim, int scheme, int s)
{
    if (scheme == ORC_E4) {
        if (dim == 2) return s == 1 ? 1.0 / 3.0 : (s == 2 ? 1.0 / 12.0 : 0.0);  /* Sec 2.3.3 */
        return s == 1 ? 1.0 / 6.0 : (s == 2 ? 1.0 / 12.0 : 0.0);
    }
    /* Higher isotropy: the weights solving sum_i w(|e_i|^2) (e_i.n)^(2m) =
     * C_m |n|^(2m) for every direction n and m = 1..order/2, with C_1 = 1 (so
     * Eq 25a is a first derivative); unique on the shells listed. */
    if (scheme == ORC_E6) {
        if (dim == 2) {     /* shells 1, 2, 4 */
            switch (s) { case 1: return 4.0 / 15.0; case 2: return 1.0 / 10.0; case 4: return 1.0 / 120.0; }
            return 0.0;
        }
        switch (s) {        /* shells 1, 2, 3, 4 */
        case 1: return 2.0 / 15.0; case 2: return 1.0 / 15.0; case 3: return 1.0 / 60.0; case 4: return 1.0 / 120.0;
        }
        return 0.0;
    }
    if (scheme == ORC_E10) {  /* two-dimensional only: shells 1, 2, 4, 5, 8, 9, 10 */
        switch (s) {
        case 1: return 262.0 / 1785.0; case 2: return 93.0 / 1190.0; case 4: return 7.0 / 340.0;
        case 5: return 6.0 / 595.0; case 8: return 9.0 / 9520.0; case 9: return 2.0 / 5355.0;
        case 10: return 1.0 / 7140.0;
        }
        return 0.0;
    }
    /* E8: shells 1, 2, 4, 5, 8 (2D); 1, 2, 3, 4, 5, 6, 8 (3D) */
    if (dim == 2) {
        switch (s) {
        case 1: return 4.0 / 21.0; case 2: return 4.0 / 45.0; case 4: return 1.0 / 60.0;
        case 5: return 2.0 / 315.0; case 8: return 1.0 / 5040.0;
        }
        return 0.0;
    }
    switch (s) {
    case 1: return 4.0 / 45.0; case 2: return 1.0 / 21.0; case 3: return 2.0 / 105.0;
    case 4: return 5.0 / 504.0; case 5: return 1.0 / 315.0; case 6: return 1.0 / 630.0;
    case 8: return 1.0 / 5040.0;
    }
    return 0.0;
}

static void iso_build(int dim, int scheme, iso_stencil *S)
{
    S->n = 0;
    int R = (scheme == ORC_E4) ? 1 : (scheme == ORC_E10 ? 3 : 2);
    int zr = (dim == 3) ? R : 0;
    for (int z = -zr; z <= zr; ++z)
        for (int y = -R; y <= R; ++y)
            for (int x = -R; x <= R; ++x) {
                int s = x * x + y * y + z * z;
                if (s == 0) continue;
                double w = iso_weight(dim, scheme, s);
                if (w == 0.0) continue;
                S->e[S->n][0] = x; S->e[S->n][1] = y; S->e[S->n][2] = z;
                S->w[S->n] = w;
                S->n++;
            }
}

/* Isotropic stencil table for the tests: returns the number of vectors. */
int orc_iso_stencil(int dim, int scheme, int *e_out, double *w_out)
{
    if (!is_iso(scheme) || (scheme == ORC_E10 && dim == 3)) return -1;
    iso_stencil S; iso_build(dim, scheme, &S);
    for (int i = 0; i < S.n; ++i) {
        for (int d = 0; d < 3; ++d) e_out[3 * i + d] = S.e[i][d];
        w_out[i] = S.w[i];
    }
    return S.n;
}

/* grad g (dim components, each N long, stored out[d*N + node]) */
static void grad_field(const grid *G, int scheme, const double *g, double *out)
{
    long N = (long)G->nx * G->ny * G->nz;
    if (is_iso(scheme)) {
        iso_stencil S; iso_build(G->dim, scheme, &S);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < G->nz; ++z)
            for (int y = 0; y < G->ny; ++y)
                for (int x = 0; x < G->nx; ++x) {
                    double s[3] = { 0.0, 0.0, 0.0 };
                    for (int i = 0; i < S.n; ++i) {
                        double v = gat(g, G, x + S.e[i][0], y + S.e[i][1], z + S.e[i][2]);
                        for (int d = 0; d < G->dim; ++d) s[d] += S.w[i] * S.e[i][d] * v;
                    }
                    long id = gidx(G, x, y, z);
                    for (int d = 0; d < G->dim; ++d) out[d * N + id] = s[d];
                }
        return;
    }
    for (int d = 0; d < G->dim; ++d) deriv_axis(G, scheme, d, g, out + d * N);
}

static void lap_field(const grid *G, int scheme, const double *g, double *out)
{
    long N = (long)G->nx * G->ny * G->nz;
    if (is_iso(scheme)) {
        iso_stencil S; iso_build(G->dim, scheme, &S);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < G->nz; ++z)
            for (int y = 0; y < G->ny; ++y)
                for (int x = 0; x < G->nx; ++x) {
                    double g0 = gat(g, G, x, y, z), s = 0.0;
                    for (int i = 0; i < S.n; ++i)
                        s += S.w[i] * (gat(g, G, x + S.e[i][0], y + S.e[i][1], z + S.e[i][2]) - g0);
                    out[gidx(G, x, y, z)] = 2.0 * s;
                }
        return;
    }
    if (is_compact(scheme)) {
        /* composition D_d(D_d g), summed over axes */
        double *t1 = (double *)malloc(sizeof(double) * N);
        double *t2 = (double *)malloc(sizeof(double) * N);
        for (long i = 0; i < N; ++i) out[i] = 0.0;
        for (int d = 0; d < G->dim; ++d) {
            deriv_axis(G, scheme, d, g, t1);
            deriv_axis(G, scheme, d, t1, t2);
            for (long i = 0; i < N; ++i) out[i] += t2[i];
        }
        free(t1); free(t2);
        return;
    }
    double c0, c[4];
    int r = efds_second(scheme, &c0, c);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < G->nz; ++z)
        for (int y = 0; y < G->ny; ++y)
            for (int x = 0; x < G->nx; ++x) {
                double s = 0.0;
                for (int d = 0; d < G->dim; ++d) {
                    double sd = c0 * gat(g, G, x, y, z);
                    for (int m = 1; m <= r; ++m) {
                        int pp[3] = { x, y, z }, pm[3] = { x, y, z };
                        pp[d] += m; pm[d] -= m;
                        sd += c[m] * (gat(g, G, pp[0], pp[1], pp[2]) + gat(g, G, pm[0], pm[1], pm[2]));
                    }
                    s += sd;
                }
                out[gidx(G, x, y, z)] = s;
            }
}

/* Public operator entry points for the tests. */
int orc_grad(int dim, int nx, int ny, int nz, int scheme, const double *g, double *out)
{
    grid G = { nx, ny, nz, dim };
    if (scheme == ORC_E10 && dim == 3) return -1;
    grad_field(&G, scheme, g, out);
    return 0;
}

int orc_lap(int dim, int nx, int ny, int nz, int scheme, const double *g, double *out)
{
    grid G = { nx, ny, nz, dim };
    if (scheme == ORC_E10 && dim == 3) return -1;
    lap_field(&G, scheme, g, out);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* The step                                                                    */
/* ------------------------------------------------------------------------- */

static int check_params(const orc_params *p)
{
    if (p->lattice != ORC_D2Q9 && p->lattice != ORC_D3Q19) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->lattice == ORC_D2Q9 && p->nz != 1) return -1;
    if (!(p->tau > 0.5)) return -1;
    if (!(p->Tr > 0.0 && p->Tr < 1.0)) return -1;
    if (!(p->k > 0.0) || !(p->kappa > 0.0)) return -1;
    if (p->scheme < 0 || p->scheme >= ORC_NSCHEMES) return -1;
    if (p->scheme == ORC_E10 && p->lattice == ORC_D3Q19) return -1;
    if (p->collision != 0 && p->collision != 1) return -1;
    if (p->collision == 1 && p->lattice != ORC_D2Q9) return -1;
    if (p->solid && p->scheme > ORC_CD6) return -1;
    return 0;
}

static void rates_of(const orc_params *p, double S[9])
{
    mrt_rates(p->tau, p->s_e > 0.0 ? p->s_e : 1.64, p->s_eps > 0.0 ? p->s_eps : 1.54,
              p->s_q > 0.0 ? p->s_q : 1.7, S);
}

typedef struct {
    double a, b, R, omega, T, aa;
} eos_t;

static int eos_of(const orc_params *p, eos_t *E)
{
    E->a = p->a > 0.0 ? p->a : 2.0 / 49.0;
    E->b = p->b > 0.0 ? p->b : 2.0 / 21.0;
    E->R = p->R > 0.0 ? p->R : 1.0;
    E->omega = p->omega > 0.0 ? p->omega : 0.344;
    double Tc, rhoc, pc;
    if (orc_pr_critical(E->a, E->b, E->R, &Tc, &rhoc, &pc)) return -1;
    E->T = p->Tr * Tc;
    E->aa = E->a * orc_pr_alpha(p->Tr, E->omega);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Wetting boundary (Appendix)                                                 */
/* ------------------------------------------------------------------------- */

static int cd_radius(int scheme) { return scheme == ORC_CD2 ? 1 : (scheme == ORC_CD4 ? 2 : 3); }

static int opposite(const orc_lattice *L, int i)
{
    for (int j = 0; j < L->q; ++j)
        if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] && L->e[j][2] == -L->e[i][2]) return j;
    return -1;
}

/* layer[n] = 0 on fluid nodes.  A solid node joins layer l (1 <= l <= r) when
 * one of its lattice neighbours x + e_i lies in layer l - 1; solid nodes that
 * no layer reaches get -1.  r is the stencil radius of the central scheme
 * (1, 2, 3 layers for CD2, CD4, CD6).  NULL when there is no solid. */
static int *wall_layers(const orc_params *p, const orc_lattice *L, const grid *G)
{
    if (!p->solid) return NULL;
    long N = (long)G->nx * G->ny * G->nz;
    int *layer = (int *)malloc(sizeof(int) * N);
    for (long n = 0; n < N; ++n) layer[n] = p->solid[n] ? -1 : 0;
    for (int l = 1; l <= cd_radius(p->scheme); ++l)
        for (int z = 0; z < G->nz; ++z)
            for (int y = 0; y < G->ny; ++y)
                for (int x = 0; x < G->nx; ++x) {
                    long n = gidx(G, x, y, z);
                    if (layer[n] != -1) continue;
                    for (int i = 1; i < L->q; ++i)
                        if (layer[gidx(G, x + L->e[i][0], y + L->e[i][1], z + L->e[i][2])] == l - 1) {
                            layer[n] = l;
                            break;
                        }
                }
    return layer;
}

/* Eq A.1: the density of a layer-l node is the lattice-weighted mean of its
 * neighbours in layer l - 1 (s_w selects them), layer after layer.  Solid
 * nodes beyond the last layer get 1 (no fluid stencil reaches them). */
static void wall_density(const orc_params *p, const orc_lattice *L, const grid *G, const int *layer, double *rho)
{
    for (int l = 1; l <= cd_radius(p->scheme); ++l)
        for (int z = 0; z < G->nz; ++z)
            for (int y = 0; y < G->ny; ++y)
                for (int x = 0; x < G->nx; ++x) {
                    long n = gidx(G, x, y, z);
                    if (layer[n] != l) continue;
                    double num = 0.0, den = 0.0;
                    for (int i = 1; i < L->q; ++i) {
                        long m = gidx(G, x + L->e[i][0], y + L->e[i][1], z + L->e[i][2]);
                        if (layer[m] == l - 1) { num += L->w[i] * rho[m]; den += L->w[i]; }
                    }
                    rho[n] = num / den;
                }
    long N = (long)G->nx * G->ny * G->nz;
    for (long n = 0; n < N; ++n)
        if (layer[n] < 0) rho[n] = 1.0;
}

/* For the tests: the layer map (int per node) and, in place, the density of
 * the solid layers by Eq A.1 from the fluid densities in rho. */
int orc_wall_density(const orc_params *p, double *rho, int *layer_out)
{
    if (check_params(p) || !p->solid) return -1;
    orc_lattice L; get_lattice(p->lattice, &L);
    grid G = { p->nx, p->ny, p->nz, p->lattice == ORC_D2Q9 ? 2 : 3 };
    int *layer = wall_layers(p, &L, &G);
    wall_density(p, &L, &G, layer, rho);
    long N = (long)p->nx * p->ny * p->nz;
    if (layer_out) memcpy(layer_out, layer, sizeof(int) * N);
    free(layer);
    return 0;
}

/* Steps 1-5 of the step on the post-streaming state f: rho, j, and the force
 * F = -rho grad(mu_hat) + cs^2 grad(rho), with
 * mu_hat = k^2 psi'(rho) - kappa_hat lap(rho) (Eq 12, 16). */
static void force_of_rho(const orc_params *p, const grid *G, const eos_t *E, const double *rho,
                         const int *layer, double *mu, double *F)
{
    long N = (long)G->nx * G->ny * G->nz;
    double *lap = (double *)malloc(sizeof(double) * N);
    double *grho = (double *)calloc(3 * N, sizeof(double));
    double *gmu = (double *)calloc(3 * N, sizeof(double));
    /* 2-3. chemical potential in mesh units */
    lap_field(G, p->scheme, rho, lap);
    #pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n)
        mu[n] = p->k * p->k * orc_pr_mub(rho[n], E->T, E->aa, E->b, E->R) - p->kappa * lap[n];
    if (layer)          /* the wall's chemical potential (Appendix) */
        for (long n = 0; n < N; ++n)
            if (layer[n] != 0) mu[n] = p->mu_wall;
    /* 4. gradients */
    grad_field(G, p->scheme, rho, grho);
    grad_field(G, p->scheme, mu, gmu);
    /* 5. force */
    for (int d = 0; d < 3; ++d)
        for (long n = 0; n < N; ++n)
            F[d * N + n] = (d < G->dim && !(layer && layer[n] != 0))
                           ? (-rho[n] * gmu[d * N + n] + CS2 * grho[d * N + n]) : 0.0;
    free(lap); free(grho); free(gmu);
}

static int force_fields(const orc_params *p, const orc_lattice *L, const double *f,
                        const int *layer, double *rho, double *j /* 3N */, double *F /* 3N */)
{
    grid G = { p->nx, p->ny, p->nz, p->lattice == ORC_D2Q9 ? 2 : 3 };
    long N = (long)p->nx * p->ny * p->nz;
    eos_t E;
    if (eos_of(p, &E)) return -1;
    /* 1. moments, Eq 7 */
    #pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < L->q; ++i) {
            double fi = f[(long)i * N + n];
            r += fi; jx += L->e[i][0] * fi; jy += L->e[i][1] * fi; jz += L->e[i][2] * fi;
        }
        rho[n] = r; j[n] = jx; j[N + n] = jy; j[2 * N + n] = jz;
    }
    if (layer) wall_density(p, L, &G, layer, rho);
    double *mu = (double *)malloc(sizeof(double) * N);
    force_of_rho(p, &G, &E, rho, layer, mu, F);
    free(mu);
    return 0;
}

/* 2-5 of the step for a given density field: mu_hat (Eq 15, 16) and
 * F = -rho grad(mu_hat) + cs^2 grad(rho) (Eq 12); F is 3N (zero beyond dim). */
int orc_force(const orc_params *p, const double *rho, double *mu, double *F)
{
    if (check_params(p)) return -1;
    grid G = { p->nx, p->ny, p->nz, p->lattice == ORC_D2Q9 ? 2 : 3 };
    eos_t E;
    if (eos_of(p, &E)) return -1;
    orc_lattice L; get_lattice(p->lattice, &L);
    int *layer = wall_layers(p, &L, &G);
    long N = (long)p->nx * p->ny * p->nz;
    double *r = (double *)malloc(sizeof(double) * N);
    memcpy(r, rho, sizeof(double) * N);
    if (layer) wall_density(p, &L, &G, layer, r);
    force_of_rho(p, &G, &E, r, layer, mu, F);
    free(r); free(layer);
    return 0;
}

/* Initial populations f = feq(rho0, 0). */
int orc_init(const orc_params *p, const double *rho0, double *f)
{
    if (check_params(p)) return -1;
    orc_lattice L; get_lattice(p->lattice, &L);
    long N = (long)p->nx * p->ny * p->nz;
    const double zero[3] = { 0.0, 0.0, 0.0 };
    for (long n = 0; n < N; ++n) {
        if (p->solid && p->solid[n]) {       /* no populations on solid nodes */
            for (int i = 0; i < L.q; ++i) f[(long)i * N + n] = 0.0;
            continue;
        }
        if (!(rho0[n] > 0.0) || !isfinite(rho0[n])) return -1;
        for (int i = 0; i < L.q; ++i) f[(long)i * N + n] = feq_i(&L, i, rho0[n], zero);
    }
    return 0;
}

/* One time step: f (post-stream, time t) -> fout (post-stream, time t+1). */
int orc_step(const orc_params *p, const double *f, double *fout)
{
    if (check_params(p)) return -1;
    orc_lattice L; get_lattice(p->lattice, &L);
    grid G = { p->nx, p->ny, p->nz, p->lattice == ORC_D2Q9 ? 2 : 3 };
    long N = (long)p->nx * p->ny * p->nz;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *j = (double *)malloc(sizeof(double) * 3 * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    int *layer = wall_layers(p, &L, &G);
    if (force_fields(p, &L, f, layer, rho, j, F)) { free(rho); free(j); free(F); free(layer); return -1; }
    double S[9];
    rates_of(p, S);
    if (p->collision == 1 && !mrt_ready) mrt_setup();
    int opp[19];
    for (int i = 0; i < L.q; ++i) opp[i] = opposite(&L, i);
    if (layer)
        for (long n = 0; n < N; ++n)
            if (layer[n] != 0)
                for (int i = 0; i < L.q; ++i) fout[(long)i * N + n] = 0.0;
    /* 6. collision, 7. streaming f_i(x + e_i, t+1) = f*_i(x, t); a population
     * whose target is solid returns to its node reversed (halfway bounce-back) */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < G.nz; ++z)
        for (int y = 0; y < G.ny; ++y)
            for (int x = 0; x < G.nx; ++x) {
                long n = gidx(&G, x, y, z);
                if (layer && layer[n] != 0) continue;
                double fl[19], fs[19];
                for (int i = 0; i < L.q; ++i) fl[i] = f[(long)i * N + n];
                double Fn[3] = { F[n], F[N + n], F[2 * N + n] };
                if (p->collision == 1) collide_node_mrt(&L, S, fl, Fn, fs);
                else collide_node(&L, p->tau, fl, Fn, fs);
                for (int i = 0; i < L.q; ++i) {
                    long m = gidx(&G, x + L.e[i][0], y + L.e[i][1], z + L.e[i][2]);
                    if (layer && layer[m] != 0) fout[(long)opp[i] * N + n] = fs[i];
                    else fout[(long)i * N + m] = fs[i];
                }
            }
    free(rho); free(j); free(F); free(layer);
    return 0;
}

int orc_run(const orc_params *p, double *f, double *work, long nsteps)
{
    /* f and work are both Q*N; the result is left in f */
    long N = (long)p->nx * p->ny * p->nz;
    int q = p->lattice == ORC_D2Q9 ? 9 : 19;
    for (long s = 0; s < nsteps; ++s) {
        if (orc_step(p, f, work)) return -1;
        memcpy(f, work, sizeof(double) * q * N);
    }
    return 0;
}

/* Macroscopic fields: rho, and the actual fluid velocity v = u + F/(2 rho)
 * (Sec 2.1, after Eq 8).  Also returns the force field if F_out is non-NULL. */
int orc_macros(const orc_params *p, const double *f, double *rho, double *vx,
               double *vy, double *vz, double *F_out)
{
    if (check_params(p)) return -1;
    orc_lattice L; get_lattice(p->lattice, &L);
    long N = (long)p->nx * p->ny * p->nz;
    double *j = (double *)malloc(sizeof(double) * 3 * N);
    double *F = (double *)malloc(sizeof(double) * 3 * N);
    grid G = { p->nx, p->ny, p->nz, p->lattice == ORC_D2Q9 ? 2 : 3 };
    int *layer = wall_layers(p, &L, &G);
    if (force_fields(p, &L, f, layer, rho, j, F)) { free(j); free(F); free(layer); return -1; }
    for (long n = 0; n < N; ++n) {
        if (layer && layer[n] != 0) {       /* solid: no fluid there */
            rho[n] = 0.0; vx[n] = 0.0; vy[n] = 0.0;
            if (vz) vz[n] = 0.0;
            continue;
        }
        double r = rho[n];
        vx[n] = j[n] / r + F[n] / (2.0 * r);
        vy[n] = j[N + n] / r + F[N + n] / (2.0 * r);
        if (vz) vz[n] = j[2 * N + n] / r + F[2 * N + n] / (2.0 * r);
    }
    if (F_out) memcpy(F_out, F, sizeof(double) * 3 * N);
    free(j); free(F); free(layer);
    return 0;
}

/* Spurious current U = max |v| over the fluid nodes (Sec 3.3) and total mass,
 * summed with Neumaier's compensated summation. */
int orc_observables(const orc_params *p, const double *f, double *umax, double *mass)
{
    long N = (long)p->nx * p->ny * p->nz;
    double *rho = (double *)malloc(sizeof(double) * N);
    double *vx = (double *)malloc(sizeof(double) * N);
    double *vy = (double *)malloc(sizeof(double) * N);
    double *vz = (double *)malloc(sizeof(double) * N);
    if (orc_macros(p, f, rho, vx, vy, vz, NULL)) { free(rho); free(vx); free(vy); free(vz); return -1; }
    double u = 0.0, s = 0.0, comp = 0.0;
    for (long n = 0; n < N; ++n) {
        double m = sqrt(vx[n] * vx[n] + vy[n] * vy[n] + vz[n] * vz[n]);
        if (m > u || m != m) u = m;
        double t = s + rho[n];
        if (fabs(s) >= fabs(rho[n])) comp += (s - t) + rho[n]; else comp += (rho[n] - t) + s;
        s = t;
    }
    *umax = u; *mass = s + comp;
    free(rho); free(vx); free(vy); free(vz);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
