/*
 * Plain FP64 CPU oracle for the per-cell real-fluid property evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file defines, as plainly as possible, what the GPU
 * property path must compute.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or constant with the
 * GPU library: every constant below is typed in here from its source, and the species data
 * arrive as raw numbers (critical constants, acentric factor, NASA-7 coefficients) from
 * the caller.
 *
 * What is computed, and from where (paper = "Detailed simulation of LOX/GCH4 flame-vortex
 * interaction in supercritical Taylor-Green flows with machine learning"):
 *   - Peng-Robinson equation of state, Section 2, Eq. (1), with the pure-fluid a and b of
 *     Section 2 (Omega constants taken at their exact critical-point values; the paper
 *     prints them rounded to 0.45724 / 0.07780) and the temperature function alpha(T) of
 *     Peng & Robinson (1976), which the paper cites but does not print.
 *   - van der Waals one-fluid mixing rules (Section 2, named only): a_m = sum_ij X_i X_j
 *     (1 - k_ij) sqrt(a_i a_j), b_m = sum_i X_i b_i.
 *   - Ideal-gas parts from NASA 7-coefficient polynomials (Cantera's thermo, Section 2).
 *   - Departure functions derived from Eq. (1): e - e_ig = int_inf^v [T dP/dT - P] dv.
 *   - Root selection by minimum Gibbs energy among the physical roots (Z > B).
 *   - Temperature inversion (rho, e, Y) -> T: the root of e(T; v, Y) = e*, here found by
 *     plain bisection to full double resolution (the definition, not an iteration scheme).
 *   - Temperature inversion (h, P, Y) -> T, the pressure-based solver's state (Section 3:
 *     properties are refreshed from h and p in every pressure-correction loop): the root of
 *     h(T; P, Y) = h* with h(T; P, Y) the (P, T, Y) state's enthalpy, by plain bisection.
 *   - The extra solver outputs of Section 4.1: psi = (d rho / d p) at constant enthalpy
 *     (and composition), thermal diffusivity lambda / (rho c_p), and each species'
 *     nondimensional standard-state enthalpy h_i/(R T) from its NASA polynomial.
 *   - Mixture-averaged diffusion coefficients (Section 2 names them, with Takahashi's
 *     high-pressure correction, whose chart is not available here): Chapman-Enskog binary
 *     coefficients with Neufeld's collision integral Omega(1,1)*, Lennard-Jones parameters
 *     from the corresponding-states relations of Chung's model (sigma = 0.809 Vc^(1/3),
 *     eps/k = Tc/1.2593), combined as D_i = (1 - Y_i) / sum_{j != i} X_j / D_ij.
 *   - Chung et al. (1988) dense-fluid viscosity and thermal conductivity ("modified Chung
 *     with mole-fraction-averaged viscosity", Section 2): Chung's high-pressure model on the
 *     one-fluid pseudo-mixture, with the low-pressure viscosity it builds on taken as the
 *     mole-fraction average of the species' low-pressure Chung viscosities, and the
 *     mixture's ideal-gas C_v in the conductivity.
 *
 * Everything is evaluated cell by cell in scalar double precision, with no reordering or
 * fusion beyond what the formulas state.  OpenMP parallelises over cells only (for timing).
 *
 * Parity unpinned: Chung's unlike-species combining rules of the pseudo-mixture and the
 * mole-fraction-averaged dilute viscosity (pinned only by reductions: identical species,
 * unit composition, permutation), and the dense terms of Chung's conductivity (B6 y and
 * the B7 term).  No printed mixture value is available to pin them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXNS 16

/* Universal gas constant, J/(mol K) (CODATA 2018, exact by SI definition). */
static const double ORC_R = 8.31446261815324;

/* Peng-Robinson constants at their exact critical-point values: with v_c the critical
 * molar volume, b/v_c = eta where eta^3 + 6 eta^2 + 12 eta - 8 = 0, and the critical
 * compressibility is Z_c = 0.30740130869870385.  They round to the paper's 0.45724 and
 * 0.07780 (Section 2). */
static const double ORC_OMEGA_A = 0.45723552892138219;
static const double ORC_OMEGA_B = 0.077796073903888456;

/* Status bits (one byte per cell). */
enum {
    ORC_NONPHYS = 1, ORC_NEWTON_MAXIT = 2, ORC_BRACKET = 4, ORC_THREE_ROOT = 8,
    ORC_GIBBS_TIE = 16, ORC_CV_NONPOS = 32
};

/* Raw species data, SI: W kg/mol, Tc K, Pc Pa, Vc m^3/mol, dipole debye. */
typedef struct {
    double W, Tc, Pc, Vc, omega, dipole, kappa, Tmid;
    double lo[7], hi[7];
} orc_species;

typedef struct {
    int ns;
    int pad;
    orc_species sp[ORC_MAXNS];
    double kij[ORC_MAXNS * ORC_MAXNS];
} orc_mech;

/* Everything the oracle knows about one cell. Mass-specific h, e, cp, cv (J/kg, J/kg/K). */
typedef struct {
    double T, P, Z, rho, v, W;
    double h, e, cp, cv, c, mu, lambda;
    double am, dam, d2am, bm, A, B;
    double h_ig, e_ig, cp_ig, cv_ig;
    double h_scale, e_scale;          /* sums of magnitudes, for relative comparisons */
    double kappa_Z, kappa_cp, kappa_T; /* condition numbers, for tolerance scaling */
    double psi, alpha;                /* (d rho/d P)_h [s^2/m^2]; lambda/(rho c_p) [m^2/s] */
    double mu_scale, lambda_scale;    /* sums of the magnitudes of the terms of mu and lambda */
    double hRT[ORC_MAXNS];            /* h_i/(R T) of each species (ideal-gas standard state) */
    double roots[3];
    int32_t nroots, nphys;
    int32_t status, iters;
} orc_cell;

/* ----------------------------------------------------------------------------------- */
/* Ideal-gas parts: NASA 7-coefficient polynomials                                     */
/* ----------------------------------------------------------------------------------- */

static const double *orc_nasa_range(const orc_species *s, double T)
{
    return (T < s->Tmid) ? s->lo : s->hi;
}

/* c_p/R of species s at T */
double orc_nasa_cp_R(const orc_species *s, double T)
{
    const double *a = orc_nasa_range(s, T);
    return a[0] + a[1] * T + a[2] * T * T + a[3] * T * T * T + a[4] * T * T * T * T;
}

/* h/(R T) of species s at T (absolute, formation-inclusive) */
double orc_nasa_h_RT(const orc_species *s, double T)
{
    const double *a = orc_nasa_range(s, T);
    return a[0] + a[1] * T / 2.0 + a[2] * T * T / 3.0 + a[3] * T * T * T / 4.0
         + a[4] * T * T * T * T / 5.0 + a[5] / T;
}

/* Mass-specific ideal-gas h, cp, e, cv of the mixture with mass fractions Y. */
static void orc_ideal(const orc_mech *m, const double *Y, double T,
                      double *h, double *cp, double *e, double *cv, double *hscale)
{
    double hh = 0, cc = 0, rw = 0, hs = 0;
    for (int i = 0; i < m->ns; i++) {
        const orc_species *s = &m->sp[i];
        double hi = ORC_R * T * orc_nasa_h_RT(s, T) / s->W;
        hh += Y[i] * hi;
        hs += fabs(Y[i] * hi);
        cc += Y[i] * ORC_R * orc_nasa_cp_R(s, T) / s->W;
        rw += Y[i] * ORC_R / s->W;
    }
    *h = hh;
    *cp = cc;
    *e = hh - rw * T;
    *cv = cc - rw;
    *hscale = hs;
}

/* ----------------------------------------------------------------------------------- */
/* Peng-Robinson pure-fluid parameters and van der Waals mixing                        */
/* ----------------------------------------------------------------------------------- */

/* kappa(omega) of Peng & Robinson (1976); the 1978 form above omega = 0.491. */
double orc_pr_kappa(double w)
{
    if (w <= 0.491)
        return 0.37464 + 1.54226 * w - 0.26992 * w * w;
    return 0.379642 + 1.48503 * w - 0.164423 * w * w + 0.016666 * w * w * w;
}

double orc_pr_ac(const orc_species *s) { return ORC_OMEGA_A * ORC_R * ORC_R * s->Tc * s->Tc / s->Pc; }
double orc_pr_b(const orc_species *s) { return ORC_OMEGA_B * ORC_R * s->Tc / s->Pc; }

/* Mole fractions and molar mass from mass fractions. */
static double orc_molefrac(const orc_mech *m, const double *Y, double *X)
{
    double s = 0;
    for (int i = 0; i < m->ns; i++) s += Y[i] / m->sp[i].W;
    double W = 1.0 / s;
    for (int i = 0; i < m->ns; i++) X[i] = Y[i] * W / m->sp[i].W;
    return W;
}

/* a_m(T), its first and second T-derivatives and b_m for mole fractions X.
 * a_i = a_c,i alpha_i with alpha_i = f_i^2, f_i = 1 + kappa_i (1 - sqrt(T/Tc_i)).
 * The cross term is the literal square root of the product a_i a_j = (g_i g_j)^2 with
 * g_i = sqrt(a_c,i) |f_i|; its derivatives follow from g_i' = sqrt(a_c,i) sign(f_i) f_i'. */
void orc_mix(const orc_mech *m, const double *X, double T,
             double *am, double *dam, double *d2am, double *bm)
{
    double g[ORC_MAXNS], g1[ORC_MAXNS], g2[ORC_MAXNS];
    for (int i = 0; i < m->ns; i++) {
        const orc_species *s = &m->sp[i];
        double k = orc_pr_kappa(s->omega);
        double ac = orc_pr_ac(s);
        double f = 1.0 + k * (1.0 - sqrt(T / s->Tc));
        double f1 = -k / (2.0 * sqrt(T * s->Tc));
        double f2 = k / (4.0 * T * sqrt(T * s->Tc));
        double sg = (f >= 0.0) ? 1.0 : -1.0;
        g[i] = sqrt(ac) * fabs(f);
        g1[i] = sqrt(ac) * sg * f1;
        g2[i] = sqrt(ac) * sg * f2;
    }
    double a = 0, a1 = 0, a2 = 0, b = 0;
    for (int i = 0; i < m->ns; i++) {
        const orc_species *si = &m->sp[i];
        double ai = orc_pr_ac(si) * pow(1.0 + orc_pr_kappa(si->omega) * (1.0 - sqrt(T / si->Tc)), 2);
        for (int j = 0; j < m->ns; j++) {
            const orc_species *sj = &m->sp[j];
            double aj = orc_pr_ac(sj) * pow(1.0 + orc_pr_kappa(sj->omega) * (1.0 - sqrt(T / sj->Tc)), 2);
            double kk = 1.0 - m->kij[i * m->ns + j];
            a += X[i] * X[j] * kk * sqrt(ai * aj);
            a1 += X[i] * X[j] * kk * (g1[i] * g[j] + g[i] * g1[j]);
            a2 += X[i] * X[j] * kk * (g2[i] * g[j] + 2.0 * g1[i] * g1[j] + g[i] * g2[j]);
        }
        b += X[i] * orc_pr_b(si);
    }
    *am = a;
    *dam = a1;
    *d2am = a2;
    *bm = b;
}

/* ----------------------------------------------------------------------------------- */
/* The cubic in Z and its real roots (no closed forms)                                 */
/* ----------------------------------------------------------------------------------- */

/* Eq. (1) with v = Z R T / P, A = a P/(R T)^2, B = b P/(R T):
 *   f(Z) = Z^3 - (1 - B) Z^2 + (A - 3 B^2 - 2 B) Z - (A B - B^2 - B^3). */
static void orc_cubic_coef(double A, double B, double c[4])
{
    c[3] = 1.0;
    c[2] = -(1.0 - B);
    c[1] = A - 3.0 * B * B - 2.0 * B;
    c[0] = -(A * B - B * B - B * B * B);
}

static double orc_poly3(const double c[4], double z) { return ((c[3] * z + c[2]) * z + c[1]) * z + c[0]; }

/* Bisect [lo, hi] (f(lo), f(hi) of opposite sign) until the midpoint is an endpoint. */
static double orc_bisect(const double c[4], double lo, double hi)
{
    double flo = orc_poly3(c, lo);
    for (int it = 0; it < 2000; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double fm = orc_poly3(c, mid);
        if (fm == 0.0) return mid;
        if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; }
        else hi = mid;
    }
    return (fabs(orc_poly3(c, lo)) <= fabs(orc_poly3(c, hi))) ? lo : hi;
}

/* All real roots of f, ascending.  The real line is split at the real roots of f'
 * (a quadratic, solved by the same bisection on its own monotone pieces), each monotone
 * piece inside the Cauchy bound is bisected where f changes sign. Returns the count. */
int orc_cubic_roots(double A, double B, double *roots)
{
    double c[4];
    orc_cubic_coef(A, B, c);
    double bound = 1.0;
    for (int k = 0; k < 3; k++) if (1.0 + fabs(c[k]) > bound) bound = 1.0 + fabs(c[k]);
    /* critical points of f: 3 Z^2 + 2 c2 Z + c1 = 0; its vertex splits it into monotone halves */
    double d[4] = {c[1], 2.0 * c[2], 3.0, 0.0};
    double vtx = -c[2] / 3.0;
    double crit[2];
    int ncrit = 0;
    double dq_v = orc_poly3(d, vtx);
    if (dq_v < 0.0) {
        /* f' < 0 at the vertex: one critical point on each side, f' > 0 at +-bound */
        crit[ncrit++] = orc_bisect(d, -bound - 1.0, vtx);
        crit[ncrit++] = orc_bisect(d, vtx, bound + 1.0);
    }
    double pts[4];
    int np = 0;
    pts[np++] = -bound;
    for (int k = 0; k < ncrit; k++) pts[np++] = crit[k];
    pts[np++] = bound;
    int nr = 0;
    for (int k = 0; k + 1 < np; k++) {
        double lo = pts[k], hi = pts[k + 1];
        double flo = orc_poly3(c, lo), fhi = orc_poly3(c, hi);
        if (flo == 0.0) { if (nr == 0 || roots[nr - 1] != lo) roots[nr++] = lo; continue; }
        if ((flo < 0) != (fhi < 0) || fhi == 0.0) {
            double r = (fhi == 0.0) ? hi : orc_bisect(c, lo, hi);
            if (nr == 0 || roots[nr - 1] != r) roots[nr++] = r;
        }
    }
    return nr;
}

/* Residual Gibbs energy over RT of a root Z (ln of the fugacity coefficient). */
double orc_gdep_RT(double Z, double A, double B)
{
    double s2 = sqrt(2.0);
    return Z - 1.0 - log(Z - B)
         - A / (2.0 * s2 * B) * log((Z + (1.0 + s2) * B) / (Z + (1.0 - s2) * B));
}

/* ----------------------------------------------------------------------------------- */
/* Chung et al. (1988) transport                                                       */
/* ----------------------------------------------------------------------------------- */

/* Viscosity coefficients E_i = a_i + b_i omega + c_i mu_r^4 + d_i kappa (Chung 1988). */
static const double CHUNG_E[10][4] = {
    {6.324, 50.412, -51.680, 1189.0},
    {1.210e-3, -1.154e-3, -6.257e-3, 0.03728},
    {5.283, 254.209, -168.48, 3898.0},
    {6.623, 38.096, -8.464, 31.42},
    {19.745, 7.630, -14.354, 31.53},
    {-1.900, -12.537, 4.985, -18.15},
    {24.275, 3.450, -11.291, 69.35},
    {0.7972, 1.117, 0.01235, -4.117},
    {-0.2382, 0.06770, -0.8163, 4.025},
    {0.06863, 0.3479, 0.5926, -0.727},
};

/* Thermal-conductivity coefficients B_i = a_i + b_i omega + c_i mu_r^4 + d_i kappa. */
static const double CHUNG_B[7][4] = {
    {2.4166, 0.74824, -0.91858, 121.72},
    {-0.50924, -1.5094, -49.991, 69.983},
    {6.6107, 5.6207, 64.760, 27.039},
    {14.543, -8.9139, -5.6379, 74.344},
    {0.79274, 0.82019, -0.69369, 6.3173},
    {-5.8634, 12.801, 9.5893, 65.529},
    {91.089, 128.11, -54.217, 523.81},
};

/* Reduced collision integral for viscosity (Neufeld, Janzen & Aziz 1972), T* = kT/eps. */
double orc_omega_v(double Ts)
{
    return 1.16145 * pow(Ts, -0.14874) + 0.52487 * exp(-0.77320 * Ts)
         + 2.16178 * exp(-2.43787 * Ts);
}

/* Reduced dipole moment mu_r = 131.3 mu / sqrt(Vc Tc), Vc in cm^3/mol. */
static double orc_mu_r(double dipole, double Vc_cm3, double Tc)
{
    return 131.3 * dipole / sqrt(Vc_cm3 * Tc);
}

/* Chung's density-correction function G2 for coefficients c1..c5 at reduced density y. */
static double orc_chung_G2(double y, const double *c)
{
    double G1 = (1.0 - 0.5 * y) / pow(1.0 - y, 3);
    double t1 = (y > 0.0) ? c[0] * (-expm1(-c[3] * y)) / y : c[0] * c[3];
    return (t1 + c[1] * G1 * exp(c[4] * y) + c[2] * G1) / (c[0] * c[3] + c[1] + c[2]);
}

/* Dense-fluid Chung viscosity [Pa s] of a fluid with the given Chung parameters at
 * temperature T [K] and molar density rho [mol/m^3]. M in g/mol, Vc in cm^3/mol. */
double orc_chung_mu(double T, double rho, double Tc, double Vc_cm3, double M,
                    double omega, double mu_r, double kappa)
{
    double mr4 = mu_r * mu_r * mu_r * mu_r;
    double E[10];
    for (int i = 0; i < 10; i++)
        E[i] = CHUNG_E[i][0] + CHUNG_E[i][1] * omega + CHUNG_E[i][2] * mr4 + CHUNG_E[i][3] * kappa;
    double Ts = 1.2593 * T / Tc;
    double Fc = 1.0 - 0.2756 * omega + 0.059035 * mr4 + kappa;
    double y = rho * 1e-6 * Vc_cm3 / 6.0;
    double G2 = orc_chung_G2(y, E);
    double muss = E[6] * y * y * G2 * exp(E[7] + E[8] / Ts + E[9] / (Ts * Ts));
    double mus = sqrt(Ts) / orc_omega_v(Ts) * Fc * (1.0 / G2 + E[5] * y) + muss;
    double mu_micropoise = 36.344 * mus * sqrt(M * Tc) / pow(Vc_cm3, 2.0 / 3.0);
    return mu_micropoise * 1e-7;
}

/* Chung low-pressure viscosity [Pa s]: the y -> 0 limit written on its own. */
double orc_chung_mu0(double T, double Tc, double Vc_cm3, double M, double omega,
                     double mu_r, double kappa)
{
    double Ts = 1.2593 * T / Tc;
    double Fc = 1.0 - 0.2756 * omega + 0.059035 * pow(mu_r, 4) + kappa;
    return 40.785 * Fc * sqrt(M * T) / (pow(Vc_cm3, 2.0 / 3.0) * orc_omega_v(Ts)) * 1e-7;
}

/* Chung dense-fluid thermal conductivity [W/(m K)] of a fluid with (pseudo-)critical
 * parameters, at T, molar density rho [mol/m^3], with ideal-gas molar Cv [J/(mol K)] and
 * low-pressure viscosity eta0 [Pa s]. */
double orc_chung_lambda_eta0(double eta0, double T, double rho, double Tc, double Vc_cm3,
                             double M, double omega, double mu_r, double kappa, double Cv,
                             double *scale)
{
    double mr4 = mu_r * mu_r * mu_r * mu_r;
    double Bc[7];
    for (int i = 0; i < 7; i++)
        Bc[i] = CHUNG_B[i][0] + CHUNG_B[i][1] * omega + CHUNG_B[i][2] * mr4 + CHUNG_B[i][3] * kappa;
    double Tr = T / Tc;
    double alpha = Cv / ORC_R - 1.5;
    double beta = 0.7862 - 0.7109 * omega + 1.3168 * omega * omega;
    double Zr = 2.0 + 10.5 * Tr * Tr;
    double psi = 1.0 + alpha * ((0.215 + 0.28288 * alpha - 1.061 * beta + 0.26665 * Zr)
                                / (0.6366 + beta * Zr + 1.061 * alpha * beta));
    double Mkg = M * 1e-3;
    double y = rho * 1e-6 * Vc_cm3 / 6.0;
    double G2 = orc_chung_G2(y, Bc);
    double q = 3.586e-3 * sqrt(Tc / Mkg) / pow(Vc_cm3, 2.0 / 3.0);
    double a = 31.2 * eta0 * psi / Mkg;
    double dense = q * Bc[6] * y * y * sqrt(Tr) * G2;
    if (scale) *scale = fabs(a / G2) + fabs(a * Bc[5] * y) + fabs(dense);
    return a * (1.0 / G2 + Bc[5] * y) + dense;
}

/* The same with the fluid's own Chung low-pressure viscosity (the textbook form). */
double orc_chung_lambda(double T, double rho, double Tc, double Vc_cm3, double M,
                        double omega, double mu_r, double kappa, double Cv)
{
    double eta0 = orc_chung_mu0(T, Tc, Vc_cm3, M, omega, mu_r, kappa);
    return orc_chung_lambda_eta0(eta0, T, rho, Tc, Vc_cm3, M, omega, mu_r, kappa, Cv, NULL);
}

/* Chung dense-fluid viscosity [Pa s] built on a given low-pressure viscosity eta0:
 * the textbook form eta = 36.344 sqrt(M Tc)/Vc^(2/3) [sqrt(T*)/Omega_v Fc (1/G2 + E6 y)
 * + eta**] with its dilute factor 36.344 sqrt(M Tc) sqrt(T*) Fc/(Vc^(2/3) Omega_v)
 * replaced by eta0. */
double orc_chung_mu_eta0(double eta0, double T, double rho, double Tc, double Vc_cm3,
                         double M, double omega, double mu_r, double kappa, double *scale)
{
    double mr4 = mu_r * mu_r * mu_r * mu_r;
    double E[10];
    for (int i = 0; i < 10; i++)
        E[i] = CHUNG_E[i][0] + CHUNG_E[i][1] * omega + CHUNG_E[i][2] * mr4 + CHUNG_E[i][3] * kappa;
    double Ts = 1.2593 * T / Tc;
    double y = rho * 1e-6 * Vc_cm3 / 6.0;
    double G2 = orc_chung_G2(y, E);
    double muss = E[6] * y * y * G2 * exp(E[7] + E[8] / Ts + E[9] / (Ts * Ts));
    double dense = 36.344 * muss * sqrt(M * Tc) / pow(Vc_cm3, 2.0 / 3.0) * 1e-7;
    if (scale) *scale = fabs(eta0 / G2) + fabs(eta0 * E[5] * y) + fabs(dense);
    return eta0 * (1.0 / G2 + E[5] * y) + dense;
}

/* Mixture transport at T and molar density rho with mole fractions X (paper, Section 2:
 * "modified Chung's transport model with mole-fraction-averaged viscosity ... for dynamic
 * viscosity and thermal conductivity").  Reading: Chung's high-pressure model with the
 * one-fluid pseudo-mixture parameters (Chung's mixing rules, xi_ij = zeta_ij = 1), in which
 * the low-pressure viscosity entering both mu and lambda is the mole-fraction average of
 * the species' own low-pressure Chung viscosities. */
void orc_transport(const orc_mech *m, const double *X, double T, double rho, double Cv,
                   double *mu, double *lam, double *mu_scale, double *lam_scale)
{
    int n = m->ns;
    double eta0 = 0;
    for (int i = 0; i < n; i++) {
        const orc_species *s = &m->sp[i];
        double Vc = s->Vc * 1e6, M = s->W * 1e3;
        eta0 += X[i] * orc_chung_mu0(T, s->Tc, Vc, M, s->omega,
                                     orc_mu_r(s->dipole, Vc, s->Tc), s->kappa);
    }

    double s3 = 0, es3 = 0, ws3 = 0, esm = 0, mu4 = 0, km = 0;
    for (int i = 0; i < n; i++) {
        const orc_species *a = &m->sp[i];
        double sig_i = 0.809 * cbrt(a->Vc * 1e6), eps_i = a->Tc / 1.2593;
        for (int j = 0; j < n; j++) {
            const orc_species *b = &m->sp[j];
            double sig_j = 0.809 * cbrt(b->Vc * 1e6), eps_j = b->Tc / 1.2593;
            double sij = sqrt(sig_i * sig_j), eij = sqrt(eps_i * eps_j);
            double wij = 0.5 * (a->omega + b->omega);
            double Mi = a->W * 1e3, Mj = b->W * 1e3;
            double Mij = 2.0 * Mi * Mj / (Mi + Mj);
            double kij = sqrt(a->kappa * b->kappa);
            double xx = X[i] * X[j];
            double sij3 = sij * sij * sij;
            s3 += xx * sij3;
            es3 += xx * eij * sij3;
            ws3 += xx * wij * sij3;
            esm += xx * eij * sij * sij * sqrt(Mij);
            mu4 += xx * a->dipole * a->dipole * b->dipole * b->dipole / sij3;
            km += xx * kij;
        }
    }
    double sm = cbrt(s3);
    double em = es3 / s3;
    double Mm = pow(esm / (em * sm * sm), 2);
    double wm = ws3 / s3;
    double mum = pow(s3 * mu4, 0.25);
    double Vcm = pow(sm / 0.809, 3);
    double Tcm = 1.2593 * em;
    double murm = 131.3 * mum / sqrt(Vcm * Tcm);
    *mu = orc_chung_mu_eta0(eta0, T, rho, Tcm, Vcm, Mm, wm, murm, km, mu_scale);
    *lam = orc_chung_lambda_eta0(eta0, T, rho, Tcm, Vcm, Mm, wm, murm, km, Cv, lam_scale);
}

/* ----------------------------------------------------------------------------------- */
/* Mixture-averaged diffusion (low-pressure Chapman-Enskog)                            */
/* ----------------------------------------------------------------------------------- */

/* Boltzmann and Avogadro constants (exact in SI since 2019). */
static const double ORC_KB = 1.380649e-23, ORC_NA = 6.02214076e23;

/* Neufeld, Janzen & Aziz (1972) fit of the Lennard-Jones diffusion collision integral
 * Omega(1,1)* as a function of T* = k T / eps. */
double orc_omega_d(double Ts)
{
    return 1.06036 / pow(Ts, 0.15610) + 0.19300 / exp(0.47635 * Ts)
         + 1.03587 / exp(1.52996 * Ts) + 1.76474 / exp(3.89411 * Ts);
}

/* Chapman-Enskog binary diffusion coefficient [m^2/s] at T [K], P [Pa] for molar masses
 * Mi, Mj [kg/mol], collision diameter sigma [m] and well depth eps/k [K]:
 * D = (3/16) sqrt(2 pi (k T)^3 / m_r) / (P pi sigma^2 Omega(1,1)*), m_r the reduced mass. */
double orc_binary_diffusion(double T, double P, double Mi, double Mj, double sigma, double eps_k)
{
    double mr = Mi * Mj / ((Mi + Mj) * ORC_NA);
    double kT = ORC_KB * T;
    double pi = acos(-1.0);
    return 3.0 / 16.0 * sqrt(2.0 * pi * kT * kT * kT / mr) / (P * pi * sigma * sigma * orc_omega_d(T / eps_k));
}

/* Lennard-Jones parameters of species s from Chung's corresponding-states relations. */
static void orc_lj(const orc_species *s, double *sigma_m, double *eps_k)
{
    *sigma_m = 0.809 * cbrt(s->Vc * 1e6) * 1e-10;
    *eps_k = s->Tc / 1.2593;
}

/* D[i] = (1 - Y_i) / sum_{j != i} X_j / D_ij, zero when no other species is present;
 * pair parameters by the Lorentz-Berthelot rules. */
void orc_mixdiff(const orc_mech *m, double P, double T, const double *Y, double *D)
{
    double X[ORC_MAXNS];
    orc_molefrac(m, Y, X);
    for (int i = 0; i < m->ns; i++) {
        double si, ei;
        orc_lj(&m->sp[i], &si, &ei);
        double sum = 0.0;
        for (int j = 0; j < m->ns; j++) {
            if (j == i) continue;
            double sj, ej;
            orc_lj(&m->sp[j], &sj, &ej);
            double Dij = orc_binary_diffusion(T, P, m->sp[i].W, m->sp[j].W, 0.5 * (si + sj), sqrt(ei * ej));
            sum += X[j] / Dij;
        }
        D[i] = (sum > 0.0) ? (1.0 - Y[i]) / sum : 0.0;
    }
}

int orc_eval_mixdiff(const orc_mech *m, int64_t n, const double *P, const double *T, const double *Y,
                     double *D, int nthreads)
{
    if (m->ns < 1 || m->ns > ORC_MAXNS) return -1;
#ifdef _OPENMP
    const int nt = (nthreads > 0) ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
#endif
    for (int64_t k = 0; k < n; k++) {
        double y[ORC_MAXNS], d[ORC_MAXNS];
        for (int i = 0; i < m->ns; i++) y[i] = Y[(int64_t)i * n + k];
        orc_mixdiff(m, P[k], T[k], y, d);
        for (int i = 0; i < m->ns; i++) D[(int64_t)i * n + k] = d[i];
    }
    return 0;
}

/* ----------------------------------------------------------------------------------- */
/* Per-cell states                                                                     */
/* ----------------------------------------------------------------------------------- */

static int orc_check_Y(const orc_mech *m, const double *Y)
{
    double s = 0;
    for (int i = 0; i < m->ns; i++) {
        if (!(Y[i] == Y[i]) || Y[i] < -1e-12) return 1;
        s += Y[i];
    }
    return fabs(s - 1.0) > 1e-6;
}

static void orc_fill_nan(orc_cell *c)
{
    double nan = NAN;
    c->T = c->P = c->Z = c->rho = c->v = nan;
    c->h = c->e = c->cp = c->cv = c->c = c->mu = c->lambda = nan;
    c->psi = c->alpha = c->mu_scale = c->lambda_scale = nan;
    for (int i = 0; i < ORC_MAXNS; i++) c->hRT[i] = nan;
}

/* Properties at molar volume v [m^3/mol] and temperature T for mass fractions Y.
 * Fills P, Z and every derived property (the part shared by both input modes). */
static void orc_props_vT(const orc_mech *m, const double *Y, const double *X, double W,
                         double v, double T, int want_transport, orc_cell *c)
{
    double am, dam, d2am, bm;
    orc_mix(m, X, T, &am, &dam, &d2am, &bm);
    double s2 = sqrt(2.0);
    double den = v * v + 2.0 * bm * v - bm * bm;
    double P = ORC_R * T / (v - bm) - am / den;
    double L = log((v + (1.0 + s2) * bm) / (v + (1.0 - s2) * bm));
    double edep = (T * dam - am) * L / (2.0 * s2 * bm);       /* J/mol */
    double cvdep = T * d2am * L / (2.0 * s2 * bm);            /* J/(mol K) */
    double hdep = edep + P * v - ORC_R * T;
    double dPdT = ORC_R / (v - bm) - dam / den;
    double dPdv = -ORC_R * T / ((v - bm) * (v - bm)) + 2.0 * am * (v + bm) / (den * den);

    double hig, cpig, eig, cvig, hs;
    orc_ideal(m, Y, T, &hig, &cpig, &eig, &cvig, &hs);
    double cv_molar = W * cvig + cvdep;
    double cp_molar = cv_molar - T * dPdT * dPdT / dPdv;
    double c2 = -(v * v / W) * (cp_molar / cv_molar) * dPdv;

    c->T = T;
    c->P = P;
    c->v = v;
    c->W = W;
    c->rho = W / v;
    c->Z = P * v / (ORC_R * T);
    c->am = am;
    c->dam = dam;
    c->d2am = d2am;
    c->bm = bm;
    c->A = am * P / (ORC_R * ORC_R * T * T);
    c->B = bm * P / (ORC_R * T);
    c->h_ig = hig;
    c->e_ig = eig;
    c->cp_ig = cpig;
    c->cv_ig = cvig;
    c->h = hig + hdep / W;
    c->e = eig + edep / W;
    c->cp = cp_molar / W;
    c->cv = cv_molar / W;
    c->c = (c2 > 0.0) ? sqrt(c2) : NAN;
    c->h_scale = hs + fabs(hdep / W) + fabs(P * v / W) + fabs(ORC_R * T / W);
    c->e_scale = hs + fabs(edep / W) + fabs(ORC_R * T / W);
    /* cancellation in (dP/dv)_T and in the c_p correction */
    double t1 = ORC_R * T / ((v - bm) * (v - bm)), t2 = 2.0 * am * (v + bm) / (den * den);
    double kdv = (t1 + t2) / fabs(dPdv);
    c->kappa_cp = kdv * (1.0 + fabs(T * dPdT * dPdT / dPdv) / fabs(cp_molar));
    c->kappa_T = fabs(c->e_scale) / (T * fabs(c->cv));
    if (cv_molar <= 0.0) c->status |= ORC_CV_NONPOS;
    /* psi = (d rho/d P) along an isenthalp at fixed composition.  With rho = W/v:
     *   (dv/dP)_h = (dv/dP)_T + (dv/dT)_P (dT/dP)_h,
     *   (dv/dP)_T = 1/(dP/dv)_T,  (dv/dT)_P = -(dP/dT)_v/(dP/dv)_T,
     *   (dT/dP)_h = -(dH/dP)_T / C_p = -(v - T (dv/dT)_P) / C_p   (molar H, C_p). */
    double dvdP_T = 1.0 / dPdv;
    double dvdT_P = -dPdT / dPdv;
    double dTdP_h = -(v - T * dvdT_P) / cp_molar;
    double dvdP_h = dvdP_T + dvdT_P * dTdP_h;
    c->psi = -(W / (v * v)) * dvdP_h;
    for (int i = 0; i < ORC_MAXNS; i++) c->hRT[i] = (i < m->ns) ? orc_nasa_h_RT(&m->sp[i], T) : 0.0;
    if (want_transport) {
        orc_transport(m, X, T, 1.0 / v, W * cvig, &c->mu, &c->lambda, &c->mu_scale, &c->lambda_scale);
        c->alpha = c->lambda / (c->rho * c->cp);
    } else {
        c->mu = c->lambda = c->alpha = c->mu_scale = c->lambda_scale = NAN;
    }
}

/* (P, T, Y) mode: the PR cubic with Gibbs root selection, then every property. */
void orc_state_PT(const orc_mech *m, double P, double T, const double *Y,
                  int want_transport, orc_cell *c)
{
    memset(c, 0, sizeof(*c));
    if (!(P > 0.0) || !(T > 0.0) || orc_check_Y(m, Y)) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    }
    double X[ORC_MAXNS];
    double W = orc_molefrac(m, Y, X);
    double am, dam, d2am, bm;
    orc_mix(m, X, T, &am, &dam, &d2am, &bm);
    double A = am * P / (ORC_R * ORC_R * T * T);
    double B = bm * P / (ORC_R * T);
    double r[3];
    int nr = orc_cubic_roots(A, B, r);
    double phys[3];
    int np = 0;
    for (int k = 0; k < nr; k++) if (r[k] > B) phys[np++] = r[k];
    double Z;
    if (np == 0) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    } else if (np == 1) {
        Z = phys[0];
    } else {
        /* two or three physical roots: compare the smallest and the largest */
        double zl = phys[0], zv = phys[np - 1];
        double gl = orc_gdep_RT(zl, A, B), gv = orc_gdep_RT(zv, A, B);
        if (np == 3) c->status |= ORC_THREE_ROOT;
        double tie = 1e-12 * fmax(1.0, fmax(fabs(gl), fabs(gv)));
        if (fabs(gl - gv) <= tie) {
            Z = zv;
            c->status |= ORC_GIBBS_TIE;
        } else {
            Z = (gl < gv) ? zl : zv;
        }
    }
    double v = Z * ORC_R * T / P;
    int status = c->status;
    orc_props_vT(m, Y, X, W, v, T, want_transport, c);
    c->status |= status;
    /* report the pressure and Z the caller asked about, not the re-evaluated EOS value */
    c->P = P;
    c->Z = Z;
    c->A = A;
    c->B = B;
    for (int k = 0; k < 3; k++) c->roots[k] = (k < nr) ? r[k] : NAN;
    c->nroots = nr;
    c->nphys = np;
    double fp = fabs((3.0 * Z - 2.0 * (1.0 - B)) * Z + (A - 3.0 * B * B - 2.0 * B));
    double mag = fabs(Z * Z * Z) + fabs((1.0 - B) * Z * Z) + fabs((A - 3.0 * B * B - 2.0 * B) * Z)
               + fabs(A * B - B * B - B * B * B);
    c->kappa_Z = mag / fmax(fabs(Z) * fp, 1e-300);
}

/* Molar-volume/temperature state (used by the finite-difference checks). */
void orc_state_vT(const orc_mech *m, double v, double T, const double *Y,
                  int want_transport, orc_cell *c)
{
    memset(c, 0, sizeof(*c));
    if (!(v > 0.0) || !(T > 0.0) || orc_check_Y(m, Y)) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    }
    double X[ORC_MAXNS];
    double W = orc_molefrac(m, Y, X);
    orc_props_vT(m, Y, X, W, v, T, want_transport, c);
}

/* Mass-specific internal energy at (v, T): ideal part plus departure. */
static double orc_energy(const orc_mech *m, const double *Y, const double *X, double W,
                         double v, double T)
{
    double am, dam, d2am, bm;
    orc_mix(m, X, T, &am, &dam, &d2am, &bm);
    double s2 = sqrt(2.0);
    double L = log((v + (1.0 + s2) * bm) / (v + (1.0 - s2) * bm));
    double edep = (T * dam - am) * L / (2.0 * s2 * bm);
    double hig, cpig, eig, cvig, hs;
    orc_ideal(m, Y, T, &hig, &cpig, &eig, &cvig, &hs);
    return eig + edep / W;
}

/* Temperature bracket of the inversion. */
static const double ORC_TLO = 60.0, ORC_THI = 5000.0;

/* (rho, e, Y) mode: T solves e(T; v = W/rho, Y) = e*, found by bisection on
 * [60 K, 5000 K] until the midpoint is an endpoint; then every property at (v, T). */
void orc_state_rhoe(const orc_mech *m, double rho, double e, const double *Y,
                    int want_transport, orc_cell *c)
{
    memset(c, 0, sizeof(*c));
    if (!(rho > 0.0) || !(e == e) || orc_check_Y(m, Y)) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    }
    double X[ORC_MAXNS];
    double W = orc_molefrac(m, Y, X);
    double v = W / rho;
    double bm = 0;
    for (int i = 0; i < m->ns; i++) bm += X[i] * orc_pr_b(&m->sp[i]);
    if (!(v > bm)) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    }
    double lo = ORC_TLO, hi = ORC_THI;
    double rlo = orc_energy(m, Y, X, W, v, lo) - e;
    double rhi = orc_energy(m, Y, X, W, v, hi) - e;
    if (rlo > 0.0 || rhi < 0.0) {
        c->status |= ORC_BRACKET;
        orc_fill_nan(c);
        return;
    }
    int it = 0;
    for (; it < 4000; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double r = orc_energy(m, Y, X, W, v, mid) - e;
        if (r == 0.0) { lo = hi = mid; break; }
        if (r < 0.0) lo = mid; else hi = mid;
    }
    double rl = fabs(orc_energy(m, Y, X, W, v, lo) - e);
    double rh = fabs(orc_energy(m, Y, X, W, v, hi) - e);
    double T = (rl <= rh) ? lo : hi;
    orc_props_vT(m, Y, X, W, v, T, want_transport, c);
    c->iters = it;
}

/* Mass-specific enthalpy of the (P, T, Y) state (Gibbs-selected root). */
static double orc_enthalpy_PT(const orc_mech *m, double P, double T, const double *Y)
{
    orc_cell c;
    orc_state_PT(m, P, T, Y, 0, &c);
    return c.h;
}

/* (h, P, Y) mode: T solves h(T; P, Y) = h* with h the (P, T, Y) state's enthalpy, found by
 * bisection on [60 K, 5000 K] until the midpoint is an endpoint; then the (P, T, Y) state.
 * Where the selected root switches (liquid- to vapour-like), h(T) jumps and the bisection
 * ends at the switch temperature; the side with the smaller |h - h*| is reported. */
void orc_state_hP(const orc_mech *m, double h, double P, const double *Y,
                  int want_transport, orc_cell *c)
{
    memset(c, 0, sizeof(*c));
    if (!(P > 0.0) || !(h == h) || orc_check_Y(m, Y)) {
        c->status |= ORC_NONPHYS;
        orc_fill_nan(c);
        return;
    }
    double lo = ORC_TLO, hi = ORC_THI;
    double rlo = orc_enthalpy_PT(m, P, lo, Y) - h;
    double rhi = orc_enthalpy_PT(m, P, hi, Y) - h;
    if (rlo > 0.0 || rhi < 0.0) {
        c->status |= ORC_BRACKET;
        orc_fill_nan(c);
        return;
    }
    int it = 0;
    for (; it < 4000; it++) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        double r = orc_enthalpy_PT(m, P, mid, Y) - h;
        if (r == 0.0) { lo = hi = mid; break; }
        if (r < 0.0) lo = mid; else hi = mid;
    }
    double rl = fabs(orc_enthalpy_PT(m, P, lo, Y) - h);
    double rh = fabs(orc_enthalpy_PT(m, P, hi, Y) - h);
    double T = (rl <= rh) ? lo : hi;
    orc_state_PT(m, P, T, Y, want_transport, c);
    c->iters = it;
}

/* ----------------------------------------------------------------------------------- */
/* Batched entry points (cells independent; OpenMP over cells only)                    */
/* ----------------------------------------------------------------------------------- */

/* mode 0: (P, T, Y) with in0 = P, in1 = T.  mode 1: (rho, e, Y) with in0 = rho, in1 = e.
 * mode 2: (v, T, Y) with in0 = molar volume, in1 = T.  mode 3: (h, P, Y) with in0 = h,
 * in1 = P.  Y is species-major [ns][n].  nthreads > 0 caps the threads of this call. */
int orc_eval(const orc_mech *m, int mode, int64_t n, const double *in0, const double *in1,
             const double *Y, int want_transport, orc_cell *out, int nthreads)
{
    if (m->ns < 1 || m->ns > ORC_MAXNS || mode < 0 || mode > 3) return -1;
#ifdef _OPENMP
    const int nt = (nthreads > 0) ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nt)
#endif
    for (int64_t k = 0; k < n; k++) {
        double y[ORC_MAXNS];
        for (int i = 0; i < m->ns; i++) y[i] = Y[(int64_t)i * n + k];
        if (mode == 0) orc_state_PT(m, in0[k], in1[k], y, want_transport, &out[k]);
        else if (mode == 1) orc_state_rhoe(m, in0[k], in1[k], y, want_transport, &out[k]);
        else if (mode == 2) orc_state_vT(m, in0[k], in1[k], y, want_transport, &out[k]);
        else orc_state_hP(m, in0[k], in1[k], y, want_transport, &out[k]);
    }
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_sizeof_cell(void) { return (int)sizeof(orc_cell); }
int orc_sizeof_mech(void) { return (int)sizeof(orc_mech); }
