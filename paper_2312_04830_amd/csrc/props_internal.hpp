// Internal declarations of libprops: device table layouts, error plumbing, handles.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/props.h"

namespace props {

// ---------------------------------------------------------------- constants
// Universal gas constant J/(mol K) (SI exact).
constexpr double kR = 8.31446261815324;
// Peng-Robinson Omega constants at their exact critical-point values (the roots of the
// critical conditions dP/dv = d2P/dv2 = 0 of Eq. (1)); the paper prints them rounded to
// 0.45724 and 0.07780 (Section 2).
constexpr double kOmegaA = 0.45723552892138219;
constexpr double kOmegaB = 0.077796073903888456;
constexpr double kSqrt2 = 1.4142135623730951;

// Temperature bracket of the (rho, e, Y) inversion, K.
constexpr double kTlo = 60.0;
constexpr double kThi = 5000.0;

// ---------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

#define PROPS_HIP_TRY(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::props::fail(PROPS_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------- device tables
// Species count the kernels are compiled for; a mechanism with ns species runs the
// smallest NSP >= ns, the extra slots holding inert zero entries.
constexpr int kPadSizes[4] = {1, 2, 4, 8};

// Thermochemistry: always double (the ideal-gas energy carries the Newton residual).
template <int NS>
struct ThermoTab {
    double invW[NS];      // 1/W_i [mol/kg]
    double RW[NS];        // R/W_i [J/(kg K)]
    double b[NS];         // PR co-volume b_i [m^3/mol]
    double cp[2][5][NS];  // (R/W_i) a1..a5 per range (0: T < Tmid, 1: T >= Tmid), J/(kg K)
    double a6[2][NS];     // (R/W_i) a6 per range, J/kg
    double WR[NS];        // W_i/R [kg K/J], turns a species' h [J/kg] at T into h/(R T) * T
    double Tmid;
    double exp2j[64];     // 2^(j/64), j = 0..63, correctly rounded: the table of fm::exp_tab
};

// Mixing and transport constants, in the working precision R of the algebra.
// A symmetric pair matrix stored upper-triangular with doubled off-diagonals gives the
// quadratic form x^T C x as sum_i x_i sum_{j >= i} C'_ij x_j.
template <typename R, int NS>
struct MixTab {
    R sqac[NS];      // sqrt(a_c,i), a_c = Omega_a R^2 Tc^2 / Pc
    R k1[NS];        // 1 + kappa_i   (alpha_i = (k1 - k2 sqrt(T))^2)
    R k2[NS];        // kappa_i / sqrt(Tc_i)
    R K[NS][NS];     // 1 - k_ij (full, symmetric)
    R tstar[NS];     // T*_i = Tc_i (1 + 1/kappa_i)^2 where 1 + kappa_i (1 - sqrt(T/Tc_i)) = 0 (inf if kappa_i = 0)
    // Chung (1988) per species
    R mu0A[NS];      // 40.785e-7 Fc_i sqrt(M_i) / Vc_i^(2/3): dilute mu_i = mu0A_i sqrt(T) / Omega_v
    R tsc[NS];       // 1.2593 / Tc_i  (T*_i = tsc_i T)
    R tsp[NS];       // 1.16145 tsc_i^-0.14874
    // Chung pseudo-mixture.  With sigma_ij = sqrt(sigma_i sigma_j), eps_ij = sqrt(eps_i eps_j),
    // kappa_ij = sqrt(kappa_i kappa_j) and omega_ij = (omega_i + omega_j)/2, five of the six
    // double sums factor into single sums:
    //   sum X_i X_j sigma_ij^3          = (sum X_i p_i)^2,          p_i = sigma_i^1.5
    //   sum X_i X_j eps_ij sigma_ij^3   = (sum X_i q_i)^2,          q_i = sqrt(eps_i) p_i
    //   sum X_i X_j omega_ij sigma_ij^3 = (sum X_i omega_i p_i)(sum X_j p_j)
    //   sum X_i X_j mu_i^2 mu_j^2 / sigma_ij^3 = (sum X_i mu_i^2 / p_i)^2
    //   sum X_i X_j kappa_ij            = (sum X_i sqrt(kappa_i))^2
    // and only the molar-mass rule (harmonic mean M_ij) stays a quadratic form.
    R cp_p[NS], cp_q[NS], cp_wp[NS], cp_m[NS], cp_k[NS];
    R ESM[NS][NS];   // eps_ij sigma_ij^2 sqrt(M_ij), upper-triangular, doubled off-diagonal
};

// Mixture-averaged diffusion (Chapman-Enskog), per unordered species pair p = (i < j),
// upper triangle in row-major order.  The binary coefficient is
//   D_ij = T^1.5 / (P G_ij Omega_D(T / eps_ij)),  G_ij = (16/3) sigma_ij^2 sqrt(pi m_ij / (2 k^3)),
// m_ij the reduced molecular mass.  With Neufeld's fit of Omega_D the product G_ij Omega_D is
//   c0 T^-0.15610 + c1 exp(x1 T) + c2 exp(x2 T) + c3 exp(x3 T).
// Pairs with a padding species hold zeros.
template <typename R, int NS>
struct DiffTab {
    static constexpr int NP = (NS * (NS - 1) / 2 > 0) ? NS * (NS - 1) / 2 : 1;
    R c0[NP];                // 1.06036 G_ij eps_ij^0.15610
    R c1[NP], c2[NP], c3[NP];  // 0.19300 G_ij, 1.03587 G_ij, 1.76474 G_ij
    R x1[NP], x2[NP], x3[NP];  // -0.47635/eps_ij, -1.52996/eps_ij, -3.89411/eps_ij  [1/K]
};

}  // namespace props

// ---------------------------------------------------------------- handles
struct props_mech_s {
    int ns = 0;
    int nsp = 0;          // padded species count the kernels run with
    int device = 0;
    int maxit = 100;
    double rtol = 1e-10;
    // one allocation: ThermoTab | MixTab<double> | MixTab<float> | DiffTab<double> | DiffTab<float>
    void *d_tab = nullptr;
    size_t off_mixd = 0, off_mixf = 0, off_diffd = 0, off_difff = 0, bytes = 0;
    props_species_desc sp[PROPS_MAX_SPECIES];
    double kij[PROPS_MAX_SPECIES * PROPS_MAX_SPECIES];
};

namespace props {
// Launch the PR property kernel for a mechanism (defined in pr_kernel.hip).
int launch_pr(const props_mech_s *m, int mode, int prec, const props_in *in,
              const props_out *out, int64_t n, uint8_t *status, hipStream_t stream);
// The same with the species rows of Y (and of the hRT output) ldy >= n elements apart, so
// that a range of cells of a larger array can be evaluated in place.
int launch_pr_strided(const props_mech_s *m, int mode, int prec, const props_in *in,
                      const props_out *out, int64_t n, int64_t ldy, uint8_t *status, hipStream_t stream);
// The same over a device list of cells: lane k < *count evaluates cell idx[k] of arrays of
// length n (species rows ldy apart), OR-ing st_or into its status byte (grid sized for n);
// entries outside [0, n) are skipped.
int launch_pr_indirect(const props_mech_s *m, int mode, int prec, const props_in *in,
                       const props_out *out, int64_t n, int64_t ldy, const int *idx, const int *count,
                       uint8_t *status, uint8_t st_or, hipStream_t stream);
// Mixture-averaged diffusion coefficients (diffusion.hip).
int launch_diffusion(const props_mech_s *m, int prec, const double *P, const double *T,
                     const double *Y, double *D, int64_t n, uint8_t *status, hipStream_t stream);
// The surrogate with caller-provided fallback scratch (idx: n ints, count: 1 int), so
// that concurrent evaluations on different streams never share scratch (mlp.hip); the
// species rows of in->Y are ldy >= n elements apart.
int dnn_eval(props_dnn_s *d, props_mech_s *fb, const props_in *in, const props_out *out, int64_t n,
             int64_t ldy, uint8_t *status, int *fb_idx, int *fb_count, hipStream_t s);
// Device a network handle was created on (mlp.hip).
int dnn_device(const props_dnn_s *d);
}  // namespace props
