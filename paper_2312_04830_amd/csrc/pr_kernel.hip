// Peng-Robinson property kernels for gfx950 (one lane per cell).
//
// What a lane computes (paper, Section 2; Eq. (1) is the Peng-Robinson equation):
//   composition      W = 1/sum(Y_i/W_i), X_i = Y_i W / W_i, b_m = sum X_i b_i
//   alpha / mixing   g_i = sqrt(a_c,i) |1 + kappa_i (1 - sqrt(T/Tc_i))|,
//                    a_m = sum_ij X_i X_j (1 - k_ij) g_i g_j, exactly A0 + A1 sqrt(T) + A2 T
//                    between the temperatures where a factor changes sign: coefficients from
//                    two mat-vecs with the (1 - k_ij) matrix (over the pairs i < j in some
//                    kernels), then O(1) per evaluation
//   ideal gas        per-cell NASA-7 mixture coefficients, one Horner each for h, cp
//   (P,T,Y)          cubic in Z (largest root in closed form, deflation for the others,
//                    Newton polish, double), physical roots Z > B, minimum residual Gibbs
//                    energy between the liquid- and vapour-like root
//   (rho,e,Y)        bracketed Newton-type iteration (Chebyshev's third-order step) on
//                    e(T; v, Y) = e* (v fixed, so the departure log is computed once),
//                    bisection whenever a step leaves the bracket or fails to halve
//   (h,P,Y)          the pressure-based solver's state (Section 3): bracketed Newton on
//                    h(T; P, Y) = h* with the cubic and root choice inside every evaluation
//                    and the real-fluid cp as the slope
//   departures       e, h, cv, cp, (dP/dT)_v, (dP/dv)_T, sound speed, and the solver
//                    outputs of Section 4.1: psi = (d rho/d P)_h, lambda/(rho cp), h_i/(R T)
//   transport        Chung's high-pressure viscosity and conductivity on the pseudo-mixture,
//                    with the mole-fraction-averaged low-pressure viscosity (Section 2)
//
// Memory: every per-cell array is structure-of-arrays in HBM, read or written once with
// unit stride across a wavefront.  Mechanism tables (a few KB) are read with
// wave-uniform addresses, so they come through the scalar data cache into SGPRs and feed
// the VALU as scalar operands; no LDS is needed for them.
#include <cmath>
#include <type_traits>

#include "fastmath.hpp"
#include "props_internal.hpp"

namespace props {

// ------------------------------------------------------------------ precision policies
// Double precision: the table-driven exp (table in LDS), the lean log and the refined
// reciprocal and reciprocal square root of fastmath.hpp, the device library's expm1 (a few ulp; outputs stay within
// 1e-15 relative of correctly rounded maths).
struct P64 {
    using R = double;
    static __device__ __forceinline__ R sqrt_(R x) { return sqrt(x); }
    static __device__ __forceinline__ R rsqrt_(R x) { return fm::rsqrt(x); }
    static __device__ __forceinline__ R log_(R x) { return fm::log(x); }
    static __device__ __forceinline__ R exp_(R x, const double *e2) { return fm::exp_tab(x, e2); }
    static __device__ __forceinline__ R expm1_(R x) { return expm1(x); }
    static __device__ __forceinline__ R cbrt_(R x) { return cbrt(x); }
    static __device__ __forceinline__ R div(R a, R b) { return a * fm::rcp(b); }
};

// Single precision with the hardware transcendental unit (v_exp_f32, v_log_f32, v_rcp_f32).
struct P32 {
    using R = float;
    static __device__ __forceinline__ R sqrt_(R x) { return __builtin_sqrtf(x); }
    static __device__ __forceinline__ R rsqrt_(R x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ R log_(R x) { return __logf(x); }
    static __device__ __forceinline__ R exp_(R x, const double *) { return __expf(x); }
    static __device__ __forceinline__ R expm1_(R x) { return expm1f(x); }
    static __device__ __forceinline__ R cbrt_(R x) { return cbrtf(x); }
    static __device__ __forceinline__ R div(R a, R b) { return a * __builtin_amdgcn_rcpf(b); }
};

// ------------------------------------------------------------------ kernel arguments
struct PRArgs {
    const double *in0, *in1, *Y, *Tg;
    double *oT, *oP, *oZ, *orho, *oh, *oe, *ocp, *oc, *omu, *olam;
    double *opsi, *oalpha, *ohRT;
    uint8_t *status, *iters;
    const int *idx;    // optional cell list: lane k evaluates cell idx[k] for k < *count
    const int *count;
    int64_t n;         // cells in the arrays
    int64_t ldy;       // element stride between species rows of Y and hRT (>= n)
    int ns, maxit;
    double rtol;
    uint8_t st_or;     // bits OR-ed into every status byte written
};

// ------------------------------------------------------------------ mixing sums
// With s = sqrt(T), each g_i = sqrt(a_c,i) |k1_i - k2_i s| is linear in s between the
// temperatures T*_i = (k1_i/k2_i)^2 where its sign flips.  For a fixed sign pattern
// sigma, u_i = X_i g_i = alpha_i - beta_i s with alpha_i = X_i sqrt(a_c,i) sigma_i k1_i and
// beta_i = X_i sqrt(a_c,i) sigma_i k2_i, so the van der Waals sum is exactly
//   a_m = u.K.u = A0 + A1 s + A2 T,  A0 = alpha.K.alpha, A1 = -2 alpha.K.beta, A2 = beta.K.beta
// and a_m' = A1/(2s) + A2, a_m'' = -A1/(4 s T).  The two mat-vecs are done once per sign
// pattern; every Newton evaluation is then O(1).  MixQuad::lo/hi bound the T interval in
// which the pattern holds.
template <class PM, int NS, bool TRI>
struct MixQuad {
    using R = typename PM::R;
    R A0, A1, A2;
    double lo, hi;   // T interval of the sign pattern

    __device__ __forceinline__ void build(const MixTab<R, NS> *__restrict__ t0, const R (&X)[NS], double T)
    {
        // Read the table here, through the scalar cache, each time a pattern is built: left
        // to itself the compiler hoists the 1 - k_ij matrix out of the Newton loop for the
        // rare rebuild, and ~130 live uniform values spill into VGPR lanes.
        const MixTab<R, NS> *tg = t0;
        asm volatile("" : "+s"(tg));
        const __attribute__((address_space(4))) MixTab<R, NS> *t =
            (const __attribute__((address_space(4))) MixTab<R, NS> *)tg;
        R al[NS], be[NS];
        lo = 0.0;
        hi = __builtin_inf();
#pragma unroll
        for (int i = 0; i < NS; i++) {
            const double ts = (double)t->tstar[i];
            const bool neg = T > ts;   // f_i = k1 - k2 sqrt(T) < 0 beyond T*_i
            if (neg) lo = fmax(lo, ts);
            else hi = fmin(hi, ts);
            const R xs = X[i] * t->sqac[i];
            const R sg = neg ? R(-1) : R(1);
            al[i] = sg * xs * t->k1[i];
            be[i] = sg * xs * t->k2[i];
        }
        R a0 = 0, a1 = 0, a2 = 0;
        if constexpr (TRI) {
            // K is symmetric with a unit diagonal (k_ii = 0, enforced when the mechanism is
            // made), so each quadratic form is its diagonal plus twice the sum over i < j:
            //   alpha.K.beta = sum_i [alpha_i (beta_i + wb_i) + beta_i wa_i],
            // wa_i = sum_{j>i} K_ij alpha_j, wb_i = sum_{j>i} K_ij beta_j.  Each row's values
            // are loaded once the previous row is done (the opaque pointer depends on its
            // result), so that few of them are live in scalar registers.
#pragma unroll
            for (int i = 0; i < NS; i++) {
                const MixTab<R, NS> *tr = t0;
                asm volatile("" : "+s"(tr) : "v"(a2));
                const __attribute__((address_space(4))) MixTab<R, NS> *tk =
                    (const __attribute__((address_space(4))) MixTab<R, NS> *)tr;
                R wa = 0, wb = 0;
#pragma unroll
                for (int j = i + 1; j < NS; j++) {
                    wa += tk->K[i][j] * al[j];
                    wb += tk->K[i][j] * be[j];
                }
                a0 += al[i] * (al[i] + R(2) * wa);
                a1 += al[i] * (be[i] + wb) + be[i] * wa;
                a2 += be[i] * (be[i] + R(2) * wb);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NS; i++) {
                R wa = 0, wb = 0;
#pragma unroll
                for (int j = 0; j < NS; j++) {
                    wa += t->K[i][j] * al[j];
                    wb += t->K[i][j] * be[j];
                }
                a0 += al[i] * wa;
                a1 += al[i] * wb;
                a2 += be[i] * wb;
            }
        }
        A0 = a0;
        A1 = R(-2) * a1;
        A2 = a2;
    }

    __device__ __forceinline__ bool valid(double T) const { return T > lo && T <= hi; }

    // a_m and its first two T-derivatives (s = sqrt T, rs = 1/s)
    __device__ __forceinline__ void eval(R T, R s, R rs, R &am, R &am1, R &am2) const
    {
        am = A0 + A1 * s + A2 * T;
        am1 = R(0.5) * A1 * rs + A2;
        am2 = R(-0.25) * A1 * rs * rs * rs;
    }
};

// ------------------------------------------------------------------ NASA-7 mixture
struct Nasa {
    double c[2][5];  // sum_i Y_i R/W_i a_k,i  (cp polynomial), per range
    double a6[2];    // sum_i Y_i R/W_i a6,i
    double rw;       // R/W of the mixture
    double Tmid;
    // mass-specific ideal-gas h and cp at T
    __device__ __forceinline__ void eval(double T, double &h, double &cp) const
    {
        const int r = (T >= Tmid) ? 1 : 0;
        const double c0 = c[r][0], c1 = c[r][1], c2 = c[r][2], c3 = c[r][3], c4 = c[r][4];
        cp = c0 + T * (c1 + T * (c2 + T * (c3 + T * c4)));
        h = T * (c0 + T * (c1 * 0.5 + T * (c2 * (1.0 / 3.0) + T * (c3 * 0.25 + T * (c4 * 0.2))))) + a6[r];
    }
    // the same with d c_p/dT
    __device__ __forceinline__ void eval(double T, double &h, double &cp, double &dcp) const
    {
        const int r = (T >= Tmid) ? 1 : 0;
        const double c0 = c[r][0], c1 = c[r][1], c2 = c[r][2], c3 = c[r][3], c4 = c[r][4];
        cp = c0 + T * (c1 + T * (c2 + T * (c3 + T * c4)));
        dcp = c1 + T * (2.0 * c2 + T * (3.0 * c3 + T * (4.0 * c4)));
        h = T * (c0 + T * (c1 * 0.5 + T * (c2 * (1.0 / 3.0) + T * (c3 * 0.25 + T * (c4 * 0.2))))) + a6[r];
    }
    // mixture coefficients of the ranges r0..r1 from the mass fractions y.  The table is read
    // here through the scalar cache each time: left to itself the compiler hoists the loads
    // of ~100 table values to the kernel entry while sinking their use, and keeps them alive
    // in spilled SGPRs across everything in between.
    template <int NS>
    __device__ __forceinline__ void build(const ThermoTab<NS> *tt0, const double (&y)[NS], int r0, int r1)
    {
        const ThermoTab<NS> *tg = tt0;
        asm volatile("" : "+s"(tg));
        const __attribute__((address_space(4))) ThermoTab<NS> *tt =
            (const __attribute__((address_space(4))) ThermoTab<NS> *)tg;
#pragma unroll
        for (int r = 0; r < 2; r++) {
            if (r < r0 || r > r1) continue;
#pragma unroll
            for (int k = 0; k < 5; k++) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < NS; i++) s += y[i] * tt->cp[r][k][i];
                c[r][k] = s;
            }
            double s6 = 0.0;
#pragma unroll
            for (int i = 0; i < NS; i++) s6 += y[i] * tt->a6[r][i];
            a6[r] = s6;
        }
        double w = 0.0;
#pragma unroll
        for (int i = 0; i < NS; i++) w += y[i] * tt->RW[i];
        rw = w;
        Tmid = tt->Tmid;
    }
};

// ------------------------------------------------------------------ Chung transport
// Chung et al. (1988) viscosity coefficients E_i = a + b omega + c mu_r^4 + d kappa.
constexpr double kChungE[10][4] = {
    {6.324, 50.412, -51.680, 1189.0},      {1.210e-3, -1.154e-3, -6.257e-3, 0.03728},
    {5.283, 254.209, -168.48, 3898.0},     {6.623, 38.096, -8.464, 31.42},
    {19.745, 7.630, -14.354, 31.53},       {-1.900, -12.537, 4.985, -18.15},
    {24.275, 3.450, -11.291, 69.35},       {0.7972, 1.117, 0.01235, -4.117},
    {-0.2382, 0.06770, -0.8163, 4.025},    {0.06863, 0.3479, 0.5926, -0.727}};
// Chung et al. (1988) conductivity coefficients B_i.
constexpr double kChungB[7][4] = {
    {2.4166, 0.74824, -0.91858, 121.72},   {-0.50924, -1.5094, -49.991, 69.983},
    {6.6107, 5.6207, 64.760, 27.039},      {14.543, -8.9139, -5.6379, 74.344},
    {0.79274, 0.82019, -0.69369, 6.3173},  {-5.8634, 12.801, 9.5893, 65.529},
    {91.089, 128.11, -54.217, 523.81}};

// Chung's density function G2 for coefficients c1..c5 (c = pointer to the 5 values), with
// its reciprocal: G2 = num/S and 1/G2 = S/num from the one reciprocal 1/(num S).
template <class PM>
__device__ __forceinline__ void chung_G2(typename PM::R y, typename PM::R G1, typename PM::R iy,
                                         const typename PM::R *c, const double *e2, typename PM::R &G2,
                                         typename PM::R &iG2)
{
    using R = typename PM::R;
    R t1 = c[0] * (-PM::expm1_(-c[3] * y)) * iy;
    R num = t1 + c[1] * G1 * PM::exp_(c[4] * y, e2) + c[2] * G1;
    const R S = c[0] * c[3] + c[1] + c[2];
    const R r = PM::div(R(1), num * S);
    G2 = num * num * r;
    iG2 = S * S * r;
}

template <class PM, int NS>
__device__ __forceinline__ typename PM::R qform(const typename PM::R (&C)[NS][NS],
                                                const typename PM::R (&X)[NS])
{
    using R = typename PM::R;
    R s = 0;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        R w = 0;
#pragma unroll
        for (int j = i; j < NS; j++) w += C[i][j] * X[j];
        s += X[i] * w;
    }
    return s;
}

// mu [Pa s] and lambda [W/(m K)] at T, molar density rhom [mol/m^3], ideal-gas molar Cv.
// The pseudo-mixture quantities are rearranged with exact identities so that few divisions
// and square roots remain: sigma_m^3 = s3 gives Vc_m = s3/0.809^3 and Vc_m Tc_m =
// 1.2593 es3/0.809^3 without the cube root, sqrt(M_m) is the quotient mq itself, one
// reciprocal square root gives sqrt(T) and 1/T and another sqrt(Tc_m) and 1/Tc_m, and
// independent reciprocals are taken in pairs (1/a = b/(ab), 1/b = a/(ab)).
template <class PM, int NS>
__device__ __forceinline__ void chung(const MixTab<typename PM::R, NS> *__restrict__ t0,
                                      const typename PM::R (&X)[NS], typename PM::R T,
                                      typename PM::R rhom, typename PM::R Cv, bool want_mu,
                                      bool want_lam, double *omu, double *olam, const double *e2)
{
    using R = typename PM::R;
    const MixTab<R, NS> *__restrict__ t = t0;
    const R rsT = PM::rsqrt_(T);
    const R sT = T * rsT;
    const R iT = rsT * rsT;
    // mole-fraction-averaged low-pressure viscosity, sum_i X_i mu0_i/Omega_v,i, accumulated
    // as one numerator over one denominator (each Omega_v lies in about [0.5, 3]) so that a
    // single division serves every species; T*^-0.14874 is shared by all species
    const R Tp = PM::exp_(R(-0.14874) * PM::log_(T), e2);
    R en = 0, ed = 1;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        R ts = t->tsc[i] * T;
        R om = t->tsp[i] * Tp + R(0.52487) * PM::exp_(R(-0.77320) * ts, e2) +
               R(2.16178) * PM::exp_(R(-2.43787) * ts, e2);
        en = en * om + ed * (X[i] * t->mu0A[i]);
        ed = ed * om;
    }
    const R eta0 = sT * PM::div(en, ed);
    // pseudo-mixture parameters (Chung's mixing rules; see MixTab for the factorisation)
    R sp = 0, sq = 0, swp = 0, sm = 0, sk = 0;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        sp += X[i] * t->cp_p[i];
        sq += X[i] * t->cp_q[i];
        swp += X[i] * t->cp_wp[i];
        sm += X[i] * t->cp_m[i];
        sk += X[i] * t->cp_k[i];
    }
    const R s3 = sp * sp;                         // sigma_m^3
    const R es3 = sq * sq;                        // (eps/k)_m sigma_m^3
    const R ws3 = swp * sp;
    const R esm = qform<PM, NS>(t->ESM, X);
    const R mu4 = sm * sm;
    const R km = sk * sk;
    const R rpq = PM::div(R(1), sp * sq);
    const R isp = sq * rpq, isq = sp * rpq;
    const R is3 = isp * isp;
    const R ies3 = isq * isq;
    const R sgm = PM::cbrt_(s3);                  // sigma_m
    const R em = es3 * is3;                       // (eps/k)_m
    const R mq = esm * sgm * ies3;                // sqrt(M_m) = esm/((eps/k)_m sigma_m^2)
    const R wm = ws3 * is3;
    const R iVc23 = R(0.809 * 0.809) * sgm * is3; // Vc_m^(-2/3) = 0.809^2/sigma_m^2, mol^(2/3)/cm^2
    const R Tcm = R(1.2593) * em;
    const R rsTc = PM::rsqrt_(Tcm);
    const R sTc = Tcm * rsTc;
    // mu_rm^4 = (131.3 mu_m)^4/(Vc_m Tc_m)^2 with mu_m^4 = s3 mu4
    const R mr4 = R(131.3 * 131.3 * 131.3 * 131.3 * (0.809 * 0.809 * 0.809) * (0.809 * 0.809 * 0.809) /
                    (1.2593 * 1.2593)) * s3 * mu4 * ies3 * ies3;
    const R y = rhom * s3 * R(1e-6 / (6.0 * 0.809 * 0.809 * 0.809));   // rho Vc_m/6
    const R om1 = R(1) - y;
    const R om13 = om1 * om1 * om1;
    const R ry = PM::div(R(1), y * om13);
    const R iy = om13 * ry;
    const R G1 = (R(1) - R(0.5) * y) * y * ry;
    if (want_mu) {
        R E[10];
#pragma unroll
        for (int i = 0; i < 10; i++)
            E[i] = R(kChungE[i][0]) + R(kChungE[i][1]) * wm + R(kChungE[i][2]) * mr4 + R(kChungE[i][3]) * km;
        R G2, iG2;
        chung_G2<PM>(y, G1, iy, E, e2, G2, iG2);
        const R its = em * iT;  // 1/T*, T* = T/(eps/k)_m
        const R muss = E[6] * y * y * G2 * PM::exp_(E[7] + E[8] * its + E[9] * its * its, e2);
        const R mu = eta0 * (iG2 + E[5] * y) + R(36.344e-7) * muss * mq * sTc * iVc23;
        *omu = (double)mu;
    }
    if (want_lam) {
        R Bc[7];
#pragma unroll
        for (int i = 0; i < 7; i++)
            Bc[i] = R(kChungB[i][0]) + R(kChungB[i][1]) * wm + R(kChungB[i][2]) * mr4 + R(kChungB[i][3]) * km;
        R G2, iG2;
        chung_G2<PM>(y, G1, iy, Bc, e2, G2, iG2);
        const R Tr = T * rsTc * rsTc;
        const R al = Cv * R(1.0 / kR) - R(1.5);
        const R be = R(0.7862) - R(0.7109) * wm + R(1.3168) * wm * wm;
        const R Zr = R(2.0) + R(10.5) * Tr * Tr;
        const R pn = R(0.215) + R(0.28288) * al - R(1.061) * be + R(0.26665) * Zr;
        const R pd = R(0.6366) + be * Zr + R(1.061) * al * be;
        const R rpm = PM::div(R(1), pd * mq);
        const R psi = R(1) + al * pn * mq * rpm;
        const R imq = pd * rpm;
        const R iMkg = R(1e3) * imq * imq;       // 1/M_m in mol/kg
        // 3.586e-3 sqrt(Tc_m/M_m[kg/mol])/Vc_m^(2/3); 0.1133992768936381 = 3.586e-3/sqrt(1e-3)
        const R q = R(0.1133992768936381) * sTc * imq * iVc23;
        const R lam = R(31.2) * eta0 * psi * iMkg * (iG2 + Bc[5] * y) + q * Bc[6] * y * y * sT * rsTc * G2;
        *olam = (double)lam;
    }
}

// ------------------------------------------------------------------ cubic (double)
// Eq. (1) as a cubic in Z: Z^3 + c2 Z^2 + c1 Z + c0 = 0.  Only the extreme roots matter for
// the phase choice, so the largest root is taken directly (Cardano's real root when the
// discriminant is positive, else the largest trigonometric root 2 r cos(phi/3)), polished by
// Newton on the cubic, and the cubic is deflated by it to a quadratic whose two roots, when
// real, are the smaller pair (each polished on the full cubic).  One transcendental chain
// per cell instead of three cosines and three polishes; the trigonometric start is taken
// in single precision and polished to double.
struct Cubic {
    double c2, c1, c0;
    __device__ __forceinline__ double f(double x) const { return ((x + c2) * x + c1) * x + c0; }
    __device__ __forceinline__ double fp(double x) const { return (3.0 * x + 2.0 * c2) * x + c1; }
    // one guarded Newton step (skipped if it would move the root by more than 0.1 %)
    __device__ __forceinline__ double polish(double x) const
    {
        const double d = fp(x);
        if (d != 0.0) {
            const double dx = f(x) * fm::rcp(d);
            if (fabs(dx) < 1e-3 * fabs(x) + 1e-12) return x - dx;
        }
        return x;
    }
};

// Roots of Eq. (1) in ascending order: z[2] is the largest; z[0] <= z[1] are the deflated
// pair when the cubic has three real roots (then 3 is returned), else 1.
__device__ __forceinline__ int cubic_roots(double A, double B, double z[3])
{
    Cubic cb;
    cb.c2 = B - 1.0;
    cb.c1 = A - 3.0 * B * B - 2.0 * B;
    cb.c0 = -(A * B - B * B - B * B * B);
    const double sh = cb.c2 * (1.0 / 3.0);
    const double p = cb.c1 - cb.c2 * sh;
    const double q = (2.0 * cb.c2 * cb.c2 * cb.c2 - 9.0 * cb.c2 * cb.c1) * (1.0 / 27.0) + cb.c0;
    const double D = 0.25 * q * q + p * p * p * (1.0 / 27.0);
    double zx;
    int nr;
    if (D > 0.0) {
        const double C = -0.5 * q - copysign(sqrt(D), q);
        const double t = cbrt(C);
        zx = ((t != 0.0) ? t - p * fm::rcp(3.0 * t) : 0.0) - sh;
        nr = 1;
    } else {
        const double r = sqrt(-p * (1.0 / 3.0));
        double arg = (r > 0.0) ? -0.5 * q * fm::rcp(r * r * r) : 0.0;
        arg = fmin(1.0, fmax(-1.0, arg));
        // cos(arccos(arg)/3) in single precision (the hardware cosine: 26 instructions
        // against 241 for the double-precision pair) is a start good to ~1e-6; the Newton
        // polish below carries it to double.  Where the two larger roots nearly coincide
        // (arg -> -1) arccos amplifies the rounding of arg, and double precision is kept.
        const double c = (arg > -0.999) ? (double)__cosf(acosf((float)arg) * (1.0f / 3.0f))
                                        : cos(acos(arg) * (1.0 / 3.0));
        zx = 2.0 * r * c - sh;
        nr = 3;
    }
    zx = cb.polish(cb.polish(cb.polish(zx)));
    z[2] = zx;
    if (nr == 3) {
        // Z^3 + c2 Z^2 + c1 Z + c0 = (Z - zx)(Z^2 + b1 Z + b0)
        const double b1 = cb.c2 + zx;
        const double b0 = cb.c1 + zx * b1;
        const double sd = sqrt(fmax(b1 * b1 - 4.0 * b0, 0.0));
        const double qq = -0.5 * (b1 + copysign(sd, b1));
        const double za = qq, zb = (qq != 0.0) ? b0 * fm::rcp(qq) : 0.0;
        z[0] = cb.polish(cb.polish(fmin(za, zb)));
        z[1] = cb.polish(cb.polish(fmax(za, zb)));
    }
    return nr;
}

// Residual Gibbs energy g_dep/RT = Z - 1 - ln(Z - B) - A/(2 sqrt2 B) ln[(Z + (1+sqrt2)B)/(Z + (1-sqrt2)B)]
// in single precision with the hardware base-2 logarithm (its arguments are normal numbers
// here): it only sets the width of the tie band below.
__device__ __forceinline__ float gdep_RT_f(double Z, float c, double B)
{
    const float q = (float)(Z + (1.0 + kSqrt2) * B) * __builtin_amdgcn_rcpf((float)(Z + (1.0 - kSqrt2) * B));
    return (float)(Z - 1.0) - 0.6931472f * (__builtin_amdgcn_logf((float)(Z - B)) + c * __builtin_amdgcn_logf(q));
}

// Z of the stable phase at (A, B): the physical roots are those above B; of the smallest
// and the largest, the one of lower residual Gibbs energy (a tie within
// 1e-12 max(1, |g_l|, |g_v|) takes the vapour-like root).  NaN if there is no physical root.
// Sets THREE_ROOT / GIBBS_TIE in st.  The difference g_l - g_v is taken in one expression
// (two logarithms of ratios instead of four logarithms, and no cancellation between them).
__device__ __forceinline__ double stable_root(double A, double B, uint8_t &st)
{
    double z[3];
    const int nr = cubic_roots(A, B, z);
    const double zv = z[2];
    if (!(zv > B)) return __builtin_nan("");
    if (nr == 1) return zv;
    const int np = 1 + (z[1] > B ? 1 : 0) + (z[0] > B ? 1 : 0);
    if (np == 1) return zv;
    const double zl = (z[0] > B) ? z[0] : z[1];
    if (np == 3) st |= PROPS_ST_THREE_ROOT;
    const double c = A * fm::rcp(2.0 * kSqrt2 * B);
    const double lp = zl + (1.0 + kSqrt2) * B, lm = zl + (1.0 - kSqrt2) * B;
    const double vp = zv + (1.0 + kSqrt2) * B, vm = zv + (1.0 - kSqrt2) * B;
    const double dg = (zl - zv) - fm::log((zl - B) * fm::rcp(zv - B)) - c * fm::log((lp * vm) * fm::rcp(lm * vp));
    const float cf = (float)c;
    const double tie = 1e-12 * (double)fmaxf(1.0f, fmaxf(fabsf(gdep_RT_f(zl, cf, B)), fabsf(gdep_RT_f(zv, cf, B))));
    if (fabs(dg) <= tie) {
        st |= PROPS_ST_GIBBS_TIE;
        return zv;
    }
    return (dg < 0.0) ? zl : zv;
}

// ------------------------------------------------------------------ the kernel
// Look-ahead stop of the (h, P, Y) inversion: the iteration also ends when the error that
// quadratic convergence predicts after the last step is below kStopAhead rtol T (with
// rtol = 1e-10, 1e-15 relative: rounding level).
constexpr double kStopAhead = 1e-5;
// Look-ahead stop of the (rho, e, Y) inversion: after two consecutive Chebyshev steps d1, d,
// cubic convergence (error e' ~ M e^3, with M ~ d / d1^3 from the two steps) predicts the error
// left after the last step as d^4 / d1^3; the iteration ends once that is below
// kStopAheadCubic rtol T, three orders of magnitude inside the (h, P, Y) bound, so that an
// estimate of M a thousand times too small still leaves the result at rounding level.
constexpr double kStopAheadCubic = 1e-8;
// Minimum waves per SIMD the register allocation must allow (1: the compiler's choice;
// forcing 4 or 5 for the 8-species FP64 kernel spills and measured slower).  The (h, P, Y)
// kernels, left to themselves at 185-213 VGPRs (2 waves), are held to 3 waves: a spill of
// a few values to scratch, mixed precision 3 % faster, double precision unchanged.
#ifndef PR_WAVES_PER_EU
#define PR_WAVES_PER_EU 1
#endif
#ifndef PR_HPY_WAVES
#define PR_HPY_WAVES 3
#endif
// OUTS selects optional output groups at compile time, so that a launch carries only the
// code (and the register pressure) of what it writes: bit 0 the transport model (mu,
// lambda, alpha), bit 1 the solver outputs (psi, alpha, h_i/RT).
constexpr int kOutTransport = 1, kOutSolver = 2;
// Threads per block.  Single-wave blocks let each SIMD take new work as soon as one of its
// waves ends, which measured 6 % faster for (P, T, Y) and 2 % for the mixed-precision
// inversions; the double-precision (rho, e, Y) kernel measured 1.6 % faster with 256.
template <int MODE, int PREC>
constexpr int kPRBlock = (PREC == PROPS_FP64 && MODE != PROPS_PTY) ? 256 : 64;
// Largest cell count of a launch, the same for every mode: a dispatch holds at most
// 2^32 - 1 work-items (its grid size is a 32-bit count of work-items), and 2^32 - 256 is
// the largest multiple of both block sizes below that.
constexpr int64_t kPRMaxCells = 0x100000000LL - 256;
template <int NS, int MODE, int PREC, int OUTS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == PROPS_HPY ? PR_HPY_WAVES : PR_WAVES_PER_EU))) void pr_kernel(const ThermoTab<NS> *__restrict__ tt,
                                                 const MixTab<double, NS> *__restrict__ tmd,
                                                 const MixTab<float, NS> *__restrict__ tmf,
                                                 PRArgs a)
{
    using PM = typename std::conditional<PREC == PROPS_FP64, P64, P32>::type;
    using R = typename PM::R;
    constexpr bool TRANSPORT = (OUTS & kOutTransport) != 0;
    constexpr bool SOLVER = (OUTS & kOutSolver) != 0;
    const MixTab<R, NS> *__restrict__ tm;
    if constexpr (PREC == PROPS_FP64) tm = tmd; else tm = tmf;

    // the double-precision transport's exponentials read 2^(j/64) from LDS (staged before
    // any lane leaves; one entry per thread of the first 64)
    __shared__ double e2s[64];
    static_assert(kPRBlock<MODE, PREC> >= 64, "the table is staged one entry per thread");
    if constexpr (TRANSPORT && PREC == PROPS_FP64) {
        if (threadIdx.x < 64) e2s[threadIdx.x] = tt->exp2j[threadIdx.x];
        __syncthreads();
    }

    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.idx) {
        if (k >= *a.count) return;
        k = a.idx[k];
        if (k < 0 || k >= a.n) return;   // a list entry outside the arrays is never evaluated
    } else if (k >= a.n) {
        return;
    }
    const int64_t n = a.ldy;   // species-row stride of Y and hRT
    // mixing build over the pairs i < j (see MixQuad::build) in single precision and in the
    // (P, T, Y) kernels (measured: (P, T, Y) with transport 3 % faster; the double-precision
    // (rho, e, Y) and (h, P, Y) kernels 12 % and 1.5 % slower, so they keep the full mat-vecs)
    constexpr bool kTriMix = (PREC == PROPS_MIXED) || (MODE == PROPS_PTY);

    // ---- composition and input checks (inputs are read once and outputs written once: both
    // go through non-temporal loads and stores, measured 4-8 % faster than cached ones)
    double y[NS];
    double sy = 0.0, syw = 0.0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        y[i] = (i < a.ns) ? __builtin_nontemporal_load(a.Y + (int64_t)i * n + k) : 0.0;
        bad |= !(y[i] >= -1e-12);
        sy += y[i];
        syw += y[i] * tt->invW[i];
    }
    bad |= !(fabs(sy - 1.0) <= 1e-6);
    const double in0 = __builtin_nontemporal_load(a.in0 + k), in1 = __builtin_nontemporal_load(a.in1 + k);
    if (MODE == PROPS_PTY) bad |= !(in0 > 0.0) || !(in1 > 0.0);
    else if (MODE == PROPS_RHOEY) bad |= !(in0 > 0.0) || !(in1 == in1);
    else bad |= !(in0 == in0) || !(in1 > 0.0);
    const double W = fm::rcp(syw);
    double X[NS];
    R Xr[NS];
    double bm = 0.0;
#pragma unroll
    for (int i = 0; i < NS; i++) {
        X[i] = y[i] * tt->invW[i] * W;
        Xr[i] = (R)X[i];
        bm += X[i] * tt->b[i];
    }

    uint8_t st = a.st_or;
    const double nan = __builtin_nan("");
    double T = nan, P = nan, v = nan;
    double am = 0, am1 = 0, am2 = 0;
    double Lv = 0.0;   // (rho, e, Y): the departure log at the fixed v, reused by the epilogue
    Nasa ig;
    // the inversions evaluate the ideal gas at many T: both NASA ranges up front; the
    // (P, T, Y) path needs one range, once, and builds it where it is used
    if (MODE != PROPS_PTY && !bad) ig.build<NS>(tt, y, 0, 1);

    if (MODE == PROPS_HPY && !bad) {
        // ---- (h, P, Y): bracketed Newton on h(T) at fixed P, the cubic in every evaluation
        P = in1;
        const double hstar = in0;
        const double iP = fm::rcp(P);
        double lo = kTlo, hi = kThi;
        T = kThi;
        if (a.Tg) {
            const double g = a.Tg[k];
            if (g > kTlo && g < kThi) T = g;
        }
        bool fin = false, conv = false, lastN = false, lastN2 = false;
        double dT1 = __builtin_inf(), dT2 = __builtin_inf();   // sizes of the last two steps
        int it = 0;
        const double rtol = (PREC == PROPS_FP64) ? a.rtol : fmax(a.rtol, 1e-6);
        MixQuad<PM, NS, kTriMix> mq;
        mq.build(tm, Xr, T);
        for (; it < a.maxit; it++) {
            if (!mq.valid(T)) mq.build(tm, Xr, T);
            const double rsT = fm::rsqrt(T), sT = T * rsT;
            R ram, ram1, ram2;
            mq.eval((R)T, (R)sT, (R)rsT, ram, ram1, ram2);
            const double RT = kR * T;
            const double iRT = fm::rcp(RT);
            const double A = (double)ram * P * iRT * iRT;
            const double B = bm * P * iRT;
            uint8_t st_dummy = 0;
            const double Z = stable_root(A, B, st_dummy);
            const double vv = Z * RT * iP;
            double h_ig, cp_ig;
            ig.eval(T, h_ig, cp_ig);
            // departures at (v, T): molar h_dep and the real-fluid c_p (the slope dh/dT at P)
            const R rv = (R)vv, rb = (R)bm, rT = (R)T;
            const R rden = rv * rv + R(2) * rb * rv - rb * rb, rvb = rv - rb;
            const R L = PM::log_(PM::div(rv + R(1.0 + kSqrt2) * rb, rv + R(1.0 - kSqrt2) * rb));
            const R Lb = PM::div(L, R(2.0 * kSqrt2) * rb);
            const R edep = (rT * ram1 - ram) * Lb;
            const R cvdep = rT * ram2 * Lb;
            const R dPdT = PM::div(R(kR), rvb) - PM::div(ram1, rden);
            const R dPdv = -PM::div((R)RT, rvb * rvb) + PM::div(R(2) * ram * (rv + rb), rden * rden);
            const R cvm = (R)(W * (cp_ig - ig.rw)) + cvdep;
            const R cpm = cvm - PM::div(rT * dPdT * dPdT, dPdv);
            const double hdep = (double)edep + P * vv - RT;
            const double r = h_ig + hdep * syw - hstar;
            const double rp = (double)cpm * syw;
            if (r > 0.0) hi = T;
            else if (r < 0.0) lo = T;
            else { conv = true; break; }
            // Newton step when it stays in the closed bracket and at least halves the step
            // taken two iterations before (else Newton can cycle where the slope varies
            // strongly, as near pseudo-boiling); otherwise bisection.  A Newton step below
            // rtol ends the iteration: convergence is quadratic, so the updated T is exact
            // to rounding.  So does the third of three Newton steps d2, d1, d whose
            // contraction rates d1/d2^2 and d/d1^2 agree within a factor 4 (the quadratic
            // regime, away from the kinks of h(T) at a phase-choice switch, the NASA range
            // boundary or a sign change in the mixing sum) once the error left behind it,
            // about d^3/d1^2, is below kStopAhead rtol T.  After a small bisection step one
            // more (polishing) step is taken, which never bisects: a converged T whose step
            // rounds to nothing sits on a bracket end, and bisecting there would throw it away.
            double Tn = T - r * fm::rcp(rp);
            const bool newton = (rp > 0.0) && (Tn >= lo && Tn <= hi) && (fabs(Tn - T) <= 0.5 * dT2);
            if (!newton) Tn = fin ? T : 0.5 * (lo + hi);
            const double dT = Tn - T, adT = fabs(dT);
            const double d13 = dT1 * dT1 * dT1, r3 = adT * dT2 * dT2;   // r3/d13: ratio of the rates
            const bool ahead = newton && lastN && lastN2 && r3 >= 0.25 * d13 && r3 <= 4.0 * d13 &&
                               adT * adT * adT <= kStopAhead * rtol * Tn * dT1 * dT1;
            lastN2 = lastN;
            lastN = newton;
            dT2 = dT1;
            dT1 = adT;
            T = Tn;
            if (fin) { conv = true; break; }
            if (adT <= rtol * T || ahead) {
                if (newton) { conv = true; break; }
                fin = true;
            }
        }
        if (a.iters) a.iters[k] = (uint8_t)min(it + (conv ? 1 : 0), 255);
        if (!conv) st |= PROPS_ST_NEWTON_MAXIT;
        if (T <= kTlo * (1.0 + 1e-9) || T >= kThi * (1.0 - 1e-9)) {
            st |= PROPS_ST_BRACKET;
            bad = true;
        }
    }
    if ((MODE == PROPS_PTY || MODE == PROPS_HPY) && !bad) {
        // ---- (P, T, Y): cubic in Z with Gibbs selection
        if (MODE == PROPS_PTY) {
            P = in0;
            T = in1;
        }
        MixQuad<PM, NS, kTriMix> mq;
        mq.build(tm, Xr, T);
        const double rsT = fm::rsqrt(T), sT = T * rsT;
        R ram, ram1, ram2;
        mq.eval((R)T, (R)sT, (R)rsT, ram, ram1, ram2);
        am = ram, am1 = ram1, am2 = ram2;
        const double RT = kR * T;
        const double iRT = fm::rcp(RT);
        const double A = am * P * iRT * iRT;
        const double B = bm * P * iRT;
        const double Z = stable_root(A, B, st);
        if (!(Z == Z)) bad = true;
        v = Z * RT * fm::rcp(P);
    } else if (MODE == PROPS_RHOEY && !bad) {
        // ---- (rho, e, Y): bracketed Chebyshev (third-order Newton) iteration on e(T) at fixed v
        v = W * fm::rcp(in0);
        if (!(v > bm)) {
            bad = true;
        } else {
            const double estar = in1;
            const double L = fm::log((v + (1.0 + kSqrt2) * bm) * fm::rcp(v + (1.0 - kSqrt2) * bm));
            Lv = L;
            const R Lw = (R)(L * fm::rcp(2.0 * kSqrt2 * bm) * syw);  // departure (per mole) -> J/kg factor
            double lo = kTlo, hi = kThi;
            T = kThi;
            if (a.Tg) {
                const double g = a.Tg[k];
                if (g > kTlo && g < kThi) T = g;
            }
            bool fin = false, conv = false, lastN = false;
            double dT1 = __builtin_inf(), dT2 = __builtin_inf();   // sizes of the last two steps
            int it = 0;
            // With single-precision departures the residual carries ~1e-7 relative noise,
            // so the step criterion is held at 1e-6 there (the double path keeps rtol).
            const double rtol = (PREC == PROPS_FP64) ? a.rtol : fmax(a.rtol, 1e-6);
            MixQuad<PM, NS, kTriMix> mq;
            mq.build(tm, Xr, T);
            for (; it < a.maxit; it++) {
                if (!mq.valid(T)) mq.build(tm, Xr, T);
                const double rsT = fm::rsqrt(T), sT = T * rsT;
                R ram, ram1, ram2;
                mq.eval((R)T, (R)sT, (R)rsT, ram, ram1, ram2);
                double h_ig, cp_ig, dcp_ig;
                ig.eval(T, h_ig, cp_ig, dcp_ig);
                const double edep = (double)(((R)T * ram1 - ram) * Lw);
                const double cvdep = (double)((R)T * ram2 * Lw);
                const double r = h_ig - ig.rw * T + edep - estar;
                const double rp = cp_ig - ig.rw + cvdep;
                // d c_v/dT: with a_m'' proportional to T^(-3/2) within the mixing piece,
                // d(T a_m'')/dT = -a_m''/2
                const double rpp = dcp_ig - 0.5 * (double)(ram2 * Lw);
                if (r > 0.0) hi = T;
                else if (r < 0.0) lo = T;
                else { conv = true; break; }
                // Chebyshev's third-order step d (1 + q), d = r/r' the Newton step and
                // q = r r''/(2 r'^2) (the plain Newton step where |q| > 1/2), taken when it
                // stays in the closed bracket and at least halves the step taken two
                // iterations before (else the iteration can cycle where the slope varies
                // strongly, as near pseudo-boiling); otherwise bisection.  Such a step below
                // rtol ends the iteration: convergence is cubic, so the updated T is exact to
                // rounding.  After a small bisection step one more (polishing) step is taken,
                // which never bisects: a converged T whose step rounds to nothing sits on a
                // bracket end, and bisecting there would throw it away.  So does the second of two
                // Chebyshev steps once the error it predicts, d^4 / d1^3, is below kStopAheadCubic
                // rtol T.
                const double irp = fm::rcp(rp);
                const double dN = r * irp;
                const double q = 0.5 * dN * rpp * irp;
                double Tn = T - ((fabs(q) <= 0.5) ? dN * (1.0 + q) : dN);
                const bool newton = (rp > 0.0) && (Tn >= lo && Tn <= hi) && (fabs(Tn - T) <= 0.5 * dT2);
                if (!newton) Tn = fin ? T : 0.5 * (lo + hi);
                const double dT = Tn - T, adT = fabs(dT);
                const double a2 = adT * adT;
                const bool ahead = newton && lastN && a2 * a2 <= kStopAheadCubic * rtol * Tn * dT1 * dT1 * dT1;
                lastN = newton;
                dT2 = dT1;
                dT1 = adT;
                T = Tn;
                if (fin) { conv = true; break; }
                if (adT <= rtol * T || ahead) {
                    if (newton) { conv = true; break; }
                    fin = true;
                }
            }
            if (a.iters) a.iters[k] = (uint8_t)min(it + (conv ? 1 : 0), 255);
            if (!conv) st |= PROPS_ST_NEWTON_MAXIT;
            if (T <= kTlo * (1.0 + 1e-9) || T >= kThi * (1.0 - 1e-9)) {
                st |= PROPS_ST_BRACKET;
                bad = true;
            } else {
                if (!mq.valid(T)) mq.build(tm, Xr, T);
                const double rsT = fm::rsqrt(T), sT = T * rsT;
                R ram, ram1, ram2;
                mq.eval((R)T, (R)sT, (R)rsT, ram, ram1, ram2);
                am = ram, am1 = ram1, am2 = ram2;
                const double den = v * v + 2.0 * bm * v - bm * bm;
                P = kR * T * fm::rcp(v - bm) - am * fm::rcp(den);
            }
        }
    }

    if (bad) {
        if (!(st & PROPS_ST_BRACKET)) st |= PROPS_ST_NONPHYS;
        st &= (PROPS_ST_NONPHYS | PROPS_ST_BRACKET | PROPS_ST_NEWTON_MAXIT | a.st_or);
        if (a.oT) a.oT[k] = nan;
        if (a.oP) a.oP[k] = nan;
        if (a.oZ) a.oZ[k] = nan;
        if (a.orho) a.orho[k] = nan;
        if (a.oh) a.oh[k] = nan;
        if (a.oe) a.oe[k] = nan;
        if (a.ocp) a.ocp[k] = nan;
        if (a.oc) a.oc[k] = nan;
        if (a.omu) a.omu[k] = nan;
        if (a.olam) a.olam[k] = nan;
        if constexpr (SOLVER) {
            if (a.opsi) a.opsi[k] = nan;
            if (a.oalpha) a.oalpha[k] = nan;
            if (a.ohRT) {
#pragma unroll
                for (int i = 0; i < NS; i++)
                    if (i < a.ns) a.ohRT[(int64_t)i * n + k] = nan;
            }
        }
        if (a.status) a.status[k] = st;
        return;
    }

    // ---- departure functions and derived properties at (v, T)
    if (MODE == PROPS_PTY) {
        const int r = (T >= tt->Tmid) ? 1 : 0;
        ig.build<NS>(tt, y, r, r);
    }
    double h_ig, cp_ig;
    ig.eval(T, h_ig, cp_ig);
    const double RT = kR * T;
    const double den = v * v + 2.0 * bm * v - bm * bm;
    const double vb = v - bm;
    double h, e, cp, c, psi = nan;
    {
        const R rv = (R)v, rb = (R)bm, rT = (R)T, rden = (R)den, rvb = (R)vb;
        const R ram = (R)am, ram1 = (R)am1, ram2 = (R)am2;
        // v is the input's in (rho, e, Y) mode: its departure log is the one of the iteration
        const R L = (MODE == PROPS_RHOEY) ? (R)Lv
                                          : PM::log_(PM::div(rv + R(1.0 + kSqrt2) * rb, rv + R(1.0 - kSqrt2) * rb));
        const R Lb = PM::div(L, R(2.0 * kSqrt2) * rb);
        const R edep = (rT * ram1 - ram) * Lb;                 // J/mol
        const R cvdep = rT * ram2 * Lb;                        // J/(mol K)
        const R dPdT = PM::div(R(kR), rvb) - PM::div(ram1, rden);
        const R dPdv = -PM::div((R)RT, rvb * rvb) + PM::div(R(2) * ram * (rv + rb), rden * rden);
        const R cvm = (R)(W * (cp_ig - ig.rw)) + cvdep;
        const R cpm = cvm - PM::div(rT * dPdT * dPdT, dPdv);
        const R c2 = -(rv * rv * (R)syw) * PM::div(cpm, cvm) * dPdv;   // 1/W = sum Y_i/W_i
        const double hdep = (double)edep + P * v - RT;
        h = h_ig + hdep * syw;
        e = h_ig - ig.rw * T + (double)edep * syw;
        cp = (double)cpm * syw;
        c = (c2 > R(0)) ? (double)PM::sqrt_(c2) : nan;
        if (!(cvm > R(0))) st |= PROPS_ST_CV_NONPOS;
        // psi = (d rho/d P)_h = -(W/v^2) (dv/dP)_h with, q = (dP/dT)_v/(dP/dv)_T,
        // (dv/dP)_h = 1/(dP/dv)_T + q (v + T q)/C_p  (molar C_p)
        if (SOLVER && a.opsi) {
            const R idPdv = PM::div(R(1), dPdv);
            const R q = dPdT * idPdv;
            const R dvdPh = idPdv + PM::div(q * (rv + rT * q), cpm);
            psi = -(double)dvdPh * W * fm::rcp(v * v);
        }
    }
    if (a.oT) __builtin_nontemporal_store((double)(T), a.oT + k);
    if (a.oP) __builtin_nontemporal_store((double)(P), a.oP + k);
    if (a.oZ) __builtin_nontemporal_store((double)(P * v * fm::rcp(RT)), a.oZ + k);
    // in (rho, e, Y) mode the density is the input; 1/v = rho/W = rho sum Y_i/W_i
    const double iv = (MODE == PROPS_RHOEY) ? in0 * syw : fm::rcp(v);
    if (a.orho) __builtin_nontemporal_store((double)((MODE == PROPS_RHOEY) ? in0 : W * iv), a.orho + k);
    if (a.oh) __builtin_nontemporal_store((double)(h), a.oh + k);
    if (a.oe) __builtin_nontemporal_store((double)(e), a.oe + k);
    if (a.ocp) __builtin_nontemporal_store((double)(cp), a.ocp + k);
    if (a.oc) __builtin_nontemporal_store((double)(c), a.oc + k);
    if (SOLVER && a.opsi) __builtin_nontemporal_store((double)(psi), a.opsi + k);
    if (SOLVER && a.ohRT) {
        // h_i/(R T) = (h_i [J/kg]) (W_i/R) / T, from the pre-scaled NASA coefficients
        const int r = (T >= ig.Tmid) ? 1 : 0;
        const double iT = fm::rcp(T);
#pragma unroll
        for (int i = 0; i < NS; i++) {
            if (i < a.ns) {
                const double hi_ = T * (tt->cp[r][0][i] + T * (tt->cp[r][1][i] * 0.5 + T * (tt->cp[r][2][i] * (1.0 / 3.0) +
                                   T * (tt->cp[r][3][i] * 0.25 + T * (tt->cp[r][4][i] * 0.2))))) + tt->a6[r][i];
                a.ohRT[(int64_t)i * n + k] = hi_ * tt->WR[i] * iT;
            }
        }
    }
    if constexpr (TRANSPORT) {
        double mu = 0, lam = 0;
        chung<PM, NS>(tm, Xr, (R)T, (R)iv, (R)(W * (cp_ig - ig.rw)), a.omu != nullptr,
                      a.olam != nullptr || (SOLVER && a.oalpha != nullptr), &mu, &lam, e2s);
        if (a.omu) __builtin_nontemporal_store((double)(mu), a.omu + k);
        if (a.olam) __builtin_nontemporal_store((double)(lam), a.olam + k);
        if (SOLVER && a.oalpha) __builtin_nontemporal_store((double)(lam * v * fm::rcp(W * cp)), a.oalpha + k);
    }
    if (a.status) a.status[k] = st;
}

// ------------------------------------------------------------------ host launch
template <int NS, int MODE, int PREC, int OUTS>
static int launch_one(const props_mech_s *m, const PRArgs &a, hipStream_t s)
{
    const auto *base = static_cast<const unsigned char *>(m->d_tab);
    const auto *tt = reinterpret_cast<const ThermoTab<NS> *>(base);
    const auto *tmd = reinterpret_cast<const MixTab<double, NS> *>(base + m->off_mixd);
    const auto *tmf = reinterpret_cast<const MixTab<float, NS> *>(base + m->off_mixf);
    if (a.n > kPRMaxCells) return fail(PROPS_ETOOBIG, "props_pr: n = %lld too large", (long long)a.n);
    constexpr int B = kPRBlock<MODE, PREC>;
    const int64_t blocks = (a.n + B - 1) / B;
    hipLaunchKernelGGL((pr_kernel<NS, MODE, PREC, OUTS>), dim3((unsigned)blocks), dim3(B), 0, s, tt, tmd, tmf, a);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

template <int NS, int MODE, int PREC>
static int launch_outs(const props_mech_s *m, int outs, const PRArgs &a, hipStream_t s)
{
    switch (outs) {
        case 0: return launch_one<NS, MODE, PREC, 0>(m, a, s);
        case kOutTransport: return launch_one<NS, MODE, PREC, kOutTransport>(m, a, s);
        case kOutSolver: return launch_one<NS, MODE, PREC, kOutSolver>(m, a, s);
        default: return launch_one<NS, MODE, PREC, kOutTransport | kOutSolver>(m, a, s);
    }
}

template <int NS, int MODE>
static int launch_prec(const props_mech_s *m, int prec, int outs, const PRArgs &a, hipStream_t s)
{
    return (prec == PROPS_FP64) ? launch_outs<NS, MODE, PROPS_FP64>(m, outs, a, s)
                                : launch_outs<NS, MODE, PROPS_MIXED>(m, outs, a, s);
}

template <int NS>
static int dispatch_ns(const props_mech_s *m, int mode, int prec, int outs, const PRArgs &a, hipStream_t s)
{
    if (mode == PROPS_PTY) return launch_prec<NS, PROPS_PTY>(m, prec, outs, a, s);
    if (mode == PROPS_RHOEY) return launch_prec<NS, PROPS_RHOEY>(m, prec, outs, a, s);
    return launch_prec<NS, PROPS_HPY>(m, prec, outs, a, s);
}

static int launch_pr_args(const props_mech_s *m, int mode, int prec, const props_in *in,
                          const props_out *out, int64_t n, int64_t ldy, uint8_t *status, const int *idx,
                          const int *count, uint8_t st_or, hipStream_t stream)
{
    PRArgs a{};
    a.idx = idx;
    a.count = count;
    a.st_or = st_or;
    a.in0 = (mode == PROPS_PTY) ? in->P : (mode == PROPS_RHOEY) ? in->rho : in->h;
    a.in1 = (mode == PROPS_PTY) ? in->T : (mode == PROPS_RHOEY) ? in->e : in->P;
    a.Y = in->Y;
    a.Tg = (mode != PROPS_PTY) ? in->T_guess : nullptr;
    a.oT = out->T, a.oP = out->P, a.oZ = out->Z, a.orho = out->rho, a.oh = out->h;
    a.oe = out->e, a.ocp = out->cp, a.oc = out->c, a.omu = out->mu, a.olam = out->lambda;
    a.opsi = out->psi, a.oalpha = out->alpha, a.ohRT = out->hRT;
    a.status = status;
    a.iters = (mode != PROPS_PTY) ? out->iters : nullptr;
    a.n = n;
    a.ldy = ldy;
    a.ns = m->ns;
    a.maxit = m->maxit;
    a.rtol = m->rtol;
    const int outs = ((out->mu || out->lambda || out->alpha) ? kOutTransport : 0) |
                     ((out->psi || out->alpha || out->hRT) ? kOutSolver : 0);
    switch (m->nsp) {
        case 1: return dispatch_ns<1>(m, mode, prec, outs, a, stream);
        case 2: return dispatch_ns<2>(m, mode, prec, outs, a, stream);
        case 4: return dispatch_ns<4>(m, mode, prec, outs, a, stream);
        default: return dispatch_ns<8>(m, mode, prec, outs, a, stream);
    }
}

int launch_pr(const props_mech_s *m, int mode, int prec, const props_in *in,
              const props_out *out, int64_t n, uint8_t *status, hipStream_t stream)
{
    return launch_pr_args(m, mode, prec, in, out, n, n, status, nullptr, nullptr, 0, stream);
}

int launch_pr_strided(const props_mech_s *m, int mode, int prec, const props_in *in,
                      const props_out *out, int64_t n, int64_t ldy, uint8_t *status, hipStream_t stream)
{
    return launch_pr_args(m, mode, prec, in, out, n, ldy, status, nullptr, nullptr, 0, stream);
}

int launch_pr_indirect(const props_mech_s *m, int mode, int prec, const props_in *in,
                       const props_out *out, int64_t n, int64_t ldy, const int *idx, const int *count,
                       uint8_t *status, uint8_t st_or, hipStream_t stream)
{
    return launch_pr_args(m, mode, prec, in, out, n, ldy, status, idx, count, st_or, stream);
}

}  // namespace props
