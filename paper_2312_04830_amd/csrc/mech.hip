// Mechanism handles: host-side derivation of the device tables, error reporting, and
// the argument checks of props_pr.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>
#include <vector>

#include "props_internal.hpp"
#include "trace.hpp"

namespace props {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

// kappa(omega) of the Peng-Robinson alpha function: the 1976 quadratic, and the 1978
// cubic for heavy components (omega > 0.491).
static double pr_kappa(double w)
{
    if (w <= 0.491) return 0.37464 + 1.54226 * w - 0.26992 * w * w;
    return 0.379642 + 1.48503 * w - 0.164423 * w * w + 0.016666 * w * w * w;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename R, int NS>
static void fill_mix(MixTab<R, NS> &t, const props_species_desc *sp, int ns, const double *kij)
{
    std::memset(&t, 0, sizeof(t));
    double sig[PROPS_MAX_SPECIES], eps[PROPS_MAX_SPECIES], mud[PROPS_MAX_SPECIES];
    for (int i = 0; i < ns; i++) {
        const props_species_desc &s = sp[i];
        double ac = kOmegaA * kR * kR * s.Tc * s.Tc / s.Pc;
        double kap = pr_kappa(s.omega);
        t.sqac[i] = (R)std::sqrt(ac);
        t.k1[i] = (R)(1.0 + kap);
        t.k2[i] = (R)(kap / std::sqrt(s.Tc));
        t.tstar[i] = (R)((kap > 0.0) ? s.Tc * (1.0 + 1.0 / kap) * (1.0 + 1.0 / kap) : HUGE_VAL);
        // Chung's constants use Vc in cm^3/mol and M in g/mol
        double Vc = s.Vc * 1e6, M = s.W * 1e3;
        double mur = 131.3 * s.dipole / std::sqrt(Vc * s.Tc);
        double Fc = 1.0 - 0.2756 * s.omega + 0.059035 * mur * mur * mur * mur + s.kappa;
        t.mu0A[i] = (R)(40.785e-7 * Fc * std::sqrt(M) / std::pow(Vc, 2.0 / 3.0));
        double tsc = 1.2593 / s.Tc;
        t.tsc[i] = (R)tsc;
        t.tsp[i] = (R)(1.16145 * std::pow(tsc, -0.14874));
        sig[i] = 0.809 * std::cbrt(Vc);
        eps[i] = s.Tc / 1.2593;
        mud[i] = s.dipole;
    }
    for (int i = 0; i < ns; i++) {
        for (int j = 0; j < ns; j++) {
            t.K[i][j] = (R)(1.0 - (kij ? kij[i * ns + j] : 0.0));
            if (j < i) continue;
            double f = (i == j) ? 1.0 : 2.0;
            double sij = std::sqrt(sig[i] * sig[j]), eij = std::sqrt(eps[i] * eps[j]);
            double Mi = sp[i].W * 1e3, Mj = sp[j].W * 1e3;
            double Mij = 2.0 * Mi * Mj / (Mi + Mj);
            t.ESM[i][j] = (R)(f * eij * sij * sij * std::sqrt(Mij));
        }
    }
    for (int i = 0; i < ns; i++) {
        const double p = std::pow(sig[i], 1.5);
        t.cp_p[i] = (R)p;
        t.cp_q[i] = (R)(std::sqrt(eps[i]) * p);
        t.cp_wp[i] = (R)(sp[i].omega * p);
        t.cp_m[i] = (R)(mud[i] * mud[i] / p);
        t.cp_k[i] = (R)std::sqrt(sp[i].kappa);
    }
}

template <int NS>
static void fill_thermo(ThermoTab<NS> &t, const props_species_desc *sp, int ns)
{
    std::memset(&t, 0, sizeof(t));
    for (int i = 0; i < ns; i++) {
        const props_species_desc &s = sp[i];
        t.invW[i] = 1.0 / s.W;
        t.RW[i] = kR / s.W;
        t.WR[i] = s.W / kR;
        t.b[i] = kOmegaB * kR * s.Tc / s.Pc;
        for (int k = 0; k < 5; k++) {
            t.cp[0][k][i] = t.RW[i] * s.nasa_lo[k];
            t.cp[1][k][i] = t.RW[i] * s.nasa_hi[k];
        }
        t.a6[0][i] = t.RW[i] * s.nasa_lo[5];
        t.a6[1][i] = t.RW[i] * s.nasa_hi[5];
    }
    t.Tmid = sp[0].Tmid;
    for (int j = 0; j < 64; j++) t.exp2j[j] = (double)exp2l((long double)j / 64.0L);
}

// Chapman-Enskog pair constants.  Lennard-Jones parameters come from the same Chung
// corresponding-states relations as the viscosity (sigma_i = 0.809 Vc_i^(1/3) Angstrom with
// Vc in cm^3/mol, eps_i/k = Tc_i/1.2593) and combine by Lorentz-Berthelot:
// sigma_ij = (sigma_i + sigma_j)/2, eps_ij = sqrt(eps_i eps_j).
template <typename R, int NS>
static void fill_diff(DiffTab<R, NS> &t, const props_species_desc *sp, int ns)
{
    std::memset(&t, 0, sizeof(t));
    constexpr double kB = 1.380649e-23, kNA = 6.02214076e23;   // exact SI values
    const double pi = std::acos(-1.0);
    int p = 0;
    for (int i = 0; i < NS; i++) {
        for (int j = i + 1; j < NS; j++, p++) {
            if (i >= ns || j >= ns) continue;
            const double si = 0.809e-10 * std::cbrt(sp[i].Vc * 1e6), sj = 0.809e-10 * std::cbrt(sp[j].Vc * 1e6);
            const double sij = 0.5 * (si + sj);
            const double eij = std::sqrt((sp[i].Tc / 1.2593) * (sp[j].Tc / 1.2593));
            const double mij = sp[i].W * sp[j].W / ((sp[i].W + sp[j].W) * kNA);
            const double G = 16.0 / 3.0 * sij * sij * std::sqrt(pi * mij / (2.0 * kB * kB * kB));
            t.c0[p] = (R)(1.06036 * G * std::pow(eij, 0.15610));
            t.c1[p] = (R)(0.19300 * G);
            t.c2[p] = (R)(1.03587 * G);
            t.c3[p] = (R)(1.76474 * G);
            t.x1[p] = (R)(-0.47635 / eij);
            t.x2[p] = (R)(-1.52996 / eij);
            t.x3[p] = (R)(-3.89411 / eij);
        }
    }
}

template <int NS>
static int build_tables(props_mech_s *m)
{
    size_t o1 = align256(sizeof(ThermoTab<NS>));
    size_t o2 = o1 + align256(sizeof(MixTab<double, NS>));
    size_t o3 = o2 + align256(sizeof(MixTab<float, NS>));
    size_t o4 = o3 + align256(sizeof(DiffTab<double, NS>));
    size_t bytes = o4 + align256(sizeof(DiffTab<float, NS>));
    std::vector<unsigned char> host(bytes, 0);
    fill_thermo<NS>(*reinterpret_cast<ThermoTab<NS> *>(host.data()), m->sp, m->ns);
    fill_mix<double, NS>(*reinterpret_cast<MixTab<double, NS> *>(host.data() + o1), m->sp, m->ns, m->kij);
    fill_mix<float, NS>(*reinterpret_cast<MixTab<float, NS> *>(host.data() + o2), m->sp, m->ns, m->kij);
    fill_diff<double, NS>(*reinterpret_cast<DiffTab<double, NS> *>(host.data() + o3), m->sp, m->ns);
    fill_diff<float, NS>(*reinterpret_cast<DiffTab<float, NS> *>(host.data() + o4), m->sp, m->ns);
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) return fail(PROPS_ENOMEM, "hipMalloc(%zu) for mechanism tables: %s", bytes, hipGetErrorString(e));
    e = hipMemcpy(d, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(PROPS_EHIP, "hipMemcpy of mechanism tables: %s", hipGetErrorString(e));
    }
    m->d_tab = d;
    m->off_mixd = o1;
    m->off_mixf = o2;
    m->off_diffd = o3;
    m->off_difff = o4;
    m->bytes = bytes;
    return PROPS_OK;
}

}  // namespace props

using namespace props;

extern "C" {

const char *props_last_error(void) { return g_err; }

const char *props_version(void) { return "props-mi355x 0.1 (gfx950)"; }

int props_mech_create(const props_species_desc *sp, int ns, const double *kij, props_mech_t *out)
{
    ApiRange range_("props_mech_create");
    if (!out) return fail(PROPS_EINVAL, "props_mech_create: out is NULL");
    *out = nullptr;
    if (!sp) return fail(PROPS_EINVAL, "props_mech_create: species array is NULL");
    if (ns < 1) return fail(PROPS_EINVAL, "props_mech_create: ns = %d < 1", ns);
    if (ns > PROPS_MAX_SPECIES)
        return fail(PROPS_ETOOBIG, "props_mech_create: ns = %d exceeds %d", ns, PROPS_MAX_SPECIES);
    for (int i = 0; i < ns; i++) {
        const props_species_desc &s = sp[i];
        if (!(s.W > 0) || !(s.Tc > 0) || !(s.Pc > 0) || !(s.Vc > 0) || !(s.Tmid > 0) ||
            !std::isfinite(s.omega) || !(s.dipole >= 0) || !(s.kappa >= 0))
            return fail(PROPS_EINVAL, "props_mech_create: species %d has invalid constants", i);
        if (s.Tmid != sp[0].Tmid)
            return fail(PROPS_EINVAL, "props_mech_create: species %d has Tmid %g != %g (one shared "
                        "NASA range switch is required)", i, s.Tmid, sp[0].Tmid);
    }
    if (kij) {
        for (int i = 0; i < ns; i++)
            for (int j = 0; j < ns; j++) {
                double a = kij[i * ns + j], b = kij[j * ns + i];
                if (!std::isfinite(a) || a != b || (i == j && a != 0.0))
                    return fail(PROPS_EINVAL, "props_mech_create: kij must be finite, symmetric, "
                                "zero on the diagonal (entry %d,%d)", i, j);
            }
    }
    props_mech_s *m = new (std::nothrow) props_mech_s();
    if (!m) return fail(PROPS_ENOMEM, "props_mech_create: out of host memory");
    m->ns = ns;
    std::memcpy(m->sp, sp, sizeof(props_species_desc) * ns);
    for (int i = 0; i < ns * ns; i++) m->kij[i] = kij ? kij[i] : 0.0;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return fail(PROPS_EHIP, "props_mech_create: hipGetDevice failed");
    }
    int nsp = 8;
    for (int p : kPadSizes) if (p >= ns) { nsp = p; break; }
    m->nsp = nsp;
    int rc;
    switch (nsp) {
        case 1: rc = build_tables<1>(m); break;
        case 2: rc = build_tables<2>(m); break;
        case 4: rc = build_tables<4>(m); break;
        default: rc = build_tables<8>(m); break;
    }
    if (rc != PROPS_OK) {
        delete m;
        return rc;
    }
    *out = m;
    return PROPS_OK;
}

void props_mech_destroy(props_mech_t m)
{
    if (!m) return;
    if (m->d_tab) (void)hipFree(m->d_tab);
    delete m;
}

int props_mech_num_species(props_mech_t m) { return m ? m->ns : fail(PROPS_EINVAL, "null mechanism"); }

int props_mech_set_newton(props_mech_t m, int max_iter, double rtol)
{
    if (!m) return fail(PROPS_EINVAL, "props_mech_set_newton: null mechanism");
    if (max_iter < 1 || max_iter > 10000 || !(rtol > 0) || !(rtol < 1))
        return fail(PROPS_EINVAL, "props_mech_set_newton: need 1 <= max_iter <= 10000, 0 < rtol < 1");
    m->maxit = max_iter;
    m->rtol = rtol;
    return PROPS_OK;
}

int props_pr(props_mech_t m, int mode, int prec, const props_in *in, const props_out *out,
             int64_t n, uint8_t *status, void *hip_stream)
{
    ApiRange range_("props_pr");
    if (!m || !in || !out) return fail(PROPS_EINVAL, "props_pr: null mechanism, input or output");
    if (mode != PROPS_PTY && mode != PROPS_RHOEY && mode != PROPS_HPY)
        return fail(PROPS_EINVAL, "props_pr: unknown mode %d", mode);
    if (prec != PROPS_FP64 && prec != PROPS_MIXED) return fail(PROPS_EINVAL, "props_pr: unknown precision %d", prec);
    if (n < 0) return fail(PROPS_EINVAL, "props_pr: n = %lld < 0", (long long)n);
    if (n == 0) return PROPS_OK;
    if (!in->Y) return fail(PROPS_EINVAL, "props_pr: Y is NULL");
    if (mode == PROPS_PTY && (!in->P || !in->T)) return fail(PROPS_EINVAL, "props_pr: PTY mode needs P and T");
    if (mode == PROPS_RHOEY && (!in->rho || !in->e)) return fail(PROPS_EINVAL, "props_pr: RHOEY mode needs rho and e");
    if (mode == PROPS_HPY && (!in->h || !in->P)) return fail(PROPS_EINVAL, "props_pr: HPY mode needs h and P");
    int dev = -1;
    PROPS_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(PROPS_EINVAL, "props_pr: mechanism lives on device %d, current device is %d", m->device, dev);
    return launch_pr(m, mode, prec, in, out, n, status, (hipStream_t)hip_stream);
}

int props_diffusion(props_mech_t m, int prec, const double *P, const double *T, const double *Y,
                    double *D, int64_t n, uint8_t *status, void *hip_stream)
{
    ApiRange range_("props_diffusion");
    if (!m) return fail(PROPS_EINVAL, "props_diffusion: null mechanism");
    if (prec != PROPS_FP64 && prec != PROPS_MIXED)
        return fail(PROPS_EINVAL, "props_diffusion: unknown precision %d", prec);
    if (n < 0) return fail(PROPS_EINVAL, "props_diffusion: n = %lld < 0", (long long)n);
    if (n == 0) return PROPS_OK;
    if (!P || !T || !Y || !D) return fail(PROPS_EINVAL, "props_diffusion: P, T, Y and D are required");
    int dev = -1;
    PROPS_HIP_TRY(hipGetDevice(&dev));
    if (dev != m->device)
        return fail(PROPS_EINVAL, "props_diffusion: mechanism lives on device %d, current device is %d", m->device, dev);
    return launch_diffusion(m, prec, P, T, Y, D, n, status, (hipStream_t)hip_stream);
}

}  // extern "C"
