// Host build of the kernels' log: maximum error in units of the last place against
// long-double libm over seeded arguments.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>

#include "../../paper_2312_04830_amd/csrc/fastmath.hpp"

static double ulp_err(double got, long double ref)
{
    if (std::isnan(got) && std::isnan((double)ref)) return 0.0;
    const double r = (double)ref;
    if (r == 0.0) return got == 0.0 ? 0.0 : 1e300;
    const double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
    return (double)(std::fabs((long double)got - ref) / u);
}

int main()
{
    std::mt19937_64 g(12345);
    std::uniform_real_distribution<double> ul(-700.0, 700.0);
    double e_log = 0;
    for (int i = 0; i < 2000000; i++) {
        double l = std::exp2(ul(g) * 1.4);
        e_log = std::fmax(e_log, ulp_err(props::fm::log(l), logl((long double)l)));
    }
    // arguments the property kernels meet: log of T and of 1 + small
    for (double T = 50.0; T < 6000.0; T += 0.37) {
        e_log = std::fmax(e_log, ulp_err(props::fm::log(T), logl((long double)T)));
        double z = 1.0 + 1e-6 * T;
        e_log = std::fmax(e_log, ulp_err(props::fm::log(z), logl((long double)z)));
    }
    // exp: normal results, the kernels' arguments (exponents of collision-integral and
    // Chung terms, -800..0 and small positives), and subnormal results by absolute error
    double e_exp = 0, e_sub = 0;
    std::uniform_real_distribution<double> ue(-708.0, 709.0);
    for (int i = 0; i < 2000000; i++) {
        double x = ue(g);
        e_exp = std::fmax(e_exp, ulp_err(props::fm::exp(x), expl((long double)x)));
    }
    for (double x = -60.0; x < 40.0; x += 1.37e-4)
        e_exp = std::fmax(e_exp, ulp_err(props::fm::exp(x), expl((long double)x)));
    for (double x = -745.0; x < -708.5; x += 1e-3)
        e_sub = std::fmax(e_sub, std::fabs((double)((long double)props::fm::exp(x) - expl((long double)x))) / 4.9406564584124654e-324);
    // exp_tab with its table of 2^(j/64) rounded from long double
    double tab[64];
    for (int j = 0; j < 64; j++) tab[j] = (double)exp2l((long double)j / 64.0L);
    double e_tab = 0, e_tsub = 0;
    for (int i = 0; i < 2000000; i++) {
        double x = ue(g);
        e_tab = std::fmax(e_tab, ulp_err(props::fm::exp_tab(x, tab), expl((long double)x)));
    }
    for (double x = -60.0; x < 40.0; x += 1.37e-4)
        e_tab = std::fmax(e_tab, ulp_err(props::fm::exp_tab(x, tab), expl((long double)x)));
    for (double x = -745.0; x < -708.5; x += 1e-3)
        e_tsub = std::fmax(e_tsub, std::fabs((double)((long double)props::fm::exp_tab(x, tab) - expl((long double)x))) / 4.9406564584124654e-324);
    std::printf("log_max_ulp %.3f\n", e_log);
    std::printf("exptab_max_ulp %.3f exptab_sub_max_denorm_ulp %.3f exptab_limits %d\n", e_tab, e_tsub,
                (int)(props::fm::exp_tab(-800.0, tab) == 0.0 && std::isinf(props::fm::exp_tab(710.0, tab)) &&
                      props::fm::exp_tab(0.0, tab) == 1.0));
    std::printf("exp_max_ulp %.3f exp_sub_max_denorm_ulp %.3f\n", e_exp, e_sub);
    std::printf("exp_under_zero %d exp_over_inf %d exp_nan %d exp_zero_one %d\n",
                (int)(props::fm::exp(-800.0) == 0.0), (int)std::isinf(props::fm::exp(710.0)),
                (int)std::isnan(props::fm::exp(NAN)), (int)(props::fm::exp(0.0) == 1.0));
    std::printf("log_neg_nan %d log_zero_nan %d\n", (int)std::isnan(props::fm::log(-1.0)),
                (int)std::isnan(props::fm::log(0.0)));
    return 0;
}
