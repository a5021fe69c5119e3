// Host build of the kernels' exp/expm1/log: maximum error in units of the last place
// against long-double libm over seeded arguments.  Prints one line per function.
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
    std::uniform_real_distribution<double> ue(-700.0, 700.0), us(-0.35, 0.35), um(-20.0, 0.5),
        ul(-700.0, 700.0);
    double e_exp = 0, e_em1 = 0, e_log = 0, e_exps = 0;
    for (int i = 0; i < 2000000; i++) {
        double x = ue(g);
        e_exp = std::fmax(e_exp, ulp_err(props::fm::exp(x), expl((long double)x)));
        double s = us(g);
        e_exps = std::fmax(e_exps, ulp_err(props::fm::exp(s), expl((long double)s)));
        double m = um(g);
        e_em1 = std::fmax(e_em1, ulp_err(props::fm::expm1(m), expm1l((long double)m)));
        double l = std::exp2(ul(g) / 1.0 * 1.4);
        e_log = std::fmax(e_log, ulp_err(props::fm::log(l), logl((long double)l)));
    }
    // arguments the property kernels meet: log of T and of 1 + small; exp of -0.77 T*
    for (double T = 50.0; T < 6000.0; T += 0.37) {
        e_log = std::fmax(e_log, ulp_err(props::fm::log(T), logl((long double)T)));
        double z = 1.0 + 1e-6 * T;
        e_log = std::fmax(e_log, ulp_err(props::fm::log(z), logl((long double)z)));
    }
    std::printf("exp_max_ulp %.3f\nexp_small_max_ulp %.3f\nexpm1_max_ulp %.3f\nlog_max_ulp %.3f\n",
                e_exp, e_exps, e_em1, e_log);
    std::printf("exp_underflow %g exp_nan %d log_neg_nan %d\n", props::fm::exp(-800.0),
                (int)std::isnan(props::fm::exp(NAN)), (int)std::isnan(props::fm::log(-1.0)));
    return 0;
}
