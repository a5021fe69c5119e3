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
    std::printf("log_max_ulp %.3f\n", e_log);
    std::printf("log_neg_nan %d log_zero_nan %d\n", (int)std::isnan(props::fm::log(-1.0)),
                (int)std::isnan(props::fm::log(0.0)));
    return 0;
}
