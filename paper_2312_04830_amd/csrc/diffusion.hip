// Mixture-averaged species diffusion coefficients for gfx950 (one lane per cell).
//
// Section 2 closes the species transport with mixture-averaged diffusion coefficients;
// what a lane computes is the low-pressure Chapman-Enskog form of them:
//   binary       D_ij = T^1.5 / (P G_ij Omega_D(T/eps_ij)) with Neufeld's fit of the
//                diffusion collision integral (the pair constants G_ij, eps_ij and the fit's
//                coefficients are folded into DiffTab on the host)
//   mixture      D_i = (1 - Y_i) / sum_{j != i} X_j / D_ij
//                    = (1 - Y_i) T^1.5 sum_k(Y_k/W_k) / (P sum_{j != i} (Y_j/W_j) G_ij Omega_ij),
//                and D_i = 0 where no other species is present (the sum is not positive).
// Takahashi's high-pressure correction of the binary coefficients, which the paper also
// names, is not applied: its correlation chart is not reproduced here.
//
// Each unordered pair is visited once and its term feeds both species' sums.  Per cell:
// one log and one exp for T^-0.15610, three exponentials per pair; FP64 uses the
// table-driven exp of fastmath.hpp (table in LDS), the mixed variant the hardware v_exp_f32.  Memory: P, T,
// Y read and D written once, species-major and unit-stride across a wavefront; the pair
// table (a few hundred values) comes through the scalar cache.
#include <cmath>
#include <type_traits>

#include "fastmath.hpp"
#include "props_internal.hpp"

namespace props {

namespace {

struct D64 {
    using R = double;
    static __device__ __forceinline__ R exp_(R x, const double *e2) { return fm::exp_tab(x, e2); }
    static __device__ __forceinline__ R log_(R x) { return fm::log(x); }
};

struct D32 {
    using R = float;
    static __device__ __forceinline__ R exp_(R x, const double *) { return __expf(x); }
    static __device__ __forceinline__ R log_(R x) { return __logf(x); }
};

struct DiffArgs {
    const double *P, *T, *Y;
    double *D;
    uint8_t *status;
    int64_t n;
    int ns;
};

// one wavefront per block (as the property kernels; the table below is staged one entry per thread)
constexpr int kDiffBlock = 64;

template <int NS, int PREC>
__global__ __launch_bounds__(256) void diffusion_kernel(const ThermoTab<NS> *__restrict__ tt,
                                                        const DiffTab<double, NS> *__restrict__ tdd,
                                                        const DiffTab<float, NS> *__restrict__ tdf,
                                                        DiffArgs a)
{
    using PM = typename std::conditional<PREC == PROPS_FP64, D64, D32>::type;
    using R = typename PM::R;
    const DiffTab<R, NS> *__restrict__ td;
    if constexpr (PREC == PROPS_FP64) td = tdd; else td = tdf;

    // 2^(j/64) for the double-precision exponentials, staged in LDS before any lane leaves
    __shared__ double e2s[64];
    if constexpr (PREC == PROPS_FP64) {
        if (threadIdx.x < 64) e2s[threadIdx.x] = tt->exp2j[threadIdx.x];
        __syncthreads();
    }
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n) return;
    const int64_t n = a.n;

    double y[NS];
    double sy = 0.0, syw = 0.0;
    bool bad = false;
    R yw[NS];
#pragma unroll
    for (int i = 0; i < NS; i++) {
        y[i] = (i < a.ns) ? __builtin_nontemporal_load(a.Y + (int64_t)i * n + k) : 0.0;
        bad |= !(y[i] >= -1e-12);
        sy += y[i];
        const double w = y[i] * tt->invW[i];
        syw += w;
        yw[i] = (R)w;
    }
    bad |= !(fabs(sy - 1.0) <= 1e-6);
    const double P = __builtin_nontemporal_load(a.P + k), T = __builtin_nontemporal_load(a.T + k);
    bad |= !(P > 0.0) || !(T > 0.0);
    if (bad) {
        const double nan = __builtin_nan("");
#pragma unroll
        for (int i = 0; i < NS; i++)
            if (i < a.ns) a.D[(int64_t)i * n + k] = nan;
        if (a.status) a.status[k] = PROPS_ST_NONPHYS;
        return;
    }

    const R Tr = (R)T;
    const R Tm = PM::exp_(R(-0.15610) * PM::log_(Tr), e2s);   // T^-0.15610
    R S[NS];
#pragma unroll
    for (int i = 0; i < NS; i++) S[i] = R(0);
    int p = 0;
    R prev = R(0);
#pragma unroll
    for (int i = 0; i < NS; i++) {
#pragma unroll
        for (int j = i + 1; j < NS; j++, p++) {
            // Re-derive the table pointer for every pair, opaquely and after the previous
            // pair's term, so that the pair's seven constants are loaded where they are
            // used: hoisted to the top, the whole table (up to 196 values) would spill out
            // of the scalar registers.
            const DiffTab<R, NS> *tg = td;
            asm volatile("" : "+s"(tg) : "v"(prev));
            const __attribute__((address_space(4))) DiffTab<R, NS> *t =
                (const __attribute__((address_space(4))) DiffTab<R, NS> *)tg;
            R h = t->c0[p] * Tm;
            h += t->c1[p] * PM::exp_(t->x1[p] * Tr, e2s);
            h += t->c2[p] * PM::exp_(t->x2[p] * Tr, e2s);
            h += t->c3[p] * PM::exp_(t->x3[p] * Tr, e2s);
            S[i] += yw[j] * h;
            S[j] += yw[i] * h;
            prev = h;
        }
    }
    // (1 - Y_i) T^1.5 sum(Y/W) / P, in double for both precisions
    const double f = T * sqrt(T) * syw * fm::rcp(P);
#pragma unroll
    for (int i = 0; i < NS; i++) {
        if (i < a.ns) {
            const double s = (double)S[i];
            __builtin_nontemporal_store((s > 0.0) ? (1.0 - y[i]) * f * fm::rcp(s) : 0.0, a.D + (int64_t)i * n + k);
        }
    }
    if (a.status) a.status[k] = 0;
}

template <int NS, int PREC>
int launch_ns(const props_mech_s *m, const DiffArgs &a, hipStream_t s)
{
    const auto *base = static_cast<const unsigned char *>(m->d_tab);
    const auto *tt = reinterpret_cast<const ThermoTab<NS> *>(base);
    const auto *tdd = reinterpret_cast<const DiffTab<double, NS> *>(base + m->off_diffd);
    const auto *tdf = reinterpret_cast<const DiffTab<float, NS> *>(base + m->off_difff);
    // a dispatch holds at most 2^32 - 1 work-items: n <= 2^32 - 256 (a multiple of the block)
    if (a.n > 0x100000000LL - 256) return fail(PROPS_ETOOBIG, "props_diffusion: n = %lld too large", (long long)a.n);
    const int64_t blocks = (a.n + kDiffBlock - 1) / kDiffBlock;
    hipLaunchKernelGGL((diffusion_kernel<NS, PREC>), dim3((unsigned)blocks), dim3(kDiffBlock), 0, s, tt, tdd, tdf, a);
    PROPS_HIP_TRY(hipGetLastError());
    return PROPS_OK;
}

template <int NS>
int launch_prec(const props_mech_s *m, int prec, const DiffArgs &a, hipStream_t s)
{
    return (prec == PROPS_FP64) ? launch_ns<NS, PROPS_FP64>(m, a, s) : launch_ns<NS, PROPS_MIXED>(m, a, s);
}

}  // namespace

int launch_diffusion(const props_mech_s *m, int prec, const double *P, const double *T,
                     const double *Y, double *D, int64_t n, uint8_t *status, hipStream_t stream)
{
    DiffArgs a{P, T, Y, D, status, n, m->ns};
    switch (m->nsp) {
        case 1: return launch_prec<1>(m, prec, a, stream);
        case 2: return launch_prec<2>(m, prec, a, stream);
        case 4: return launch_prec<4>(m, prec, a, stream);
        default: return launch_prec<8>(m, prec, a, stream);
    }
}

}  // namespace props
