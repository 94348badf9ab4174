// mu-derivatives of the HISQ Dslash at mu = 0: the operators d^n M / d mu^n of
// Sec. 1 eq. (2) for n >= 1.  With the chemical potential on the time links, an
// h-step temporal hop carries exp(h mu); its n-th derivative at mu = 0 weights
// the hop by h^n and every spatial hop drops out.  So d^n D / d mu^n is the
// Dslash restricted to the four temporal slots (+1, -1, +3, -3), weighted by
// 1, (-1)^n, 3^n, (-3)^n.  FP64 links, site-major fields [Vh][3][n]; one thread
// per output site and rhs, so the n threads of a site are adjacent lanes that
// read n consecutive complex numbers per colour (one contiguous stretch) and
// the same link (one request).  Off the CG's hot path: the estimator spends
// its time in the solves.
#include "stencil.h"

namespace hisq {

template <int NRHS>
__global__ __launch_bounds__(256) void k_dslash_dmu(Lat lat, int parity, const d2* __restrict__ lk,
                                                    const d2* __restrict__ in, d2* __restrict__ out,
                                                    double wp1, double wm1, double wp3, double wm3)
{
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / NRHS), k = (int)(t - (long)i * NRHS);
    if (i >= lat.Vh) return;
    const SiteCoord sc = site_coord(lat, parity, i);
    d2 acc[3] = {d2{0.0, 0.0}, d2{0.0, 0.0}, d2{0.0, 0.0}};
    auto slot = [&](auto S, double w) {
        constexpr int s = decltype(S)::value;
        d2 m[9];
        load_link<double, HISQ_NAIK_FULL, s>(lk, lat.Vh, i, m);
        const int nb = neighbour<s>(lat, sc);
        d2 v[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) v[b] = in[((size_t)nb * 3 + b) * NRHS + k];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const d2 wv = d2{w * v[b].x, w * v[b].y};
#pragma unroll
            for (int a = 0; a < 3; ++a) cfma(acc[a], m[3 * a + b], wv);
        }
    };
    // slot s = 4 * hop + mu; the packed backward slots already carry the minus
    // sign of eq. (3)
    slot(std::integral_constant<int, 3>{}, wp1);
    slot(std::integral_constant<int, 7>{}, wm1);
    slot(std::integral_constant<int, 11>{}, wp3);
    slot(std::integral_constant<int, 15>{}, wm3);
#pragma unroll
    for (int a = 0; a < 3; ++a) out[((size_t)i * 3 + a) * NRHS + k] = acc[a];
}

hipError_t launch_dslash_dmu(const Lat& lat, int parity, int nrhs, int nder, const d2* lk,
                             const d2* in, d2* out, hipStream_t s)
{
    auto pw = [](double h, int n) {
        double w = 1.0;
        for (int j = 0; j < n; ++j) w *= h;
        return w;
    };
    const double wp1 = pw(1, nder), wm1 = pw(-1, nder), wp3 = pw(3, nder), wm3 = pw(-3, nder);
    const long threads = (long)lat.Vh * nrhs;
    const dim3 grid((unsigned)((threads + 255) / 256)), block(256);
    switch (nrhs) {
#define HISQ_DMU_CASE(N)                                                                          \
    case N:                                                                                       \
        hipLaunchKernelGGL(k_dslash_dmu<N>, grid, block, 0, s, lat, parity, lk, in, out, wp1, wm1, \
                           wp3, wm3);                                                            \
        break;
        HISQ_DMU_CASE(1)
        HISQ_DMU_CASE(2)
        HISQ_DMU_CASE(3)
        HISQ_DMU_CASE(4)
        HISQ_DMU_CASE(5)
        HISQ_DMU_CASE(6)
        HISQ_DMU_CASE(7)
        HISQ_DMU_CASE(8)
#undef HISQ_DMU_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hisq
