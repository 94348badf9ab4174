// Link force of the backward solve: gradient of L = sum_k Re(phi_k^dag x_k),
// A x_k = eta_k, with respect to the links of Sec. 1 eq. (3).
//
// With y = A^{-1} phi (even), t = D_oe x and s = D_oe y (odd), varying
// A = 4m^2 - D_eo D_oe gives dL = sum_k [Re y^dag dD_eo t - Re s^dag dD_oe x]
// (plus the mass term, reduced separately).  Collecting the terms of eq. (3)
// that hold link (a, mu), with b = a + mu for U and b = a + 3 mu for N:
//   a even:  G[mu][a] =  sum_k ( y_a t_b^dag + x_a s_b^dag )
//   a odd :  G[mu][a] = -sum_k ( t_a y_b^dag + s_a x_b^dag )
// in the convention G = dL/dRe + i dL/dIm.  Every link has one writer, so no
// atomics are needed.
#include "hisq_device.h"

namespace hisq {

__device__ __forceinline__ d2 cmul_conj(d2 a, d2 b)  // a * conj(b)
{
    return d2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

constexpr int kForceSites = 32;                   // sites per work-group
constexpr int kForceLinks = 4 * kForceSites;      // links (direction, site) per work-group
constexpr int kForceBlock = 2 * kForceLinks;      // two threads per link, one per term

// Work-group -> block of kForceSites canonical sites.  Where the lattice allows
// (L[2] a multiple of the 8 XCDs, whole blocks per (x, y) plane), XCD j (the
// work-groups b with b mod 8 = j) owns z-planes [j zc, (j+1) zc) of every time
// slice and walks them with the plane block outermost, then t, then z: the
// neighbours of a link in x, y and t, and most in z, are fetched by the same
// XCD shortly before or after, so they come from its L2.  Otherwise b itself.
__device__ inline int force_block(int b, int nb, const Lat& lat)
{
    const int plane = lat.L[0] * lat.L[1];
    if ((lat.L[2] & 7) || plane % kForceSites || nb != plane / kForceSites * lat.L[2] * lat.L[3])
        return b;
    const int zc = lat.L[2] >> 3, C = plane / kForceSites;
    const int j = b & 7, m = b >> 3;
    const int zl = m % zc, t = (m / zc) % lat.L[3], c = m / (zc * lat.L[3]);
    return (t * lat.L[2] + j * zc + zl) * C + c;
}

// Two threads per link (mu, a), one per term of the sum over the bundle
// (thread = term * 128 + mu * 32 + site): term 0 accumulates u1 v1^dag, term 1
// u2 v2^dag, so each thread holds half the loads of a link, which keeps the
// register count (and so the waves resident per SIMD) at about half of what
// one thread per link needs.  A work-group covers the links of all four
// directions of kForceSites consecutive canonical sites, so a site's own
// fields, read by its four links, come from the cache after the first.
// Fields are colour-major, [3][Vh][n]: the rhs of one colour of a site are n
// consecutive complex numbers; the bundle size is a template parameter, so
// the loop over rhs unrolls and all of a term's loads are in flight together.
// The two terms meet in LDS and the sums are written as four contiguous
// stretches of the output ([4][V][3][3], one per direction), 16 bytes per
// lane per store.
template <int NRHS>
__global__ __launch_bounds__(kForceBlock) void k_force(Lat lat, const d2* __restrict__ xc,
                                                       const d2* __restrict__ yc,
                                                       const d2* __restrict__ txc,
                                                       const d2* __restrict__ syc,
                                                       d2* __restrict__ GU, d2* __restrict__ GN)
{
    __shared__ d2 sg[2][kForceLinks * 9];
    const int V = 2 * lat.Vh;
    const int a0 = force_block(blockIdx.x, gridDim.x, lat) * kForceSites;
    const int nsites = min(kForceSites, V - a0);
    const int term = threadIdx.x / kForceLinks;
    const int link = threadIdx.x - term * kForceLinks;
    const int mu = link / kForceSites;
    const int al = link - mu * kForceSites;
    const bool live = al < nsites;
    const int a = live ? a0 + al : a0;
    int c[4];
    int r = a;
    for (int nu = 0; nu < 4; ++nu) {
        c[nu] = r % lat.L[nu];
        r /= lat.L[nu];
    }
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    const size_t cs = (size_t)lat.Vh * NRHS;  // colour stride
    const size_t ia = (size_t)(a >> 1) * NRHS;
    // even root: term 0 (u, v) = (y_a, t_b), term 1 (x_a, s_b);
    // odd root:  term 0 (t_a, y_b), term 1 (s_a, x_b)
    const d2* u = par == 0 ? (term == 0 ? yc : xc) : (term == 0 ? txc : syc);
    const d2* v = par == 0 ? (term == 0 ? txc : syc) : (term == 0 ? yc : xc);
    const double sign = par == 0 ? 1.0 : -1.0;
    for (int pass = 0; pass < 2; ++pass) {
        const int h = pass == 0 ? 1 : 3;
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] = (d[mu] + h) % lat.L[mu];
        const int b = d[0] + lat.L[0] * (d[1] + lat.L[1] * (d[2] + lat.L[2] * d[3]));
        const size_t ib = (size_t)(b >> 1) * NRHS;
        d2 G[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) G[e] = d2{0, 0};
        if (live) {
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                d2 ua[3], vb[3];
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    ua[cc] = u[cc * cs + ia + k];
                    vb[cc] = v[cc * cs + ib + k];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) G[3 * i + j] += cmul_conj(ua[i], vb[j]);
            }
        }
        __syncthreads();  // the previous pass's stores have read sg
#pragma unroll
        for (int e = 0; e < 9; ++e) sg[term][link * 9 + e] = d2{sign * G[e].x, sign * G[e].y};
        __syncthreads();
        d2* out = pass == 0 ? GU : GN;
        // sg[.] holds [mu][site][9]; direction m's links are out[(m V + a0) * 9 ...]
        for (int q = threadIdx.x; q < kForceLinks * 9; q += kForceBlock) {
            const int m = q / (kForceSites * 9), w = q - m * (kForceSites * 9);
            if (w < nsites * 9) {
                const d2 g0 = sg[0][q], g1 = sg[1][q];
                out[((size_t)m * V + a0) * 9 + w] = d2{g0.x + g1.x, g0.y + g1.y};
            }
        }
    }
}

hipError_t launch_force(const Lat& lat, int nrhs, const d2* xc, const d2* yc, const d2* txc,
                        const d2* syc, d2* GU, d2* GN, hipStream_t s)
{
    const int V = 2 * lat.Vh;
    const int grid = (V + kForceSites - 1) / kForceSites;
    switch (nrhs) {
#define HISQ_FORCE_CASE(N)                                                                         \
    case N:                                                                                        \
        hipLaunchKernelGGL(k_force<N>, dim3(grid), dim3(kForceBlock), 0, s, lat, xc, yc, txc, syc, GU, \
                           GN);                                                                    \
        break;
        HISQ_FORCE_CASE(1)
        HISQ_FORCE_CASE(2)
        HISQ_FORCE_CASE(3)
        HISQ_FORCE_CASE(4)
        HISQ_FORCE_CASE(5)
        HISQ_FORCE_CASE(6)
        HISQ_FORCE_CASE(7)
        HISQ_FORCE_CASE(8)
#undef HISQ_FORCE_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hisq
