// Link force of the backward solve: gradient of L = sum_k Re(phi_k^dag x_k),
// A x_k = eta_k, with respect to the links of Sec. 1 eq. (3).
//
// With y = A^{-1} phi (even), t = D_oe x and s = D_oe y (odd), varying
// A = 4m^2 - D_eo D_oe gives dL = sum_k [Re y^dag dD_eo t - Re s^dag dD_oe x]
// (plus the mass term, reduced separately).  Collecting the terms of eq. (3)
// that hold link (a, mu), with b = a + mu for U and b = a + 3 mu for N:
//   a even:  G[mu][a] =  sum_k ( y_a t_b^dag + x_a s_b^dag )
//   a odd :  G[mu][a] = -sum_k ( t_a y_b^dag + s_a x_b^dag )
// in the convention G = dL/dRe + i dL/dIm.  One thread per link; every link
// has one writer, so no atomics are needed.
#include "hisq_device.h"

namespace hisq {

__device__ __forceinline__ d2 cmul_conj(d2 a, d2 b)  // a * conj(b)
{
    return d2{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

__global__ void k_force(Lat lat, int nrhs, const d2* __restrict__ x, const d2* __restrict__ y,
                        const d2* __restrict__ tx, const d2* __restrict__ sy, d2* __restrict__ GU,
                        d2* __restrict__ GN)
{
    const int V = 2 * lat.Vh;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 4 * V) return;
    const int mu = idx / V;
    const int a = idx - mu * V;
    int c[4];
    int r = a;
    for (int nu = 0; nu < 4; ++nu) {
        c[nu] = r % lat.L[nu];
        r /= lat.L[nu];
    }
    const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
    const size_t ia = (size_t)(a >> 1) * 3 * nrhs;
    for (int pass = 0; pass < 2; ++pass) {
        const int h = pass == 0 ? 1 : 3;
        int d[4] = {c[0], c[1], c[2], c[3]};
        d[mu] = (d[mu] + h) % lat.L[mu];
        const int b = d[0] + lat.L[0] * (d[1] + lat.L[1] * (d[2] + lat.L[2] * d[3]));
        const size_t ib = (size_t)(b >> 1) * 3 * nrhs;
        // even root: (u1, v1, u2, v2) = (y_a, t_b, x_a, s_b); odd: (t_a, y_b, s_a, x_b)
        const d2* u1 = par == 0 ? y : tx;
        const d2* v1 = par == 0 ? tx : y;
        const d2* u2 = par == 0 ? x : sy;
        const d2* v2 = par == 0 ? sy : x;
        const double sign = par == 0 ? 1.0 : -1.0;
        d2 G[9];
        for (int e = 0; e < 9; ++e) G[e] = d2{0, 0};
        for (int k = 0; k < nrhs; ++k) {
            d2 a1[3], b1[3], a2[3], b2[3];
            for (int cc = 0; cc < 3; ++cc) {
                a1[cc] = u1[ia + cc * nrhs + k];
                b1[cc] = v1[ib + cc * nrhs + k];
                a2[cc] = u2[ia + cc * nrhs + k];
                b2[cc] = v2[ib + cc * nrhs + k];
            }
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) G[3 * i + j] += cmul_conj(a1[i], b1[j]) + cmul_conj(a2[i], b2[j]);
        }
        d2* out = (pass == 0 ? GU : GN) + ((size_t)mu * V + a) * 9;
        for (int e = 0; e < 9; ++e) out[e] = d2{sign * G[e].x, sign * G[e].y};
    }
}

hipError_t launch_force(const Lat& lat, int nrhs, const d2* x, const d2* y, const d2* tx,
                        const d2* sy, d2* GU, d2* GN, hipStream_t s)
{
    const long n = 4L * 2 * lat.Vh;
    const int bs = 128;
    const int grid = (int)((n + bs - 1) / bs);
    hipLaunchKernelGGL(k_force, dim3(grid), dim3(bs), 0, s, lat, nrhs, x, y, tx, sy, GU, GN);
    return hipGetLastError();
}

}  // namespace hisq
