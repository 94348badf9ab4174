// Link packing: canonical [4][V][3][3] complex128 U, N -> the per-parity slot
// blocks the Dslash kernels stream (layout described in hisq_internal.h).
//
// For output site z the 16 slots are U_{z,mu}, -U^dag_{z-mu,mu}, N_{z,mu} and
// -N^dag_{z-3mu,mu} (the four terms of Sec. 1 eq. (3), sign folded in).  In r14
// storage a Naik slot keeps rows 0 and 1 and c = <w, row2> / |w|^2 with
// w = conj(row0 x row1), so that row2 = c w exactly when the matrix is a
// positive multiple of a U(3) matrix; the worst relative round-trip error is
// kept in the buffer header (atomicMax on the float's bits, valid for
// non-negative floats).  In r9 storage a Naik slot keeps H = -i log(M / s),
// s = |det M|^(1/3); the header tracks the smallest and largest s, and the
// round trip is checked through the FP32 decoder on the FP32-rounded H.
#include "hisq_device.h"
#include "naik.h"

namespace hisq {

__device__ __forceinline__ d2 cmul_d(d2 a, d2 b)
{
    return d2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ int site_of(const Lat& lat, const int x[4])
{
    return x[0] + lat.L[0] * (x[1] + lat.L[1] * (x[2] + lat.L[2] * x[3]));
}

template <typename T, int NK>
__global__ void k_pack(Lat lat, const d2* __restrict__ U, const d2* __restrict__ N,
                       T* __restrict__ out, LinkHeader* hdr)
{
    using C = cplx<T>;
    const int Vh = lat.Vh;
    const int V = 2 * Vh;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= V) return;
    const int P = idx / Vh;
    const int i = idx - P * Vh;
    int r = i / lat.Lh0;
    const int xh = i - r * lat.Lh0;
    int c[4];
    c[1] = r % lat.L[1];
    r /= lat.L[1];
    c[2] = r % lat.L[2];
    c[3] = r / lat.L[2];
    c[0] = 2 * xh + ((P + c[1] + c[2] + c[3]) & 1);
    const int s = site_of(lat, c);
    T* blk = out + (size_t)P * link_block_reals(Vh, NK);
    // real r of site i's matrix in a slot of nr reals
    auto put = [&](T* slot, int nr, int r, T v) {
        if constexpr (sizeof(T) == 4)
            slot[slot_real_offset32(r, nr, Vh, i)] = v;
        else
            slot[((size_t)(r >> 1) * Vh + i) * 2 + (r & 1)] = v;
    };
    float worst = 0.0f;
    for (int slot = 0; slot < 16; ++slot) {
        const int mu = slot & 3, kind = slot >> 2;  // 0: U fwd, 1: U bwd, 2: N fwd, 3: N bwd
        const d2* W = (kind < 2) ? U : N;
        int root = s;
        if (kind == 1 || kind == 3) {
            int y[4] = {c[0], c[1], c[2], c[3]};
            const int h = kind == 1 ? 1 : 3;
            y[mu] = (y[mu] - h + lat.L[mu]) % lat.L[mu];
            root = site_of(lat, y);
        }
        const d2* src = W + ((size_t)mu * V + root) * 9;
        d2 m[9];
        for (int e = 0; e < 9; ++e) m[e] = src[e];
        if (kind == 1 || kind == 3) {  // -W^dag
            d2 t[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) t[3 * a + b] = d2{-m[3 * b + a].x, m[3 * b + a].y};
            for (int e = 0; e < 9; ++e) m[e] = t[e];
        }
        T* dst = blk + (size_t)slot_real_start(slot, NK) * Vh;
        const int nr = slot_reals(slot, NK);
        if (NK == HISQ_NAIK_R9 && slot >= 8) {
            // s = |det M|^(1/3), W = M / s, H = -i log W
            Cx<double> Wm[9];
            for (int e = 0; e < 9; ++e) Wm[e] = Cx<double>{m[e].x, m[e].y};
            const Cx<double> a1 = cx_mul(Wm[4], Wm[8]), a2 = cx_mul(Wm[5], Wm[7]);
            const Cx<double> b1 = cx_mul(Wm[3], Wm[8]), b2 = cx_mul(Wm[5], Wm[6]);
            const Cx<double> g1 = cx_mul(Wm[3], Wm[7]), g2 = cx_mul(Wm[4], Wm[6]);
            const Cx<double> t0 = cx_mul(Wm[0], Cx<double>{a1.re - a2.re, a1.im - a2.im});
            const Cx<double> t1 = cx_mul(Wm[1], Cx<double>{b1.re - b2.re, b1.im - b2.im});
            const Cx<double> t2 = cx_mul(Wm[2], Cx<double>{g1.re - g2.re, g1.im - g2.im});
            const double dre = t0.re - t1.re + t2.re, dim = t0.im - t1.im + t2.im;
            const double sc = cbrt(sqrt(dre * dre + dim * dim));
            double hreal[9];
            double fro = 0, err = 0;
            for (int e = 0; e < 9; ++e) fro += m[e].x * m[e].x + m[e].y * m[e].y;
            if (sc > 0) {
                for (int e = 0; e < 9; ++e) Wm[e] = Cx<double>{m[e].x / sc, m[e].y / sc};
                log_unitary(Wm, hreal);
                float hf[9], ore[9], oim[9];
                for (int e = 0; e < 9; ++e) hf[e] = (float)hreal[e];
                expi_hermitian<float>(hf, (float)sc, ore, oim);
                for (int e = 0; e < 9; ++e) {
                    const double dx = ore[e] - m[e].x, dy = oim[e] - m[e].y;
                    err += dx * dx + dy * dy;
                }
            } else {
                for (int e = 0; e < 9; ++e) hreal[e] = 0;
                err = fro;
            }
            const double rel = fro > 0 ? sqrt(err / fro) : 0.0;
            worst = fmaxf(worst, (rel == rel) ? (float)rel : 3.0e38f);
            const float scf = (float)sc;
            atomicMin(&hdr->scale_min_bits, __float_as_uint(scf));
            atomicMax(&hdr->scale_max_bits, __float_as_uint(scf));
            for (int e = 0; e < 9; ++e) put(dst, nr, e, (T)hreal[e]);
        } else if (NK != HISQ_NAIK_FULL && slot >= 8) {
            // w = conj(row0 x row1); c = <w, row2> / |w|^2
            d2 w[3];
            w[0] = cmul_d(m[1], m[5]) - cmul_d(m[2], m[4]);
            w[1] = cmul_d(m[2], m[3]) - cmul_d(m[0], m[5]);
            w[2] = cmul_d(m[0], m[4]) - cmul_d(m[1], m[3]);
            for (int j = 0; j < 3; ++j) w[j].y = -w[j].y;
            d2 num = d2{0, 0};
            double den = 0, fro = 0, err = 0;
            for (int j = 0; j < 3; ++j) {
                num += cmul_d(d2{w[j].x, -w[j].y}, m[6 + j]);
                den += w[j].x * w[j].x + w[j].y * w[j].y;
            }
            d2 cc = den > 0 ? d2{num.x / den, num.y / den} : d2{0, 0};
            const double phi = atan2(cc.y, cc.x);
            if (NK == HISQ_NAIK_R13) {
                // r13 keeps only the phase; the modulus is 1 / |row0|
                const double r0 = sqrt(m[0].x * m[0].x + m[0].y * m[0].y + m[1].x * m[1].x +
                                       m[1].y * m[1].y + m[2].x * m[2].x + m[2].y * m[2].y);
                cc = r0 > 0 ? d2{cos(phi) / r0, sin(phi) / r0} : d2{0, 0};
            }
            for (int e = 0; e < 9; ++e) fro += m[e].x * m[e].x + m[e].y * m[e].y;
            for (int j = 0; j < 3; ++j) {
                const d2 d = m[6 + j] - cmul_d(cc, w[j]);
                err += d.x * d.x + d.y * d.y;
            }
            const double rel = fro > 0 ? sqrt(err / fro) : 0.0;
            const float relf = (rel == rel) ? (float)rel : 3.0e38f;
            worst = fmaxf(worst, relf);
            for (int e = 0; e < 6; ++e) {
                put(dst, nr, 2 * e, (T)m[e].x);
                put(dst, nr, 2 * e + 1, (T)m[e].y);
            }
            if (NK == HISQ_NAIK_R14) {
                put(dst, nr, 12, (T)cc.x);
                put(dst, nr, 13, (T)cc.y);
            } else {
                put(dst, nr, 12, (T)phi);
            }
        } else {
            for (int e = 0; e < 9; ++e) {
                put(dst, nr, 2 * e, (T)m[e].x);
                put(dst, nr, 2 * e + 1, (T)m[e].y);
            }
        }
    }
    if (NK != HISQ_NAIK_FULL && worst > 0.0f) atomicMax(&hdr->naik_err_bits, __float_as_uint(worst));
}

__global__ void k_pack_header(LinkHeader h, LinkHeader* dst) { *dst = h; }

hipError_t launch_pack(const Lat& lat, const d2* U, const d2* N, int prec, int naik, void* packed,
                       hipStream_t s)
{
    LinkHeader h{};
    h.magic = kLinkMagic;
    for (int mu = 0; mu < 4; ++mu) h.L[mu] = lat.L[mu];
    h.prec = prec;
    h.naik = naik;
    h.naik_err_bits = 0u;
    h.scale_min_bits = 0x7f800000u;  // +inf
    h.scale_max_bits = 0u;
    h.naik_scale = 1.0f;
    LinkHeader* hdr = reinterpret_cast<LinkHeader*>(packed);
    hipLaunchKernelGGL(k_pack_header, dim3(1), dim3(1), 0, s, h, hdr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    char* body = reinterpret_cast<char*>(packed) + kLinkHeaderBytes;
    const int V = 2 * lat.Vh, bs = 128, grid = (V + bs - 1) / bs;
    if (prec == HISQ_PREC_F64)
        hipLaunchKernelGGL((k_pack<double, HISQ_NAIK_FULL>), dim3(grid), dim3(bs), 0, s, lat, U, N,
                           reinterpret_cast<double*>(body), hdr);
    else if (naik == HISQ_NAIK_R14)
        hipLaunchKernelGGL((k_pack<float, HISQ_NAIK_R14>), dim3(grid), dim3(bs), 0, s, lat, U, N,
                           reinterpret_cast<float*>(body), hdr);
    else if (naik == HISQ_NAIK_R13)
        hipLaunchKernelGGL((k_pack<float, HISQ_NAIK_R13>), dim3(grid), dim3(bs), 0, s, lat, U, N,
                           reinterpret_cast<float*>(body), hdr);
    else if (naik == HISQ_NAIK_R9)
        hipLaunchKernelGGL((k_pack<float, HISQ_NAIK_R9>), dim3(grid), dim3(bs), 0, s, lat, U, N,
                           reinterpret_cast<float*>(body), hdr);
    else
        hipLaunchKernelGGL((k_pack<float, HISQ_NAIK_FULL>), dim3(grid), dim3(bs), 0, s, lat, U, N,
                           reinterpret_cast<float*>(body), hdr);
    return hipGetLastError();
}

}  // namespace hisq
