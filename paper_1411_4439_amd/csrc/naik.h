// Compressed Naik-link encodings (Sec. 1: the Naik links are reconstructed from
// fewer than 18 floats).  For N = s W with W in U(3), s > 0:
//   r13: rows 0 and 1 and the phase of c, row2 = c conj(row0 x row1), |c| = 1/s;
//   r9:  one Hermitian H with W = exp(iH) (9 reals), s shared by every Naik link
//        of the field.
// exp(iH) is evaluated in the Cayley-Hamilton form exp(iQ) = f0 + f1 Q + f2 Q^2
// for the traceless part Q of H (the form used by Morningstar and Peardon,
// Phys. Rev. D 69 (2004) 054501), with f0..f2 by scaling and squaring of the
// power series instead of their closed form, and without library
// transcendentals, so that the Dslash keeps its registers.
#pragma once

#include "hisq_internal.h"

namespace hisq {

// exp(i phi) for phi in [-pi, pi]: Taylor series of sin and cos at phi/2 in
// [-pi/2, pi/2] (truncation below 6e-8), then the double-angle formulas;
// within 4e-7 of the exact value in FP32.
__host__ __device__ inline void unit_phase(float phi, float* cs, float* sn)
{
    const float t = 0.5f * phi, t2 = t * t;
    float s = 1.0f - t2 * (1.0f / (12 * 13));
    s = 1.0f - t2 * (1.0f / (10 * 11)) * s;
    s = 1.0f - t2 * (1.0f / (8 * 9)) * s;
    s = 1.0f - t2 * (1.0f / (6 * 7)) * s;
    s = 1.0f - t2 * (1.0f / (4 * 5)) * s;
    s = t * (1.0f - t2 * (1.0f / (2 * 3)) * s);
    float c = 1.0f - t2 * (1.0f / (13 * 14));
    c = 1.0f - t2 * (1.0f / (11 * 12)) * c;
    c = 1.0f - t2 * (1.0f / (9 * 10)) * c;
    c = 1.0f - t2 * (1.0f / (7 * 8)) * c;
    c = 1.0f - t2 * (1.0f / (5 * 6)) * c;
    c = 1.0f - t2 * (1.0f / (3 * 4)) * c;
    c = 1.0f - t2 * (1.0f / (1 * 2)) * c;
    *cs = c * c - s * s;
    *sn = 2.0f * s * c;
}

// FP64 (packing only): the library functions
__host__ __device__ inline void unit_phase(double phi, double* cs, double* sn)
{
    *cs = cos(phi);
    *sn = sin(phi);
}

// x reduced to [-pi, pi] (a whole number of turns removed; the turn count is
// taken from x / 2pi rounded, so the product with the rounded reciprocal is
// exact enough)
template <typename T>
__host__ __device__ inline T wrap_pi(T x)
{
    const T twopi = T(6.283185307179586), inv_twopi = T(0.15915494309189535);
    return x - twopi * rint(x * inv_twopi);
}

template <typename T>
struct Cx {
    T re, im;
};

template <typename T>
__host__ __device__ inline Cx<T> cx_mul(Cx<T> a, Cx<T> b)
{
    return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename T>
__host__ __device__ inline Cx<T> cx_sq(Cx<T> a)
{
    return Cx<T>{a.re * a.re - a.im * a.im, T(2) * a.re * a.im};
}

// out = scale * exp(iH), H Hermitian given by its 9 reals
// (H00, H11, H22, Re H01, Im H01, Re H02, Im H02, Re H12, Im H12); out is
// row-major, element e as (re, im) in out_re[e], out_im[e].
//
// With t = tr(H)/3 and the traceless Q = H - t, exp(iH) = e^{it} exp(iQ), and
// every power of Q is a + b Q + d Q^2 with real a, b, d, because
// Q^3 = c1 Q + c0 (Cayley-Hamilton; c1 = tr(Q^2)/2, c0 = det Q).  exp(iQ) is
// computed in that basis by scaling and squaring: Q' = Q / 4, the power series
// of exp(iQ') to order 12, then two squarings, each reduced with
// Q'^3 = c1' Q' + c0'.  H from the packer has its eigenvalues in a window of
// width 2pi, so c1 <= 4pi^2/3, c1' <= 0.83, every eigenvalue of Q' is within
// 1.05 in magnitude and the series is truncated below 3e-10.  Straight-line
// code without loops or branches: inlined into the Dslash, it keeps the
// kernel's registers (a data-dependent number of squarings did not).
template <typename T>
__host__ __device__ inline void expi_hermitian(const T (&h)[9], T scale, T (&out_re)[9], T (&out_im)[9])
{
    // Q: diagonal d0..d2, upper triangle qa = Q01, qb = Q02, qc = Q12
    const T t = (h[0] + h[1] + h[2]) * T(1.0 / 3.0);
    const T d0 = h[0] - t, d1 = h[1] - t, d2 = h[2] - t;
    const Cx<T> qa{h[3], h[4]}, qb{h[5], h[6]}, qc{h[7], h[8]};
    const T na = qa.re * qa.re + qa.im * qa.im, nb = qb.re * qb.re + qb.im * qb.im,
            nc = qc.re * qc.re + qc.im * qc.im;
    // c1 = tr(Q^2) / 2 >= 0; c0 = det Q = d0 d1 d2 + 2 Re(a c conj b) - d0|c|^2 - d1|b|^2 - d2|a|^2
    const T c1 = T(0.5) * (d0 * d0 + d1 * d1 + d2 * d2) + na + nb + nc;
    const Cx<T> ac = cx_mul(qa, qc);
    const T c0 = d0 * d1 * d2 + T(2) * (ac.re * qb.re + ac.im * qb.im) - d0 * nc - d1 * nb - d2 * na;
    constexpr int k = 2;
    const T c1s = c1 * T(0.0625), c0s = c0 * T(0.015625);
    // series: sum_j (i^j / j!) Q'^j with Q'^j = a + b Q' + d Q'^2 (real a, b, d)
    Cx<T> f0{1, 0}, f1{0, 0}, f2{0, 0};
    {
        T a = 1, b = 0, d = 0;
        T fact = 1;
#pragma unroll
        for (int j = 1; j <= 12; ++j) {
            const T na2 = d * c0s, nb2 = a + d * c1s;
            d = b;
            a = na2;
            b = nb2;
            fact *= T(1) / T(j);  // folded by the compiler: every j is a constant
            // i^j: 1, i, -1, -i
            const T w = (j % 4 == 0 || j % 4 == 1) ? fact : -fact;
            if (j % 2 == 0) {
                f0.re += w * a;
                f1.re += w * b;
                f2.re += w * d;
            } else {
                f0.im += w * a;
                f1.im += w * b;
                f2.im += w * d;
            }
        }
    }
    // k squarings: (f0 + f1 Q' + f2 Q'^2)^2 with Q'^3 = c1' Q' + c0' and
    // Q'^4 = c1' Q'^2 + c0' Q'
#pragma unroll
    for (int r = 0; r < k; ++r) {
        const Cx<T> p00 = cx_sq(f0), p11 = cx_sq(f1), p22 = cx_sq(f2);
        const Cx<T> p01 = cx_mul(f0, f1), p02 = cx_mul(f0, f2), p12 = cx_mul(f1, f2);
        const T c0t = T(2) * c0s, c1t = T(2) * c1s;
        f0 = Cx<T>{p00.re + c0t * p12.re, p00.im + c0t * p12.im};
        f1 = Cx<T>{T(2) * p01.re + c1t * p12.re + c0s * p22.re, T(2) * p01.im + c1t * p12.im + c0s * p22.im};
        f2 = Cx<T>{T(2) * p02.re + p11.re + c1s * p22.re, T(2) * p02.im + p11.im + c1s * p22.im};
    }
    // back to the basis of Q (Q' = Q / 2^k), with scale * e^{it} folded in
    Cx<T> ph;
    unit_phase(wrap_pi(t), &ph.re, &ph.im);
    const T s1 = ldexp(scale, -k), s2 = ldexp(scale, -2 * k);
    f0 = cx_mul(Cx<T>{ph.re * scale, ph.im * scale}, f0);
    f1 = cx_mul(Cx<T>{ph.re * s1, ph.im * s1}, f1);
    f2 = cx_mul(Cx<T>{ph.re * s2, ph.im * s2}, f2);
    // Q^2 (Hermitian): diagonal and upper triangle
    const T e0 = d0 * d0 + na + nb, e1 = na + d1 * d1 + nc, e2 = nb + nc + d2 * d2;
    const Cx<T> bc = cx_mul(qb, Cx<T>{qc.re, -qc.im}), ab = cx_mul(Cx<T>{qa.re, -qa.im}, qb);
    const Cx<T> g01{qa.re * (d0 + d1) + bc.re, qa.im * (d0 + d1) + bc.im};
    const Cx<T> g02{qb.re * (d0 + d2) + ac.re, qb.im * (d0 + d2) + ac.im};
    const Cx<T> g12{qc.re * (d1 + d2) + ab.re, qc.im * (d1 + d2) + ab.im};
    auto diag = [&](int e, T q, T q2) {
        out_re[e] = f0.re + f1.re * q + f2.re * q2;
        out_im[e] = f0.im + f1.im * q + f2.im * q2;
    };
    // upper element f1 q + f2 g, lower element f1 conj(q) + f2 conj(g)
    auto pair = [&](int up, int lo, Cx<T> q, Cx<T> g) {
        out_re[up] = f1.re * q.re - f1.im * q.im + f2.re * g.re - f2.im * g.im;
        out_im[up] = f1.re * q.im + f1.im * q.re + f2.re * g.im + f2.im * g.re;
        out_re[lo] = f1.re * q.re + f1.im * q.im + f2.re * g.re + f2.im * g.im;
        out_im[lo] = f1.im * q.re - f1.re * q.im + f2.im * g.re - f2.re * g.im;
    };
    diag(0, d0, e0);
    diag(4, d1, e1);
    diag(8, d2, e2);
    pair(1, 3, qa, g01);
    pair(2, 6, qb, g02);
    pair(5, 7, qc, g12);
}

}  // namespace hisq

namespace hisq {

// Hermitian H with exp(iH) = W for a unitary 3x3 W (FP64, packing only), as
// the 9 reals that expi_hermitian reads.  Shift first, V = exp(-i gamma) W with
// gamma among six candidates the one that keeps every eigenvalue of V furthest
// from -1 (largest |det(1 + V)|); then the Cayley map K = i (1 - V)(1 + V)^-1 is
// Hermitian with eigenvalues tan(phi/2) for the eigenphases phi of V.  Cyclic
// Jacobi rotations diagonalise K = Z diag(k) Z^dag, and
// H = gamma + Z diag(2 atan k) Z^dag.
__host__ __device__ inline void log_unitary(const Cx<double> (&W)[9], double (&h)[9])
{
    auto det3 = [](const Cx<double>* m) {
        auto sub = [&](int a, int b, int c, int d) {
            const Cx<double> x = cx_mul(m[a], m[b]), y = cx_mul(m[c], m[d]);
            return Cx<double>{x.re - y.re, x.im - y.im};
        };
        const Cx<double> t0 = cx_mul(m[0], sub(4, 8, 5, 7));
        const Cx<double> t1 = cx_mul(m[1], sub(3, 8, 5, 6));
        const Cx<double> t2 = cx_mul(m[2], sub(3, 7, 4, 6));
        return Cx<double>{t0.re - t1.re + t2.re, t0.im - t1.im + t2.im};
    };
    double gamma = 0, best = -1;
    for (int c = 0; c < 6; ++c) {
        const double g = c * (3.141592653589793 / 3.0);
        const Cx<double> e{cos(g), -sin(g)};
        Cx<double> P[9];
        for (int k = 0; k < 9; ++k) P[k] = cx_mul(e, W[k]);
        for (int k = 0; k < 9; k += 4) P[k].re += 1.0;
        const Cx<double> d = det3(P);
        const double mag = d.re * d.re + d.im * d.im;
        if (mag > best) {
            best = mag;
            gamma = g;
        }
    }
    const Cx<double> e{cos(gamma), -sin(gamma)};
    Cx<double> Vm[9], Pm[9], Mm[9];
    for (int k = 0; k < 9; ++k) Vm[k] = cx_mul(e, W[k]);
    for (int k = 0; k < 9; ++k) {
        Pm[k] = Vm[k];  // 1 + V
        Mm[k] = Cx<double>{-Vm[k].re, -Vm[k].im};  // 1 - V
    }
    for (int k = 0; k < 9; k += 4) {
        Pm[k].re += 1.0;
        Mm[k].re += 1.0;
    }
    // (1 + V)^-1 by the adjugate
    const Cx<double> dp = det3(Pm);
    const double dn = dp.re * dp.re + dp.im * dp.im;
    const Cx<double> dinv{dp.re / dn, -dp.im / dn};
    Cx<double> inv[9];
    const int r0[3] = {1, 0, 0}, r1[3] = {2, 2, 1};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            // cofactor C_ji / det -> inv_ij
            const int a = r0[j], b = r1[j], c = r0[i], d = r1[i];
            const Cx<double> x = cx_mul(Pm[3 * a + c], Pm[3 * b + d]);
            const Cx<double> y = cx_mul(Pm[3 * a + d], Pm[3 * b + c]);
            Cx<double> cof{x.re - y.re, x.im - y.im};
            if ((i + j) & 1) cof = Cx<double>{-cof.re, -cof.im};
            inv[3 * i + j] = cx_mul(cof, dinv);
        }
    // K = i (1 - V) inv, then its Hermitian part
    Cx<double> K[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Cx<double> acc{0, 0};
            for (int k = 0; k < 3; ++k) {
                const Cx<double> p = cx_mul(Mm[3 * i + k], inv[3 * k + j]);
                acc.re += p.re;
                acc.im += p.im;
            }
            K[3 * i + j] = Cx<double>{-acc.im, acc.re};
        }
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            const Cx<double> a = K[3 * i + j], b = K[3 * j + i];
            const Cx<double> s{0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
            K[3 * i + j] = s;
            K[3 * j + i] = Cx<double>{s.re, -s.im};
        }
    // cyclic Jacobi: A <- J^dag A J, Z <- Z J, J = P R on the (p, q) plane,
    // P = diag(1, conj(phase of A_pq)), R the real rotation zeroing it
    Cx<double> Z[9] = {{1, 0}, {0, 0}, {0, 0}, {0, 0}, {1, 0}, {0, 0}, {0, 0}, {0, 0}, {1, 0}};
    const int pp[3] = {0, 0, 1}, qq[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 12; ++sweep) {
        double off = 0, diag = 0;
        for (int k = 0; k < 3; ++k) {
            const Cx<double> a = K[3 * pp[k] + qq[k]];
            off += a.re * a.re + a.im * a.im;
            diag += K[4 * k].re * K[4 * k].re;
        }
        if (off <= 1e-32 * (1.0 + diag)) break;
        for (int k = 0; k < 3; ++k) {
            const int p = pp[k], q = qq[k];
            const Cx<double> apq = K[3 * p + q];
            const double r = sqrt(apq.re * apq.re + apq.im * apq.im);
            if (r == 0.0) continue;
            const Cx<double> phc{apq.re / r, -apq.im / r};  // conj(phase)
            const double tau = (K[4 * q].re - K[4 * p].re) / (2.0 * r);
            const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            const double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
            // J columns p, q: J_pp = c, J_pq = s, J_qp = -s phc, J_qq = c phc
            const Cx<double> Jpp{c, 0}, Jpq{s, 0};
            const Cx<double> Jqp{-s * phc.re, -s * phc.im}, Jqq{c * phc.re, c * phc.im};
            // A <- A J (columns p, q), Z <- Z J
            for (int i = 0; i < 3; ++i) {
                const Cx<double> ap = K[3 * i + p], aq = K[3 * i + q];
                const Cx<double> x0 = cx_mul(ap, Jpp), x1 = cx_mul(aq, Jqp);
                const Cx<double> y0 = cx_mul(ap, Jpq), y1 = cx_mul(aq, Jqq);
                K[3 * i + p] = Cx<double>{x0.re + x1.re, x0.im + x1.im};
                K[3 * i + q] = Cx<double>{y0.re + y1.re, y0.im + y1.im};
                const Cx<double> zp = Z[3 * i + p], zq = Z[3 * i + q];
                const Cx<double> u0 = cx_mul(zp, Jpp), u1 = cx_mul(zq, Jqp);
                const Cx<double> v0 = cx_mul(zp, Jpq), v1 = cx_mul(zq, Jqq);
                Z[3 * i + p] = Cx<double>{u0.re + u1.re, u0.im + u1.im};
                Z[3 * i + q] = Cx<double>{v0.re + v1.re, v0.im + v1.im};
            }
            // A <- J^dag A (rows p, q)
            for (int j = 0; j < 3; ++j) {
                const Cx<double> ap = K[3 * p + j], aq = K[3 * q + j];
                const Cx<double> cJpp{Jpp.re, -Jpp.im}, cJqp{Jqp.re, -Jqp.im};
                const Cx<double> cJpq{Jpq.re, -Jpq.im}, cJqq{Jqq.re, -Jqq.im};
                const Cx<double> x0 = cx_mul(cJpp, ap), x1 = cx_mul(cJqp, aq);
                const Cx<double> y0 = cx_mul(cJpq, ap), y1 = cx_mul(cJqq, aq);
                K[3 * p + j] = Cx<double>{x0.re + x1.re, x0.im + x1.im};
                K[3 * q + j] = Cx<double>{y0.re + y1.re, y0.im + y1.im};
            }
        }
    }
    double phi[3];
    for (int k = 0; k < 3; ++k) phi[k] = 2.0 * atan(K[4 * k].re);
    // H = gamma + Z diag(phi) Z^dag
    Cx<double> H[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Cx<double> acc{i == j ? gamma : 0.0, 0};
            for (int k = 0; k < 3; ++k) {
                const Cx<double> zi = Z[3 * i + k], zj{Z[3 * j + k].re, -Z[3 * j + k].im};
                const Cx<double> p = cx_mul(zi, zj);
                acc.re += phi[k] * p.re;
                acc.im += phi[k] * p.im;
            }
            H[3 * i + j] = acc;
        }
    h[0] = H[0].re;
    h[1] = H[4].re;
    h[2] = H[8].re;
    h[3] = 0.5 * (H[1].re + H[3].re);
    h[4] = 0.5 * (H[1].im - H[3].im);
    h[5] = 0.5 * (H[2].re + H[6].re);
    h[6] = 0.5 * (H[2].im - H[6].im);
    h[7] = 0.5 * (H[5].re + H[7].re);
    h[8] = 0.5 * (H[5].im - H[7].im);
}

}  // namespace hisq
