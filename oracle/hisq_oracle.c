/*
 * hisq_oracle.c -- plain, slow, FP64 CPU oracle for the HISQ even-odd CG.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load the library built from this file.
 * It shares no code, header, table or helper with the HIP library, and it never
 * sees the HIP library's outputs.
 *
 * Source: O. Kaczmarek, C. Schmidt, P. Steinbrecher, M. Wagner, "Conjugate
 * gradient solvers on Intel Xeon Phi and NVIDIA GPUs", GPUHEP2014.
 *
 *   orc_dslash_full   HISQ Dslash, Sec. 1 eq. (3), summed over the four lattice
 *                     directions mu = 0..3 (the printed upper limit 4 is read as
 *                     a typo for a 4-D lattice), periodic in every direction;
 *                     applied to every rhs of a bundle independently (eq. (4)).
 *   orc_dslash_eo     the same operator restricted to one output parity; D only
 *                     couples sites of opposite parity because 1 and 3 are odd hops.
 *   orc_apply_A       A = 4 m^2 - D_eo D_oe, the even block of M^dag M for the
 *                     reading M = 2m + D (the paper does not write M out).
 *   orc_cg            textbook conjugate gradient on A, one rhs at a time (the
 *                     paper names CG but does not list it); the stop test is the
 *                     true residual ||b - A x|| <= tol ||b||.
 *   orc_residual      ||b - A x|| / ||b|| per rhs.
 *   orc_force         gradient of L = sum_k Re(phi_k^dag x_k), A x_k = eta_k, with
 *                     respect to U, N (complex gradient dL/dRe + i dL/dIm) and m,
 *                     from y = A^{-1} phi, t = D_oe x and s = D_oe y.
 *   orc_r14_pack /    the 14-real compressed Naik storage of Sec. 1 (Table 1,
 *   orc_r14_unpack    "r14"): rows 0 and 1 plus one complex c with
 *                     row2 = c * conj(row0 x row1), exact for N = s * U(3).
 *   orc_r13_pack /    13 reals: rows 0 and 1 plus the phase phi of that c; its
 *   orc_r13_unpack    modulus follows from N = s V, V in U(3): |row0| = s, and
 *                     row2 = s det(V) conj(v0 x v1) = (e^{i phi} / s) conj(row0 x row1).
 *   orc_dslash_chem_eo
 *                     d^n/dmu^n of the Dslash at quark chemical potential mu,
 *                     one output parity: the operators dM/dmu of Sec. 1 eq. (2).
 *                     The paper does not write M(mu) out; the reading is the
 *                     usual one: a hop of h steps in the time direction carries
 *                     exp(h mu) (forward 1-hop e^mu, backward e^-mu, Naik e^{+-3mu}),
 *                     spatial hops carry no mu.  So the n-th derivative weights a
 *                     temporal h-hop by h^n exp(h mu) and drops spatial hops for
 *                     n >= 1; n = 0 is D(mu) itself.
 *
 * Layouts: site s = x0 + L0*(x1 + L1*(x2 + L2*x3)); links [4][V][3][3] complex;
 * full fields [V][3][n]; half fields [V/2][3][n] indexed by s/2 within a parity.
 * Complex numbers are C99 double complex, i.e. interleaved (re, im) pairs.
 *
 * Return codes: 0 ok, -1 bad argument, -2 bad geometry (any L_mu odd or < 4),
 * -3 out of memory.  orc_cg also writes a per-rhs status: 0 converged,
 * 1 maxiter reached, 2 breakdown (Re<p,Ap> <= 0 or not finite).
 */
#ifdef _OPENMP
#include <omp.h>
#endif
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex zc;

typedef struct {
    int L[4];
    long V;
    long Vh;
} lat_t;

static int lat_init(lat_t* t, const int* L)
{
    if (!L) return -1;
    t->V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (L[mu] < 4 || (L[mu] % 2) != 0) return -2;
        t->L[mu] = L[mu];
        t->V *= L[mu];
    }
    t->Vh = t->V / 2;
    return 0;
}

static void coords(const lat_t* t, long s, int x[4])
{
    for (int mu = 0; mu < 4; ++mu) {
        x[mu] = (int)(s % t->L[mu]);
        s /= t->L[mu];
    }
}

static long index_of(const lat_t* t, const int x[4])
{
    return x[0] + (long)t->L[0] * (x[1] + (long)t->L[1] * (x[2] + (long)t->L[2] * x[3]));
}

/* site reached from s by h steps in direction mu, periodic */
static long hop(const lat_t* t, long s, int mu, int h)
{
    int x[4];
    coords(t, s, x);
    x[mu] = ((x[mu] + h) % t->L[mu] + t->L[mu]) % t->L[mu];
    return index_of(t, x);
}

static int parity_of(const lat_t* t, long s)
{
    int x[4];
    coords(t, s, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* Matrix element (a, b) of link (mu, s) of a [4][V][3][3] array. */
static zc link_el(const zc* W, const lat_t* t, int mu, long s, int a, int b)
{
    return W[((long)mu * t->V + s) * 9 + 3 * a + b];
}

/*
 * One output site of eq. (3) for all n rhs:
 *   w_x = sum_mu [ U_{x,mu} v_{x+mu} - U^dag_{x-mu,mu} v_{x-mu}
 *                + N_{x,mu} v_{x+3mu} - N^dag_{x-3mu,mu} v_{x-3mu} ].
 * vidx(s) maps a full-lattice site to the row of v that holds it.  Where two of
 * the hops reach the same site (L_mu = 4 or 6) the contributions add.
 */
static void dslash_site(const lat_t* t, int n, const zc* U, const zc* N,
                        const zc* v, long (*vidx)(long), long x, zc* w)
{
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n; ++k) w[a * n + k] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        long xp1 = hop(t, x, mu, +1), xm1 = hop(t, x, mu, -1);
        long xp3 = hop(t, x, mu, +3), xm3 = hop(t, x, mu, -3);
        long ip1 = vidx(xp1), im1 = vidx(xm1), ip3 = vidx(xp3), im3 = vidx(xm3);
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k < n; ++k) {
                zc acc = 0;
                for (int b = 0; b < 3; ++b) {
                    acc += link_el(U, t, mu, x, a, b) * v[(ip1 * 3 + b) * n + k];
                    acc -= conj(link_el(U, t, mu, xm1, b, a)) * v[(im1 * 3 + b) * n + k];
                    acc += link_el(N, t, mu, x, a, b) * v[(ip3 * 3 + b) * n + k];
                    acc -= conj(link_el(N, t, mu, xm3, b, a)) * v[(im3 * 3 + b) * n + k];
                }
                w[a * n + k] += acc;
            }
        }
    }
}

static long ident(long s) { return s; }
static long halve(long s) { return s / 2; }

/* h^n exp(h mu): the n-th mu-derivative of the weight of an h-step temporal hop */
static double hop_weight(int h, int nder, double mu)
{
    double w = exp(h * mu);
    for (int j = 0; j < nder; ++j) w *= h;
    return w;
}

/* One output site of d^n D(mu) / d mu^n (reading above), all n rhs. */
static void dslash_chem_site(const lat_t* t, int n, const zc* U, const zc* N, const zc* v,
                             long x, double mu_c, int nder, zc* w)
{
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < n; ++k) w[a * n + k] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        double wp1, wm1, wp3, wm3;
        if (mu == 3) {
            wp1 = hop_weight(+1, nder, mu_c);
            wm1 = hop_weight(-1, nder, mu_c);
            wp3 = hop_weight(+3, nder, mu_c);
            wm3 = hop_weight(-3, nder, mu_c);
        } else {
            wp1 = wm1 = wp3 = wm3 = nder == 0 ? 1.0 : 0.0;
        }
        long xp1 = hop(t, x, mu, +1), xm1 = hop(t, x, mu, -1);
        long xp3 = hop(t, x, mu, +3), xm3 = hop(t, x, mu, -3);
        long ip1 = xp1 / 2, im1 = xm1 / 2, ip3 = xp3 / 2, im3 = xm3 / 2;
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k < n; ++k) {
                zc acc = 0;
                for (int b = 0; b < 3; ++b) {
                    acc += wp1 * link_el(U, t, mu, x, a, b) * v[(ip1 * 3 + b) * n + k];
                    acc -= wm1 * conj(link_el(U, t, mu, xm1, b, a)) * v[(im1 * 3 + b) * n + k];
                    acc += wp3 * link_el(N, t, mu, x, a, b) * v[(ip3 * 3 + b) * n + k];
                    acc -= wm3 * conj(link_el(N, t, mu, xm3, b, a)) * v[(im3 * 3 + b) * n + k];
                }
                w[a * n + k] += acc;
            }
        }
    }
}

int orc_dslash_chem_eo(const int* L, int n, int out_parity, const double* U, const double* N,
                       double mu_c, int nder, const double* in, double* out)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || nder < 0 || (out_parity != 0 && out_parity != 1) || !U || !N || !in || !out)
        return -1;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < t.V; ++x) {
        if (parity_of(&t, x) != out_parity) continue;
        dslash_chem_site(&t, n, (const zc*)U, (const zc*)N, (const zc*)in, x, mu_c, nder,
                         (zc*)out + (x / 2) * 3 * n);
    }
    return 0;
}

int orc_dslash_full(const int* L, int n, const double* U, const double* N,
                    const double* v, double* w)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || !U || !N || !v || !w) return -1;
    const zc* Uc = (const zc*)U;
    const zc* Nc = (const zc*)N;
    const zc* vc = (const zc*)v;
    zc* wc = (zc*)w;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < t.V; ++x)
        dslash_site(&t, n, Uc, Nc, vc, ident, x, wc + x * 3 * n);
    return 0;
}

/* out (parity out_parity) = D restricted to in (parity 1 - out_parity) */
static void dslash_eo_c(const lat_t* t, int n, int out_parity, const zc* U, const zc* N,
                        const zc* in, zc* out)
{
#pragma omp parallel for schedule(static)
    for (long x = 0; x < t->V; ++x) {
        if (parity_of(t, x) != out_parity) continue;
        dslash_site(t, n, U, N, in, halve, x, out + (x / 2) * 3 * n);
    }
}

int orc_dslash_eo(const int* L, int n, int out_parity, const double* U, const double* N,
                  const double* in, double* out)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || (out_parity != 0 && out_parity != 1) || !U || !N || !in || !out) return -1;
    dslash_eo_c(&t, n, out_parity, (const zc*)U, (const zc*)N, (const zc*)in, (zc*)out);
    return 0;
}

/*
 * The same half-lattice Dslash evaluated only at `count` chosen output sites
 * (full-lattice indices, all of parity out_parity): out[j] = (D in)_{sites[j]},
 * shape [count][3][n].  Used to check outputs of very large lattices site by site.
 */
int orc_dslash_sites(const int* L, int n, int out_parity, const double* U, const double* N,
                     const double* in, long count, const long* sites, double* out)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || (out_parity != 0 && out_parity != 1) || !U || !N || !in || !out || count < 0 ||
        (count > 0 && !sites))
        return -1;
    for (long j = 0; j < count; ++j)
        if (sites[j] < 0 || sites[j] >= t.V || parity_of(&t, sites[j]) != out_parity) return -1;
#pragma omp parallel for schedule(static)
    for (long j = 0; j < count; ++j)
        dslash_site(&t, n, (const zc*)U, (const zc*)N, (const zc*)in, halve, sites[j],
                    (zc*)out + j * 3 * n);
    return 0;
}

/* y = A x = 4 m^2 x - D_eo (D_oe x) on even half fields */
static int apply_A_c(const lat_t* t, int n, double m, const zc* U, const zc* N,
                     const zc* x, zc* y)
{
    long len = t->Vh * 3 * n;
    zc* tmp = (zc*)malloc(sizeof(zc) * (size_t)len);
    zc* u = (zc*)malloc(sizeof(zc) * (size_t)len);
    if (!tmp || !u) {
        free(tmp);
        free(u);
        return -3;
    }
    dslash_eo_c(t, n, 1, U, N, x, tmp);
    dslash_eo_c(t, n, 0, U, N, tmp, u);
    for (long i = 0; i < len; ++i) y[i] = 4.0 * m * m * x[i] - u[i];
    free(tmp);
    free(u);
    return 0;
}

int orc_apply_A(const int* L, int n, double m, const double* U, const double* N,
                const double* x, double* y)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || !U || !N || !x || !y) return -1;
    return apply_A_c(&t, n, m, (const zc*)U, (const zc*)N, (const zc*)x, (zc*)y);
}

static zc dot(long len, const zc* a, const zc* b)
{
    zc s = 0;
    for (long i = 0; i < len; ++i) s += conj(a[i]) * b[i];
    return s;
}

static double norm2(long len, const zc* a)
{
    double s = 0;
    for (long i = 0; i < len; ++i) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

/*
 * Conjugate gradient for A x = b, one rhs (half fields with n = 1).
 * x holds the start vector on entry.  The iterated residual is used until it
 * drops below tol^2 ||b||^2; then the true residual b - A x is formed, and the
 * solve ends if it passes, else restarts from it with p = r.
 */
static int cg_one(const lat_t* t, double m, const zc* U, const zc* N, const zc* b, zc* x,
                  double tol, int maxiter, int* iters, double* true_res, double* iter_res)
{
    long len = t->Vh * 3;
    zc* r = (zc*)malloc(sizeof(zc) * (size_t)len);
    zc* p = (zc*)malloc(sizeof(zc) * (size_t)len);
    zc* q = (zc*)malloc(sizeof(zc) * (size_t)len);
    int status = 1, it = 0, rc;
    double bb, rr, rr_new = 0;
    if (!r || !p || !q) {
        free(r);
        free(p);
        free(q);
        return -3;
    }
    bb = norm2(len, b);
    *iters = 0;
    if (bb == 0.0) {
        memset(x, 0, sizeof(zc) * (size_t)len);
        *true_res = 0;
        *iter_res = 0;
        free(r);
        free(p);
        free(q);
        return 0;
    }
    rc = apply_A_c(t, 1, m, U, N, x, q);
    if (rc) goto out;
    for (long i = 0; i < len; ++i) r[i] = b[i] - q[i];
    memcpy(p, r, sizeof(zc) * (size_t)len);
    rr = norm2(len, r);
    rr_new = rr;
    if (rr <= tol * tol * bb) {
        status = 0;
        goto done;
    }
    while (it < maxiter) {
        rc = apply_A_c(t, 1, m, U, N, p, q);
        if (rc) goto out;
        double pq = creal(dot(len, p, q));
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = 2;
            break;
        }
        double alpha = rr / pq;
        for (long i = 0; i < len; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++it;
        rr_new = norm2(len, r);
        if (!isfinite(rr_new)) {
            status = 2;
            break;
        }
        if (rr_new <= tol * tol * bb) {
            rc = apply_A_c(t, 1, m, U, N, x, q);
            if (rc) goto out;
            for (long i = 0; i < len; ++i) r[i] = b[i] - q[i];
            double rr_true = norm2(len, r);
            if (rr_true <= tol * tol * bb) {
                status = 0;
                break;
            }
            memcpy(p, r, sizeof(zc) * (size_t)len);
            rr = rr_true;
            continue;
        }
        double beta = rr_new / rr;
        for (long i = 0; i < len; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
done:
    *iters = it;
    *iter_res = sqrt(rr_new / bb);
    rc = apply_A_c(t, 1, m, U, N, x, q);
    if (rc) goto out;
    {
        double rt = 0;
        for (long i = 0; i < len; ++i) {
            zc d = b[i] - q[i];
            rt += creal(d) * creal(d) + cimag(d) * cimag(d);
        }
        *true_res = sqrt(rt / bb);
    }
    rc = status;
out:
    free(r);
    free(p);
    free(q);
    return rc;
}

/* Split rhs k out of a [Vh][3][n] bundle, or put it back. */
static void take_rhs(long Vh, int n, int k, const zc* bundle, zc* one)
{
    for (long i = 0; i < Vh * 3; ++i) one[i] = bundle[i * n + k];
}

static void put_rhs(long Vh, int n, int k, const zc* one, zc* bundle)
{
    for (long i = 0; i < Vh * 3; ++i) bundle[i * n + k] = one[i];
}

/*
 * Solve A x_k = b_k for each rhs of the bundle independently (eq. (4)).
 * x holds the start vectors on entry (zeros for x0 = 0).
 */
int orc_cg(const int* L, int n, double m, const double* U, const double* N, const double* b,
           double* x, double tol, int maxiter, int* iters, double* true_res, double* iter_res,
           int* status)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || !U || !N || !b || !x || !iters || !true_res || !iter_res || !status ||
        !(tol > 0) || maxiter < 0)
        return -1;
    zc* b1 = (zc*)malloc(sizeof(zc) * (size_t)(t.Vh * 3));
    zc* x1 = (zc*)malloc(sizeof(zc) * (size_t)(t.Vh * 3));
    if (!b1 || !x1) {
        free(b1);
        free(x1);
        return -3;
    }
    int worst = 0;
    for (int k = 0; k < n; ++k) {
        take_rhs(t.Vh, n, k, (const zc*)b, b1);
        take_rhs(t.Vh, n, k, (const zc*)x, x1);
        int s = cg_one(&t, m, (const zc*)U, (const zc*)N, b1, x1, tol, maxiter, &iters[k],
                       &true_res[k], &iter_res[k]);
        if (s < 0) {
            free(b1);
            free(x1);
            return s;
        }
        status[k] = s;
        if (s > worst) worst = s;
        put_rhs(t.Vh, n, k, x1, (zc*)x);
    }
    free(b1);
    free(x1);
    return worst;
}

int orc_residual(const int* L, int n, double m, const double* U, const double* N,
                 const double* b, const double* x, double* rel)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || !U || !N || !b || !x || !rel) return -1;
    long len = t.Vh * 3 * n;
    zc* q = (zc*)malloc(sizeof(zc) * (size_t)len);
    if (!q) return -3;
    rc = apply_A_c(&t, n, m, (const zc*)U, (const zc*)N, (const zc*)x, q);
    if (rc) {
        free(q);
        return rc;
    }
    const zc* bc = (const zc*)b;
    for (int k = 0; k < n; ++k) {
        double num = 0, den = 0;
        for (long i = 0; i < t.Vh * 3; ++i) {
            zc d = bc[i * n + k] - q[i * n + k];
            num += creal(d) * creal(d) + cimag(d) * cimag(d);
            den += creal(bc[i * n + k]) * creal(bc[i * n + k]) +
                   cimag(bc[i * n + k]) * cimag(bc[i * n + k]);
        }
        rel[k] = den > 0 ? sqrt(num / den) : sqrt(num);
    }
    free(q);
    return 0;
}

/* G += sign * sum_k u_k v_k^dag for 3-vectors u, v held in [3][n] rows */
static void outer_acc(int n, double sign, const zc* u, const zc* v, zc* G)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            zc s = 0;
            for (int k = 0; k < n; ++k) s += u[i * n + k] * conj(v[j * n + k]);
            G[3 * i + j] += sign * s;
        }
}

/*
 * Gradient of L = sum_k Re(phi_k^dag x_k) with A x_k = eta_k, given x and
 * y = A^{-1} phi (both even).  With t = D_oe x and s = D_oe y, varying A gives
 *   dL = -8 m dm sum_k Re(y_k^dag x_k) + sum_k [Re y^dag dD_eo t - Re s^dag dD_oe x],
 * because y^dag D_eo = -(D_oe y)^dag (D is anti-Hermitian).  Collecting the
 * terms of eq. (3) that contain a given link (a, mu), with b = a + mu
 * (a + 3 mu for N), and the convention that Re(u^dag dW v) has gradient u v^dag:
 *   a even:  G[a, mu] =  sum_k ( y_a t_b^dag + x_a s_b^dag )
 *   a odd :  G[a, mu] = -sum_k ( t_a y_b^dag + s_a x_b^dag )
 * U and N are independent inputs.  dL/dm = -8 m sum_k Re(y_k^dag x_k).
 */
int orc_force(const int* L, int n, double m, const double* U, const double* N,
              const double* x, const double* y, double* GU, double* GN, double* dm)
{
    lat_t t;
    int rc = lat_init(&t, L);
    if (rc) return rc;
    if (n < 1 || !U || !N || !x || !y || !GU || !GN || !dm) return -1;
    long len = t.Vh * 3 * n;
    zc* tx = (zc*)malloc(sizeof(zc) * (size_t)len);
    zc* sy = (zc*)malloc(sizeof(zc) * (size_t)len);
    if (!tx || !sy) {
        free(tx);
        free(sy);
        return -3;
    }
    const zc* xc = (const zc*)x;
    const zc* yc = (const zc*)y;
    dslash_eo_c(&t, n, 1, (const zc*)U, (const zc*)N, xc, tx);
    dslash_eo_c(&t, n, 1, (const zc*)U, (const zc*)N, yc, sy);
    zc* GUc = (zc*)GU;
    zc* GNc = (zc*)GN;
    for (int pass = 0; pass < 2; ++pass) {
        zc* G = pass == 0 ? GUc : GNc;
        int h = pass == 0 ? 1 : 3;
#pragma omp parallel for schedule(static)
        for (long a = 0; a < t.V; ++a) {
            for (int mu = 0; mu < 4; ++mu) {
                zc* g = G + ((long)mu * t.V + a) * 9;
                for (int e = 0; e < 9; ++e) g[e] = 0;
                long bs = hop(&t, a, mu, h);
                long ia = (a / 2) * 3 * n, ib = (bs / 2) * 3 * n;
                if (parity_of(&t, a) == 0) {
                    outer_acc(n, +1.0, yc + ia, tx + ib, g);
                    outer_acc(n, +1.0, xc + ia, sy + ib, g);
                } else {
                    outer_acc(n, -1.0, tx + ia, yc + ib, g);
                    outer_acc(n, -1.0, sy + ia, xc + ib, g);
                }
            }
        }
    }
    *dm = -8.0 * m * creal(dot(len, yc, xc));
    free(tx);
    free(sy);
    return 0;
}

/*
 * r14: store rows 0 and 1 of W (12 reals) and c (2 reals) such that
 * row2 = c * conj(row0 x row1).  For W = s V with V in U(3) and s > 0 this is
 * exact with c = det(V) / s.  c is fitted by least squares; max_err receives the
 * largest round-trip error ||row2 - c conj(row0 x row1)|| / ||W||_F.
 */
static void cross_conj(const zc* r0, const zc* r1, zc* out)
{
    out[0] = conj(r0[1] * r1[2] - r0[2] * r1[1]);
    out[1] = conj(r0[2] * r1[0] - r0[0] * r1[2]);
    out[2] = conj(r0[0] * r1[1] - r0[1] * r1[0]);
}

int orc_r14_pack(long count, const double* M, double* packed, double* max_err)
{
    if (count < 0 || !M || !packed || !max_err) return -1;
    double worst = 0;
    const zc* Mc = (const zc*)M;
    for (long i = 0; i < count; ++i) {
        const zc* W = Mc + i * 9;
        zc cr[3];
        cross_conj(W, W + 3, cr);
        zc num = 0;
        double den = 0, fro = 0, err = 0;
        for (int j = 0; j < 3; ++j) {
            num += conj(cr[j]) * W[6 + j];
            den += creal(cr[j]) * creal(cr[j]) + cimag(cr[j]) * cimag(cr[j]);
        }
        zc c = den > 0 ? num / den : 0;
        for (int e = 0; e < 9; ++e) fro += creal(W[e]) * creal(W[e]) + cimag(W[e]) * cimag(W[e]);
        for (int j = 0; j < 3; ++j) {
            zc d = W[6 + j] - c * cr[j];
            err += creal(d) * creal(d) + cimag(d) * cimag(d);
        }
        err = fro > 0 ? sqrt(err / fro) : 0;
        if (err > worst || isnan(err)) worst = err;
        double* P = packed + i * 14;
        for (int e = 0; e < 6; ++e) {
            P[2 * e] = creal(W[e]);
            P[2 * e + 1] = cimag(W[e]);
        }
        P[12] = creal(c);
        P[13] = cimag(c);
    }
    *max_err = worst;
    return 0;
}

int orc_r14_unpack(long count, const double* packed, double* M)
{
    if (count < 0 || !packed || !M) return -1;
    zc* Mc = (zc*)M;
    for (long i = 0; i < count; ++i) {
        const double* P = packed + i * 14;
        zc* W = Mc + i * 9;
        for (int e = 0; e < 6; ++e) W[e] = P[2 * e] + I * P[2 * e + 1];
        zc c = P[12] + I * P[13];
        zc cr[3];
        cross_conj(W, W + 3, cr);
        for (int j = 0; j < 3; ++j) W[6 + j] = c * cr[j];
    }
    return 0;
}

/*
 * r13: rows 0 and 1 (12 reals) and phi = arg(c), where for N = s V, V in U(3),
 * row2 = c conj(row0 x row1) with c = det(V) / s and s = |row0|.  Here phi is
 * taken from det(N) = s^3 det(V); max_err as for r14.
 */
int orc_r13_unpack(long count, const double* packed, double* M);

int orc_r13_pack(long count, const double* M, double* packed, double* max_err)
{
    if (count < 0 || !M || !packed || !max_err) return -1;
    const zc* A = (const zc*)M;
    double worst = 0;
    for (long j = 0; j < count; ++j) {
        const zc* m = A + 9 * j;
        double* p = packed + 13 * j;
        for (int e = 0; e < 6; ++e) {
            p[2 * e] = creal(m[e]);
            p[2 * e + 1] = cimag(m[e]);
        }
        const zc det = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                       m[2] * (m[3] * m[7] - m[4] * m[6]);
        p[12] = carg(det);
        zc back[9];
        orc_r13_unpack(1, p, (double*)back);
        double err = 0, fro = 0;
        for (int e = 0; e < 9; ++e) {
            err += cabs(back[e] - m[e]) * cabs(back[e] - m[e]);
            fro += cabs(m[e]) * cabs(m[e]);
        }
        const double rel = fro > 0 ? sqrt(err / fro) : 0;
        if (!(rel <= worst)) worst = rel;
    }
    *max_err = worst;
    return 0;
}

int orc_r13_unpack(long count, const double* packed, double* M)
{
    if (count < 0 || !packed || !M) return -1;
    zc* A = (zc*)M;
    for (long j = 0; j < count; ++j) {
        const double* p = packed + 13 * j;
        zc* m = A + 9 * j;
        for (int e = 0; e < 6; ++e) m[e] = p[2 * e] + I * p[2 * e + 1];
        const double s = sqrt(creal(m[0] * conj(m[0]) + m[1] * conj(m[1]) + m[2] * conj(m[2])));
        const zc c = s > 0 ? cexp(I * p[12]) / s : 0;
        zc w[3];
        cross_conj(m, m + 3, w);
        for (int k = 0; k < 3; ++k) m[6 + k] = c * w[k];
    }
    return 0;
}

/* Threads the oracle's OpenMP loops use from now on (k >= 1). */
int orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k >= 1) omp_set_num_threads(k);
#else
    (void)k;
#endif
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
