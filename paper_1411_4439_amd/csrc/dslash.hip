// HISQ half-Dslash kernels for gfx950 (Sec. 1, eqs. (3) and (4)).
//
// One thread computes NR rhs of one output site; the G = n/NR threads of a
// site are adjacent lanes, so their spinor loads are contiguous and their link
// loads hit the same cache line.  Per output site the thread streams the 16
// matrices of its parity block once (non-temporal loads: links have no reuse
// within a half-Dslash) and gathers the 16 neighbour colour vectors of its rhs
// tile; the neighbour vectors are re-read by up to 16 sites and are served from
// L2 / Infinity Cache.  All accumulation is in the storage precision; the CG
// dot products are accumulated in FP64.
//
// This file is compiled once per (precision, Naik storage, epilogue):
//   HISQ_KPREC 0 = FP64, 1 = FP32, 2 = FP32 with r14 Naik links,
//              3 = FP32 with r13 Naik links, 4 = FP32 with r9 Naik links
//   HISQ_KEPI  one of EPI_PLAIN, EPI_NORM, EPI_CG, EPI_RESID
#include <type_traits>

#include "naik.h"
#include "stencil.h"

#ifndef HISQ_KPREC
#error "HISQ_KPREC must be defined"
#endif
#ifndef HISQ_KEPI
#error "HISQ_KEPI must be defined"
#endif

namespace hisq {

#if HISQ_KPREC == 0
using KT = double;
constexpr int kNK = HISQ_NAIK_FULL;
#elif HISQ_KPREC == 1
using KT = float;
constexpr int kNK = HISQ_NAIK_FULL;
#elif HISQ_KPREC == 2
using KT = float;
constexpr int kNK = HISQ_NAIK_R14;
#elif HISQ_KPREC == 3
using KT = float;
constexpr int kNK = HISQ_NAIK_R13;
#else
using KT = float;
constexpr int kNK = HISQ_NAIK_R9;
#endif

template <typename T, int NRHS, int NR, bool CM>
__device__ __forceinline__ void load_vec(const cplx<T>* __restrict__ in, int Vh, int nbr, int g,
                                         cplx<T> (&v)[3][NR])
{
    using Lay = Layout<NRHS, CM>;
    const cplx<T>* vp = in + Lay::site(nbr) + g * NR;
#pragma unroll
    for (int b = 0; b < 3; ++b) load_rhs<NR>(vp + Lay::colour(b, Vh), v[b]);
}

// Naik storage r13: c = exp(i phi) / |row0|, phi loaded into m[6].x (for
// N = s V, V in U(3): |row0| = s and c = det V / s)
template <typename T>
__device__ __forceinline__ cplx<T> r13_coefficient(const cplx<T> (&m)[9])
{
    static_assert(sizeof(T) == 4, "r13 is an FP32 storage");
    const float n2 = m[0].x * m[0].x + m[0].y * m[0].y + m[1].x * m[1].x + m[1].y * m[1].y +
                     m[2].x * m[2].x + m[2].y * m[2].y;
    float cs, sn;
    unit_phase(m[6].x, &cs, &sn);
    const float inv = __builtin_amdgcn_rsqf(n2);
    return cplx<T>{cs * inv, sn * inv};
}

// Naik storage r9: m[0..3] and m[4].x hold the 9 reals of H; the matrix is
// ns exp(iH), ns the field's Naik scale.
template <typename T>
__device__ __forceinline__ void r9_matrix(cplx<T> (&m)[9], T ns)
{
    static_assert(sizeof(T) == 4, "r9 is an FP32 storage");
    const T h[9] = {m[0].x, m[0].y, m[1].x, m[1].y, m[2].x, m[2].y, m[3].x, m[3].y, m[4].x};
    T re[9], im[9];
    expi_hermitian<T>(h, ns, re, im);
#pragma unroll
    for (int e = 0; e < 9; ++e) m[e] = cplx<T>{re[e], im[e]};
}

template <typename T, int NR, int NK, int S>
__device__ __forceinline__ void apply_slot(cplx<T> (&m)[9], const cplx<T> (&v)[3][NR],
                                           cplx<T> (&acc)[3][NR], T ns)
{
    if constexpr (NK == HISQ_NAIK_R9 && S >= 8) {
        r9_matrix<T>(m, ns);
    } else if constexpr (NK != HISQ_NAIK_FULL && S >= 8) {
        // row 2 = c * conj(row0 x row1); r14 loaded c into m[6], r13 its phase
        cplx<T> cc = m[6];
        if constexpr (NK == HISQ_NAIK_R13) cc = r13_coefficient<T>(m);
        m[6] = cmul(cc, cconj(cmul(m[1], m[5]) - cmul(m[2], m[4])));
        m[7] = cmul(cc, cconj(cmul(m[2], m[3]) - cmul(m[0], m[5])));
        m[8] = cmul(cc, cconj(cmul(m[0], m[4]) - cmul(m[1], m[3])));
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int k = 0; k < NR; ++k) cfma(acc[a][k], m[3 * a + b], v[b][k]);
}

// Pipeline step k -> slot: even steps take the z and t slots, odd steps the x
// and y slots, hops +1, -1, +3, -3 within each direction.  The LDS-staged
// kernel reads the x and y neighbours from LDS and overlaps them with the
// global z and t reads; the unstaged kernel sums the slots in the same order,
// so the two give bitwise identical results.
__host__ __device__ constexpr int slot_at(int k)
{
    return ((k & 1) ? ((k >> 3) & 1) : 2 + ((k >> 3) & 1)) + 4 * ((k >> 1) & 3);
}

// acc[c][k] = (D in)_{i}, colour c, rhs g*NR + k, output parity P.
// Slot s = 4*hop + mu applies matrix s of the parity block to the neighbour
// reached by hop (+1, -1, +3, -3) in direction mu.  The 16 slots run as a
// software pipeline: while one slot is multiplied, the neighbour vectors of
// the next slot and its matrix are in flight (links stream from HBM and see
// the longest latency; neighbour vectors mostly hit L2).  The scheduling
// barriers keep the compiler from hoisting further loads, which would
// otherwise exhaust the register file.
template <typename T, int NRHS, int NR, int NK, bool CM>
__device__ __forceinline__ void dslash_site(const Lat& lat, int P, int i, int g,
                                            const cplx<T>* __restrict__ lk,
                                            const cplx<T>* __restrict__ in,
                                            cplx<T> (&acc)[3][NR], T ns)
{
    using C = cplx<T>;
    const int Vh = lat.Vh;
    const SiteCoord sc = site_coord(lat, P, i);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[c][k] = C{0, 0};

    // link lookahead: two slots in FP32; one in FP64, whose 36-register
    // matrices would otherwise cost a wave of occupancy
#ifndef HISQ_FP32_LINK_LOOKAHEAD
#define HISQ_FP32_LINK_LOOKAHEAD 1
#endif
    constexpr int LD = sizeof(T) == 4 ? HISQ_FP32_LINK_LOOKAHEAD : 1;
    // lanes sharing a link: the site's lanes, in quads when there are 8
    constexpr int G = (NRHS / NR) < 4 ? NRHS / NR : 4;
    const int gl = g % G;
    LinkRaw<T, G> lr[LD + 1];
    C v[2][3][NR];
    load_link_part<T, NK, slot_at(0), G>(lk, Vh, i, gl, lr[0]);
    if constexpr (LD == 2) load_link_part<T, NK, slot_at(1), G>(lk, Vh, i, gl, lr[1]);
    load_vec<T, NRHS, NR, CM>(in, Vh, neighbour<slot_at(0)>(lat, sc), g, v[0]);
    static_for<0, 16>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (k + LD < 16)
            load_link_part<T, NK, slot_at(k + LD), G>(lk, Vh, i, gl, lr[(k + LD) % (LD + 1)]);
        if constexpr (k + 1 < 16)
            load_vec<T, NRHS, NR, CM>(in, Vh, neighbour<slot_at(k + 1)>(lat, sc), g, v[(k + 1) & 1]);
        __builtin_amdgcn_sched_barrier(0);
        C m[9];
        share_link<T, NK, slot_at(k), G>(lr[k % (LD + 1)], m);
        apply_slot<T, NR, NK, slot_at(k)>(m, v[k & 1], acc, ns);
        __builtin_amdgcn_sched_barrier(0);
    });
}

// ---------------------------------------------------------------------------
// LDS-staged form (colour-major fields).  A work-group covers R whole x-rows
// of one (z, t) plane.  The input rows y0-3 .. y0+R+2 of that plane (periodic
// in y) are copied to LDS once, laid out [3][R+6][L0/2][n]; the x and y
// neighbours (8 of the 16 slots) are then read from LDS and only the z and t
// neighbours and the links come from global memory.

template <typename T, int NRHS>
__device__ __forceinline__ void stage_rows(const cplx<T>* __restrict__ in, cplx<T>* lds,
                                           const Lat& lat, int row0, int R)
{
    const int Ly = lat.L[1];
    const int plane = row0 / Ly, y0 = row0 - plane * Ly;
    const unsigned rows = (unsigned)R + 6;
    // half-site of staged row j (y0 - 3 + j, periodic; Ly >= 4 > 3)
    auto row_site = [&](unsigned j) -> size_t {
        int yy = y0 - 3 + (int)j;
        yy += yy < 0 ? Ly : 0;
        yy -= yy >= Ly ? Ly : 0;
        return (size_t)(plane * Ly + yy) * lat.Lh0;
    };
    // Each thread copies its units in batches of kStageBatch: all the batch's
    // reads are issued before the first LDS write, so a thread waits for one
    // memory round trip per batch instead of one per unit.
    constexpr unsigned kStageBatch = 16;
    const unsigned nt = blockDim.x;
    // unit u -> (colour c, staged row j, offset): u / chunk through a float
    // reciprocal with a one-step correction (u < 2^16 here, so the estimate
    // is off by at most one), c by comparisons (c < 3)
    auto split = [rows](unsigned u, unsigned chunk, float inv, unsigned& c, unsigned& j,
                        unsigned& off) {
        unsigned cj = (unsigned)((float)u * inv);
        int r = (int)u - (int)(cj * chunk);
        if (r < 0) {
            --cj;
            r += (int)chunk;
        } else if (r >= (int)chunk) {
            ++cj;
            r -= (int)chunk;
        }
        off = (unsigned)r;
        c = (cj >= rows ? 1u : 0u) + (cj >= 2 * rows ? 1u : 0u);
        j = cj - c * rows;
    };
    if constexpr (sizeof(T) == 4) {
        if ((lat.Lh0 * NRHS) % 2 == 0) {
            // 16-byte units of two complex numbers
            const unsigned chunk = (unsigned)(lat.Lh0 * NRHS / 2);
            const unsigned total = 3u * rows * chunk;
            const float inv = 1.0f / (float)chunk;
            const f4* src = reinterpret_cast<const f4*>(in);
            f4* dst = reinterpret_cast<f4*>(lds);
            for (unsigned u0 = threadIdx.x; u0 < total; u0 += kStageBatch * nt) {
                f4 buf[kStageBatch];
#pragma unroll
                for (unsigned q = 0; q < kStageBatch; ++q) {
                    const unsigned u = u0 + q * nt;
                    if (u < total) {
                        unsigned c, j, off;
                        split(u, chunk, inv, c, j, off);
                        buf[q] = src[((size_t)c * lat.Vh + row_site(j)) * NRHS / 2 + off];
                    }
                }
#pragma unroll
                for (unsigned q = 0; q < kStageBatch; ++q)
                    if (u0 + q * nt < total) dst[u0 + q * nt] = buf[q];
            }
            return;
        }
    }
    const unsigned chunk = (unsigned)(lat.Lh0 * NRHS);
    const unsigned total = 3u * rows * chunk;
    const float inv = 1.0f / (float)chunk;
    for (unsigned u0 = threadIdx.x; u0 < total; u0 += kStageBatch * nt) {
        cplx<T> buf[kStageBatch];
#pragma unroll
        for (unsigned q = 0; q < kStageBatch; ++q) {
            const unsigned u = u0 + q * nt;
            if (u < total) {
                unsigned c, j, off;
                split(u, chunk, inv, c, j, off);
                buf[q] = in[((size_t)c * lat.Vh + row_site(j)) * NRHS + off];
            }
        }
#pragma unroll
        for (unsigned q = 0; q < kStageBatch; ++q)
            if (u0 + q * nt < total) lds[u0 + q * nt] = buf[q];
    }
}

template <typename T, int NRHS, int NR>
__device__ __forceinline__ void load_vec_lds(const cplx<T>* lds, int cstride, int site, int g,
                                             cplx<T> (&v)[3][NR])
{
    const cplx<T>* vp = lds + site * NRHS + g * NR;
#pragma unroll
    for (int b = 0; b < 3; ++b) load_rhs<NR>(vp + b * cstride, v[b]);
}

// Staged row-local index of the x / y neighbour of slot S (mu = 0 or 1) of the
// output site in row r of the tile, half-x xh, full x coordinate x.
template <int S>
__device__ __forceinline__ int lds_neighbour(const Lat& lat, int r, int xh, int x)
{
    constexpr int mu = S & 3;
    constexpr int hh = S >> 2;
    constexpr int h = hh == 0 ? 1 : hh == 1 ? -1 : hh == 2 ? 3 : -3;
    static_assert(mu < 2, "only x and y neighbours are staged");
    if constexpr (mu == 0) {
        const int xp = x + wrap_delta(x, h, lat.L[0]);
        return (r + 3) * lat.Lh0 + (xp >> 1);
    } else {
        return (r + 3 + h) * lat.Lh0 + xh;
    }
}

// As dslash_site, for the site in row r of an LDS-staged tile.  Issue order
// follows use order, because a wait for one global read is a wait for every
// read issued before it: an even (global) step issues the next link, computes,
// then issues the link after that and the global neighbour of four steps ahead
// (two global slots of lookahead), and the LDS neighbour of the next step.
// The global reads that open the pipeline (slot 0's link, the first two
// global neighbours): issued before the work-group's staging barrier, so
// that their latency overlaps the staging reads instead of following them.
// lanes that share one site's link loads (quads when a site has 8 lanes)
template <int NRHS, int NR>
constexpr int link_group() { return (NRHS / NR) < 4 ? NRHS / NR : 4; }

template <typename T, int NRHS, int NR, int NK>
struct LdsHead {
    LinkRaw<T, link_group<NRHS, NR>()> m;
    cplx<T> v0[3][NR], v1[3][NR];
};

template <typename T, int NRHS, int NR, int NK>
__device__ __forceinline__ void lds_head(const Lat& lat, int P, int i, int g,
                                         const cplx<T>* __restrict__ lk,
                                         const cplx<T>* __restrict__ in, LdsHead<T, NRHS, NR, NK>& h)
{
    const SiteCoord sc = site_coord(lat, P, i);
    constexpr int G = link_group<NRHS, NR>();
    load_link_part<T, NK, slot_at(0), G>(lk, lat.Vh, i, g % G, h.m);
    load_vec<T, NRHS, NR, true>(in, lat.Vh, neighbour<slot_at(0)>(lat, sc), g, h.v0);
    load_vec<T, NRHS, NR, true>(in, lat.Vh, neighbour<slot_at(2)>(lat, sc), g, h.v1);
}

template <typename T, int NRHS, int NR, int NK>
__device__ __forceinline__ void dslash_site_lds(const Lat& lat, int P, int i, int g, int r,
                                                const cplx<T>* __restrict__ lk,
                                                const cplx<T>* __restrict__ in,
                                                const cplx<T>* lds, int rows,
                                                const LdsHead<T, NRHS, NR, NK>& h,
                                                cplx<T> (&acc)[3][NR], T ns)
{
    using C = cplx<T>;
    const int Vh = lat.Vh;
    const SiteCoord sc = site_coord(lat, P, i);
    const int xh = i - sc.row;
    const int cstride = rows * lat.Lh0 * NRHS;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < NR; ++k) acc[c][k] = C{0, 0};
    constexpr int G = link_group<NRHS, NR>();
    const int gl = g % G;
    LinkRaw<T, G> m[2];
    C vg[2][3][NR];
    C vl[3][NR];
    m[0] = h.m;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            vg[0][b][k] = h.v0[b][k];
            vg[1][b][k] = h.v1[b][k];
        }
    static_for<0, 16>([&](auto K) {
        constexpr int k = decltype(K)::value;
        if constexpr (k % 2 == 0) {
            load_link_part<T, NK, slot_at(k + 1), G>(lk, Vh, i, gl, m[(k + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            C mk[9];
            share_link<T, NK, slot_at(k), G>(m[k & 1], mk);
            apply_slot<T, NR, NK, slot_at(k)>(mk, vg[(k >> 1) & 1], acc, ns);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (k + 2 < 16) load_link_part<T, NK, slot_at(k + 2), G>(lk, Vh, i, gl, m[k & 1]);
            if constexpr (k + 4 < 16)
                load_vec<T, NRHS, NR, true>(in, Vh, neighbour<slot_at(k + 4)>(lat, sc), g,
                                            vg[(k >> 1) & 1]);
            load_vec_lds<T, NRHS, NR>(lds, cstride,
                                      lds_neighbour<slot_at(k + 1)>(lat, r, xh, sc.x), g, vl);
        } else {
            C mk[9];
            share_link<T, NK, slot_at(k), G>(m[k & 1], mk);
            apply_slot<T, NR, NK, slot_at(k)>(mk, vl, acc, ns);
        }
        __builtin_amdgcn_sched_barrier(0);
    });
}

// An empty asm that reads every accumulator: keeps the compiler from sinking
// the site's arithmetic into a later conditional block (past the loads of all
// 16 slots, which would keep every loaded operand live at once).
template <typename C, int NR>
__device__ __forceinline__ void pin_acc(C (&acc)[3][NR])
{
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < NR; ++k) asm volatile("" ::"v"(acc[c][k].x), "v"(acc[c][k].y));
}

template <int EPI>
__device__ __forceinline__ void finish(CgState* st, int k, double tot, double m4)
{
    if (st->frozen) return;
    if constexpr (EPI == EPI_NORM) {
        // alpha = rr / <p, A p>, with <p, A p> = 4m^2 |p|^2 + |D_oe p|^2 (D_eo^dag = -D_oe)
        st->tt[k] = tot;
        if (st->active[k]) {
            const double den = m4 * st->pp[k] + tot;
            if (!(den > 0.0) || !finite_d(den)) {
                st->status[k] = HISQ_BREAKDOWN;
                st->active[k] = 0;
                st->alpha[k] = 0.0;
            } else {
                st->alpha[k] = st->rr[k] / den;
            }
        } else {
            st->alpha[k] = 0.0;
        }
    } else if constexpr (EPI == EPI_CG) {
        if (st->active[k]) {
            st->iters[k] += 1;
            if (!finite_d(tot)) {
                st->status[k] = HISQ_BREAKDOWN;
                st->active[k] = 0;
            } else {
                st->beta[k] = tot / st->rr[k];
                st->rr[k] = tot;
                if (tot > st->rrmax[k]) st->rrmax[k] = tot;
                if (tot <= st->thresh[k] || st->iters[k] >= st->maxiter) st->active[k] = 0;
            }
        }
    } else if constexpr (EPI == EPI_RESID) {
        st->rr_true[k] = tot;
    }
}

template <typename T>
__device__ __forceinline__ double norm2c(cplx<T> v)
{
    return (double)v.x * (double)v.x + (double)v.y * (double)v.y;
}

// One tile (one work-group's worth of sites) of a half-Dslash with epilogue
// EPI; `tile` is the tile index, the problem's grid has nblk work-groups and
// this one is number bid (for the reductions).
template <typename T, int NRHS, int NR, int NK, int EPI, bool CM, bool ST = false>
__device__ __forceinline__ void dslash_tile(const DslashArgs<T>& a, int tile, int nblk, int bid,
                                            cplx<T>* lds = nullptr)
{
    using C = cplx<T>;
    constexpr int G = NRHS / NR;
    if constexpr (EPI == EPI_NORM || EPI == EPI_CG) {
        // every rhs of the bundle converged: the iteration is a no-op
        bool any_prob = false;
#pragma unroll
        for (int k = 0; k < NRHS; ++k) any_prob = any_prob || (a.state->active[k] != 0);
        if (!any_prob) return;
    }
    const int g = threadIdx.x % G;
    double part[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) part[k] = 0.0;

    bool act[NR];
    T alpha[NR];
    bool any_act = false;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        act[k] = false;
        alpha[k] = T(0);
        if constexpr (EPI == EPI_CG) {
            act[k] = a.state->active[g * NR + k] != 0;
            alpha[k] = act[k] ? (T)a.state->alpha[g * NR + k] : T(0);
        } else if constexpr (EPI == EPI_RESID) {
            act[k] = a.state->sel[g * NR + k] != 0;
        }
        any_act = any_act || act[k];
    }
    const T m4 = (T)a.mass4;
    T ns = T(1);  // r9: the Naik scale of the links
    if constexpr (NK == HISQ_NAIK_R9) ns = (T)*a.naik_scale;

    const int i = (tile * (int)blockDim.x + (int)threadIdx.x) / G;
    LdsHead<T, NRHS, NR, NK> head;
    if constexpr (ST) {
        // the tile is `rows` whole x-rows: stage them and their +-3 row halo
        static_assert(CM, "staging reads colour-major fields");
        if (i < a.lat.Vh) lds_head<T, NRHS, NR, NK>(a.lat, a.parity, i, g, a.links, a.in, head);
        stage_rows<T, NRHS>(a.in, lds, a.lat, tile * a.rows, a.rows);
        __syncthreads();
    }
    // The epilogue computes everything before its stores, posts the
    // work-group's reduction partials, and only then stores the outputs: the
    // completion wait that orders the partials before the counter update does
    // not wait for the output stores.
    const bool on_site = i < a.lat.Vh;
    using Lay = Layout<NRHS, CM>;
    const int base = Lay::site(on_site ? i : 0) + g * NR;
    C acc[3][NR];
    C xo[3][NR], ro[3][NR];  // EPI_CG: updated x and r
    d2 rr[3][NR];            // EPI_RESID: the FP64 residual
    if (on_site) {
        if constexpr (ST)
            dslash_site_lds<T, NRHS, NR, NK>(a.lat, a.parity, i, g,
                                              ((int)threadIdx.x / G) / a.lat.Lh0, a.links, a.in,
                                              lds, a.rows + 6, head, acc, ns);
        else
            dslash_site<T, NRHS, NR, NK, CM>(a.lat, a.parity, i, g, a.links, a.in, acc, ns);
        pin_acc(acc);
        if constexpr (EPI == EPI_NORM) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int k = 0; k < NR; ++k) part[k] += norm2c<T>(acc[c][k]);
        } else if constexpr (EPI == EPI_CG) {
            if (any_act) {
            // converged (masked) rhs are not written (and not read where the
            // whole tile of the thread is masked); their partial sums stay
            // zero and their finisher ignores them
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                C pv[NR];
                load_rhs<NR, true>(a.p + base + Lay::colour(c, a.lat.Vh), pv);
                load_rhs<NR, true>(a.x + base + Lay::colour(c, a.lat.Vh), xo[c]);
                load_rhs<NR, true>(a.r + base + Lay::colour(c, a.lat.Vh), ro[c]);
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const C q = C{m4 * pv[k].x - acc[c][k].x, m4 * pv[k].y - acc[c][k].y};
                    xo[c][k] = C{xo[c][k].x + alpha[k] * pv[k].x, xo[c][k].y + alpha[k] * pv[k].y};
                    ro[c][k] = C{ro[c][k].x - alpha[k] * q.x, ro[c][k].y - alpha[k] * q.y};
                    if (act[k]) part[k] += norm2c<T>(ro[c][k]);
                }
            }
            }
        } else if constexpr (EPI == EPI_RESID) {
            if (any_act) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d2 bv[NR], xv[NR];
                load_rhs<NR>(a.b + base + Lay::colour(c, a.lat.Vh), bv);
                load_rhs<NR>(a.xh + base + Lay::colour(c, a.lat.Vh), xv);
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    rr[c][k] = d2{bv[k].x - (m4 * xv[k].x - acc[c][k].x),
                                  bv[k].y - (m4 * xv[k].y - acc[c][k].y)};
                    part[k] += norm2c<double>(rr[c][k]);
                }
            }
            }
        }
    }

    bool last = false;
    if constexpr (EPI != EPI_PLAIN) last = grid_reduce_post<NRHS, NR>(part, a.red, a.cnt, nblk, bid);

    if (on_site) {
        if constexpr (EPI == EPI_PLAIN || EPI == EPI_NORM) {
#pragma unroll
            for (int c = 0; c < 3; ++c) store_rhs<NR>(a.out + base + Lay::colour(c, a.lat.Vh), acc[c]);
        } else if constexpr (EPI == EPI_CG) {
            if (any_act) {
                // plain stores: L2 merges the partial lines of consecutive
                // store instructions before they reach HBM
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    store_rhs_on<NR>(a.x + base + Lay::colour(c, a.lat.Vh), xo[c], act);
                    store_rhs_on<NR>(a.r + base + Lay::colour(c, a.lat.Vh), ro[c], act);
                }
            }
        } else if constexpr (EPI == EPI_RESID) {
            if (any_act) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    store_rhs_on<NR>(a.out + base + Lay::colour(c, a.lat.Vh), rr[c], act);
            }
        }
    }

    if constexpr (EPI != EPI_PLAIN) {
        double total;
        if (last && grid_reduce_finish<NRHS>(a.red, a.cnt, nblk, bid, &total)) {
            if (threadIdx.x < NRHS) finish<EPI>(a.state, threadIdx.x, total, a.mass4);
        }
    }
}

#ifdef HISQ_WAVES_PER_EU
#define HISQ_KATTR __attribute__((amdgpu_waves_per_eu(HISQ_WAVES_PER_EU)))
#else
#define HISQ_KATTR
#endif

template <typename T, int NRHS, int NR, int NK, int EPI, bool CM>
__global__ __launch_bounds__(kMaxBlock) HISQ_KATTR void k_dslash(const DslashArgs<T> a)
{
    const int tile_sites = (int)blockDim.x / (NRHS / NR);
    dslash_tile<T, NRHS, NR, NK, EPI, CM>(
        a, tile_of_block(blockIdx.x, gridDim.x, a.remap, a.lat, tile_sites), gridDim.x, blockIdx.x);
}

template <typename T, int NRHS, int NR, int NK, int EPI>
__global__ __launch_bounds__(kMaxBlockLds) void k_dslash_lds(const DslashArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char hisq_stage[];
    const int tile_sites = (int)blockDim.x / (NRHS / NR);
    dslash_tile<T, NRHS, NR, NK, EPI, true, true>(
        a, tile_of_block(blockIdx.x, gridDim.x, a.remap, a.lat, tile_sites), gridDim.x, blockIdx.x,
        reinterpret_cast<cplx<T>*>(hisq_stage));
}

// Batched form: one launch covers the tiles of every problem of a BatchTable;
// each work-group finds its problem (uniform scalar search over <= 16 entries)
// and runs the body specialised for that problem's bundle size and tile.
template <typename T, int NK, int EPI>
__global__ __launch_bounds__(kMaxBlock) void k_dslash_batched(const BatchTable<T>* __restrict__ tab)
{
    int q = 0;
    for (int j = 1; j < tab->nprob; ++j)
        if ((int)blockIdx.x >= tab->p[j].block_start) q = j;
    const BatchProb<T>& bp = tab->p[q];
    const int bid = (int)blockIdx.x - bp.block_start;
    if (bid >= bp.nblocks) return;
    const DslashArgs<T>& a = EPI == EPI_NORM ? bp.k2 : bp.k3;
    const int nb = bp.nblocks;
    // the problem's tile order, on its own block range (the blocks with equal
    // bid mod 8 still share one XCD)
    const int tile = tile_of_block(bid, nb, a.remap, a.lat, (int)blockDim.x / (bp.n / bp.nr));
    switch (bp.n * 16 + bp.nr) {
    case 1 * 16 + 1: dslash_tile<T, 1, 1, NK, EPI, true>(a, tile, nb, bid); break;
    case 2 * 16 + 2: dslash_tile<T, 2, 2, NK, EPI, true>(a, tile, nb, bid); break;
    case 2 * 16 + 1: dslash_tile<T, 2, 1, NK, EPI, true>(a, tile, nb, bid); break;
    case 3 * 16 + 3: dslash_tile<T, 3, 3, NK, EPI, true>(a, tile, nb, bid); break;
    case 4 * 16 + 4: dslash_tile<T, 4, 4, NK, EPI, true>(a, tile, nb, bid); break;
    case 4 * 16 + 2: dslash_tile<T, 4, 2, NK, EPI, true>(a, tile, nb, bid); break;
    case 5 * 16 + 5: dslash_tile<T, 5, 5, NK, EPI, true>(a, tile, nb, bid); break;
    case 6 * 16 + 6: dslash_tile<T, 6, 6, NK, EPI, true>(a, tile, nb, bid); break;
    case 6 * 16 + 3: dslash_tile<T, 6, 3, NK, EPI, true>(a, tile, nb, bid); break;
    case 7 * 16 + 7: dslash_tile<T, 7, 7, NK, EPI, true>(a, tile, nb, bid); break;
    case 8 * 16 + 8: dslash_tile<T, 8, 8, NK, EPI, true>(a, tile, nb, bid); break;
    case 8 * 16 + 4: dslash_tile<T, 8, 4, NK, EPI, true>(a, tile, nb, bid); break;
    default: break;
    }
}

template <typename T, int NK, int EPI, int NRHS, int NR>
static hipError_t go(const Tile& t, DslashArgs<T> a, hipStream_t s, bool cm)
{
    constexpr int G = NRHS / NR;
    const long threads = (long)a.lat.Vh * G;
    a.ntiles = (int)((threads + t.bs - 1) / t.bs);
    a.remap = t.remap;
    a.rows = t.rows;
    // each kernel is built for a maximum work-group size; the grid
    // reductions need whole waves
    if (t.bs < 64 || t.bs % 64 != 0 || t.bs > (t.rows > 0 ? kMaxBlockLds : kMaxBlock))
        return hipErrorInvalidValue;
    if (t.rows > 0) {
        // LDS-staged: colour-major only; the host has checked that a tile is
        // t.rows whole x-rows of one plane and that the rows fit in LDS
        if (!cm) return hipErrorInvalidValue;
        const size_t lds = (size_t)3 * (t.rows + 6) * a.lat.Lh0 * NRHS * sizeof(cplx<T>);
        hipLaunchKernelGGL((k_dslash_lds<T, NRHS, NR, NK, EPI>), dim3(a.ntiles), dim3(t.bs), lds, s, a);
        return hipGetLastError();
    }
    // the solver's kernels exist in colour-major form only; the plain Dslash in both
    if (cm)
        hipLaunchKernelGGL((k_dslash<T, NRHS, NR, NK, EPI, true>), dim3(a.ntiles), dim3(t.bs), 0, s, a);
    else if constexpr (EPI == EPI_PLAIN)
        hipLaunchKernelGGL((k_dslash<T, NRHS, NR, NK, EPI, false>), dim3(a.ntiles), dim3(t.bs), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, int NK, int EPI, int NRHS>
static hipError_t pick_nr(const Tile& t, const DslashArgs<T>& a, hipStream_t s, bool cm)
{
    if (t.nr == NRHS) return go<T, NK, EPI, NRHS, NRHS>(t, a, s, cm);
    if constexpr (NRHS % 2 == 0)
        if (t.nr == NRHS / 2) return go<T, NK, EPI, NRHS, NRHS / 2>(t, a, s, cm);
    if constexpr (NRHS % 4 == 0)
        if (t.nr == NRHS / 4) return go<T, NK, EPI, NRHS, NRHS / 4>(t, a, s, cm);
    if constexpr (NRHS % 8 == 0)
        if (t.nr == NRHS / 8) return go<T, NK, EPI, NRHS, NRHS / 8>(t, a, s, cm);
    return hipErrorInvalidValue;
}

#define HISQ_CAT2(a, b) a##b
#define HISQ_CAT(a, b) HISQ_CAT2(a, b)
#define HISQ_LAUNCH_NAME HISQ_CAT(HISQ_CAT(HISQ_CAT(launch_dslash_p, HISQ_KPREC), _e), HISQ_KEPI)

hipError_t HISQ_LAUNCH_NAME(int nrhs, const Tile& t, const DslashArgs<KT>& a, hipStream_t s, bool cm)
{
    constexpr int EPI = HISQ_KEPI;
    if constexpr (EPI == EPI_RESID && HISQ_KPREC != 0) {
        return hipErrorInvalidValue;
    } else {
        switch (nrhs) {
        case 1: return pick_nr<KT, kNK, EPI, 1>(t, a, s, cm);
        case 2: return pick_nr<KT, kNK, EPI, 2>(t, a, s, cm);
        case 3: return pick_nr<KT, kNK, EPI, 3>(t, a, s, cm);
        case 4: return pick_nr<KT, kNK, EPI, 4>(t, a, s, cm);
        case 5: return pick_nr<KT, kNK, EPI, 5>(t, a, s, cm);
        case 6: return pick_nr<KT, kNK, EPI, 6>(t, a, s, cm);
        case 7: return pick_nr<KT, kNK, EPI, 7>(t, a, s, cm);
        case 8: return pick_nr<KT, kNK, EPI, 8>(t, a, s, cm);
        default: return hipErrorInvalidValue;
        }
    }
}

#if HISQ_KEPI == 1 || HISQ_KEPI == 2
#define HISQ_BNAME HISQ_CAT(HISQ_CAT(HISQ_CAT(launch_dslash_batched_p, HISQ_KPREC), _e), HISQ_KEPI)
hipError_t HISQ_BNAME(const BatchTable<KT>* tab, int total_blocks, int bs, hipStream_t s)
{
    // built for at most kMaxBlock threads, whole waves (the grid reductions)
    if (bs < 64 || bs > kMaxBlock || bs % 64 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_dslash_batched<KT, kNK, HISQ_KEPI>), dim3(total_blocks), dim3(bs), 0, s,
                       tab);
    return hipGetLastError();
}
#endif

}  // namespace hisq
