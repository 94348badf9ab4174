// Stencil helpers shared by the Dslash kernels: complex arithmetic in the
// storage precision, lattice coordinates and neighbour indices of the 16 slots
// of the HISQ stencil (Sec. 1 eq. (3)), and loads of packed link matrices.
#pragma once

#include <type_traits>

#include "hisq_device.h"

namespace hisq {

template <typename C>
__device__ __forceinline__ C cmul(C a, C b)
{
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename C>
__device__ __forceinline__ C cconj(C a)
{
    return C{a.x, -a.y};
}

// Fused multiply-add in the storage precision (the plain __builtin_fma is the
// double-precision builtin and would promote FP32 operands).
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc += m * v in four fused multiply-adds
template <typename C>
__device__ __forceinline__ void cfma(C& acc, C m, C v)
{
    acc.x = fmadd(m.x, v.x, acc.x);
    acc.x = fmadd(-m.y, v.y, acc.x);
    acc.y = fmadd(m.x, v.y, acc.y);
    acc.y = fmadd(m.y, v.x, acc.y);
}

__device__ __forceinline__ int wrap_delta(int c, int h, int L)
{
    const int cp = c + h;
    return h + (cp < 0 ? L : 0) - (cp >= L ? L : 0);
}

template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Link matrix of slot S for site i, non-temporal (no reuse within a
// half-Dslash).  m[e] holds element e of the 3x3 matrix, row-major; for a
// compressed Naik slot (NK = R14, R13) m[0..5] hold rows 0 and 1 and m[6] the
// stored coefficient (r14: c; r13: its phase in m[6].x).  FP32 reads 16-byte
// words of four reals, then the remaining 1 or 2 reals: the same bytes in
// fewer, wider requests than one 8-byte read per element.
template <typename T, int NK, int S>
__device__ __forceinline__ void load_link(const cplx<T>* __restrict__ lk, int Vh, int i,
                                          cplx<T> (&m)[9])
{
    const T* base = reinterpret_cast<const T*>(lk) + (size_t)slot_real_start(S, NK) * Vh;
    if constexpr (sizeof(T) == 4) {
        constexpr int nr = slot_reals(S, NK);
        constexpr int nw = nr / 4, rem = nr % 4;
        const f4* wp = reinterpret_cast<const f4*>(base) + i;
#pragma unroll
        for (int w = 0; w < nw; ++w) {
            const f4 q = __builtin_nontemporal_load(wp + (size_t)w * Vh);
            m[2 * w] = cplx<T>{q.x, q.y};
            m[2 * w + 1] = cplx<T>{q.z, q.w};
        }
        const T* tail = base + (size_t)4 * nw * Vh;
        if constexpr (rem == 2) {
            m[2 * nw] = __builtin_nontemporal_load(reinterpret_cast<const cplx<T>*>(tail) + i);
        } else if constexpr (rem == 1) {
            m[2 * nw] = cplx<T>{__builtin_nontemporal_load(tail + i), T(0)};
        }
    } else {
        static_assert(NK == HISQ_NAIK_FULL, "FP64 links are stored in full");
        const cplx<T>* lp = reinterpret_cast<const cplx<T>*>(base) + i;
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = __builtin_nontemporal_load(lp + (size_t)e * Vh);
    }
}

// A link matrix shared by the G adjacent lanes that compute the rhs tiles of
// one site (G = 1, 2, 4).  Loading the whole matrix in every lane would move
// each 16-byte word G times through the vector memory pipeline; instead the
// slot's nw = nr / 4 words are dealt round-robin to the lanes of the group
// (word w to lane w mod G), each lane loads only its own, and when the slot is
// used every lane gathers all words with DPP permutes inside its quad (a VALU
// operation, no memory traffic).  The nr mod 4 trailing reals are one small
// load per lane.  FP64 links keep one lane per load (their kernels run G <= 2
// and use every register for the doubles).
template <typename T, int G>
struct LinkRaw {
    static constexpr int kW = (4 + G - 1) / G;  // words per lane (<= 4 per slot)
    f4 w[kW];
    f2 t;
};
template <int G>
struct LinkRaw<double, G> {
    d2 m[9];
};

// Value of v held by lane SRC of this lane's group of G (quad permute:
// G = 4, lanes 4k..4k+3; G = 2, lanes 2k, 2k+1).  Every lane of the group must
// be active.
template <int G, int SRC>
__device__ __forceinline__ float group_bcast(float v)
{
    static_assert(G == 2 || G == 4, "groups of 2 or 4 lanes");
    constexpr int ctrl = G == 4 ? SRC * 0x55 : (SRC | SRC << 2 | (2 + SRC) << 4 | (2 + SRC) << 6);
    return __builtin_bit_cast(
        float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), ctrl, 0xF, 0xF, false));
}

template <int G, int SRC>
__device__ __forceinline__ f4 group_bcast4(f4 v)
{
    if constexpr (G == 1) {
        return v;
    } else {
        return f4{group_bcast<G, SRC>(v.x), group_bcast<G, SRC>(v.y), group_bcast<G, SRC>(v.z),
                  group_bcast<G, SRC>(v.w)};
    }
}

// Issue this lane's share of the loads of slot S (lane g of its group).
template <typename T, int NK, int S, int G>
__device__ __forceinline__ void load_link_part(const cplx<T>* __restrict__ lk, int Vh, int i, int g,
                                               LinkRaw<T, G>& r)
{
    if constexpr (sizeof(T) == 8) {
        load_link<T, NK, S>(lk, Vh, i, r.m);
    } else {
        const T* base = reinterpret_cast<const T*>(lk) + (size_t)slot_real_start(S, NK) * Vh;
        constexpr int nr = slot_reals(S, NK);
        constexpr int nw = nr / 4, rem = nr % 4;
        const f4* wp = reinterpret_cast<const f4*>(base) + i;
#pragma unroll
        for (int j = 0; j < LinkRaw<T, G>::kW; ++j) {
            if (j * G < nw) {
                // a lane left without a word of this round loads the last one
                // again (no divergent branch in the pipeline; same cache line)
                const int w = min((G == 1 ? 0 : g) + j * G, nw - 1);
                r.w[j] = __builtin_nontemporal_load(wp + (size_t)w * Vh);
            }
        }
        const T* tail = base + (size_t)4 * nw * Vh;
        if constexpr (rem == 2) {
            r.t = __builtin_nontemporal_load(reinterpret_cast<const f2*>(tail) + i);
        } else if constexpr (rem == 1) {
            r.t = f2{__builtin_nontemporal_load(tail + i), 0.f};
        }
    }
}

// The whole matrix of slot S from the group's shares: m[e] element e (row-major);
// for compressed Naik slots m[0..5] rows 0 and 1 and m[6] the stored coefficient.
template <typename T, int NK, int S, int G>
__device__ __forceinline__ void share_link(const LinkRaw<T, G>& r, cplx<T> (&m)[9])
{
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int e = 0; e < 9; ++e) m[e] = r.m[e];
    } else {
        constexpr int nr = slot_reals(S, NK);
        constexpr int nw = nr / 4, rem = nr % 4;
        static_for<0, nw>([&](auto W) {
            constexpr int w = decltype(W)::value;
            const f4 q = group_bcast4<G, w % G>(r.w[w / G]);
            m[2 * w] = cplx<T>{q.x, q.y};
            m[2 * w + 1] = cplx<T>{q.z, q.w};
        });
        if constexpr (rem > 0) m[2 * nw] = r.t;
    }
}

// Site coordinates and the neighbour index of slot S = 4*hop + mu, hop
// (+1, -1, +3, -3), in the other parity's index space.
struct SiteCoord {
    int i, row, x, c[4];
};

__device__ __forceinline__ SiteCoord site_coord(const Lat& lat, int P, int i)
{
    SiteCoord sc;
    int r = i / lat.Lh0;
    const int xh = i - r * lat.Lh0;
    sc.c[1] = r % lat.L[1];
    r /= lat.L[1];
    sc.c[2] = r % lat.L[2];
    sc.c[3] = r / lat.L[2];
    sc.x = 2 * xh + ((P + sc.c[1] + sc.c[2] + sc.c[3]) & 1);
    sc.c[0] = sc.x;
    sc.row = i - xh;
    sc.i = i;
    return sc;
}

template <int S>
__device__ __forceinline__ int neighbour(const Lat& lat, const SiteCoord& sc)
{
    constexpr int mu = S & 3;
    constexpr int hh = S >> 2;
    constexpr int h = hh == 0 ? 1 : hh == 1 ? -1 : hh == 2 ? 3 : -3;
    if constexpr (mu == 0) {
        const int xp = sc.x + wrap_delta(sc.x, h, lat.L[0]);
        return sc.row + (xp >> 1);
    } else {
        const int stride = mu == 1 ? lat.sy : mu == 2 ? lat.sz : lat.st;
        return sc.i + wrap_delta(sc.c[mu], h, lat.L[mu]) * stride;
    }
}

}  // namespace hisq
