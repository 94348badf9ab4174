// Device helpers shared by the HIP kernels: tile scheduling and the per-rhs
// FP64 reductions of the CG dot products.
#pragma once

#include "hisq_internal.h"

namespace hisq {

// Work-group -> tile map (a bijection on [0, nb); correctness never depends on
// it, only cache locality does).  Work-groups are dealt to the 8 XCDs of the
// chip round-robin (work-group b starts on XCD b mod 8).
//   order 0: tile = b.
//   order 1: the tiles are split into 8 contiguous ranges and XCD j walks range
//            j in order, so each XCD's L2 sees a contiguous slab of the lattice.
//   order 2: as 1, but the walk visits all Lt time slices of one position of the
//            slice before moving on (t fastest).  An input site is read by the
//            outputs at t+-1 and t+-3; in canonical order those run a whole time
//            slice apart and the site is fetched again for each, in this order
//            they run back to back and hit L2.  Needs nb = Lt * (tiles per slice).
__device__ inline int tile_of_block(int b, int nb, int order, const Lat& lat, int tile_sites)
{
    if (order == 0 || nb < 8) return b;
    const int j = b & 7, m = b >> 3;
    if (order == 3) {
        // XCD j owns the z-chunk [j*zc, (j+1)*zc) of every time slice and walks
        // it with the (y, x) plane position outermost, then t, then z, so the
        // +-1 and +-3 neighbours in every direction but the chunk's z faces
        // are read while they are still in that XCD's L2.
        const int zc = lat.L[2] >> 3, C = lat.L[0] * lat.L[1] / 2 / tile_sites;
        const int zl = m % zc, t = (m / zc) % lat.L[3], c = m / (zc * lat.L[3]);
        return ((t * lat.L[2] + j * zc + zl) * C) + c;
    }
    const int q = nb >> 3, rem = nb & 7;
    const int c = j * q + (j < rem ? j : rem) + m;  // XCD-contiguous position
    if (order == 1) return c;
    const int per_slice = nb / lat.L[3];
    return (c % lat.L[3]) * per_slice + c / lat.L[3];
}

__device__ inline double shfl_xor_d(double v, int m) { return __shfl_xor(v, m, 64); }

constexpr int kRedGroup = 64;  // work-groups per second-stage group

// Coherent accesses for the cross-work-group reduction.  Plain stores stay in
// the L2 of the XCD that wrote them; agent-scope atomic accesses are performed
// at the device-coherent level, so a work-group on another XCD sees them.
// (No release fence is used: on this chip an agent-scope release writes back
// the whole L2, far too costly once per work-group.)
__device__ __forceinline__ void store_coherent(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coherent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coherent(const double* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t add_coherent(uint32_t* p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wave's outstanding memory operations have completed, i.e.
// its coherent stores have been performed, before it signals a counter.
__device__ __forceinline__ void wait_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// The reading side: once a work-group has seen from the counter that it
// arrived last, an agent-scope acquire keeps its loads of the partials after
// that observation (the compiler may not hoist them, and the vector L1 is
// invalidated, so no line cached before the counter update is reused).
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Sum over all 64 lanes by an xor butterfly: every lane ends with the same,
// bitwise identical total (each step adds the same two values).
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += shfl_xor_d(v, off);
    return v;
}

// Per-rhs FP64 sums over the whole grid, in a fixed order (bitwise
// reproducible, no floating-point atomics).  Each thread contributes part[k]
// to rhs g*NR + k, where g = lane mod G is its rhs group.
//   stage 1: wave butterflies + LDS -> one partial per work-group and rhs;
//   stage 2: the last work-group of each group of 64 (atomic counter) sums the
//            group's partials;
//   stage 3: the last group to finish sums the group sums.
// Only wave 0 of a work-group takes part after stage 1.  Returns true in wave 0
// of the one work-group that finished last; lane k < NRHS then holds the total
// of rhs k in *total.  The grid is the nblk work-groups of one problem, this
// one being number bid.  red: [nblk][NRHS] partials then [ngroups][NRHS] group
// sums; cnt: [1 + ngroups] counters, zero on entry and re-armed on exit.
//
// Ordering.  A writer stores its partials with agent-scope atomic stores,
// waits (s_waitcnt vmcnt(0)) until the memory system has acknowledged them --
// an agent-scope atomic store is acknowledged once it is visible at the
// device-coherent level, bypassing the XCD's non-coherent L2 -- and only then
// issues its counter increment.  The last arriving work-group observes the
// final count through the returned value of its own read-modify-write, then
// executes an agent-scope acquire before it loads the partials with
// agent-scope atomic loads.  So every partial was performed at the coherent
// level before the increment that counted it, and every load of the reader
// follows its observation of that count.  The writer side uses no release
// fence: on this chip an agent-scope release writes back the XCD's whole L2,
// which one work-group per launch can afford but every work-group cannot; the
// completion wait orders exactly the stores the reader needs.
// Stage 1 of grid_reduce_rhs: the work-group's partials are posted and its
// group's counter advanced.  Returns true in wave 0 of the work-group that
// arrived last in its group of 64, which must then call grid_reduce_finish.
// A kernel may issue stores that the reduction does not read (its output
// fields) between the two calls, so that the completion wait before the
// counter update covers only the partials.
template <int NRHS, int NR>
__device__ bool grid_reduce_post(double (&part)[NR], double* red, uint32_t* cnt, int nblk, int bid)
{
    constexpr int G = NRHS / NR;
    static_assert(G == 1 || G == 2 || G == 4 || G == 8, "rhs groups must be a power of two");
    __shared__ double sred[kMaxBlockLds / 64][kMaxRhs];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
#pragma unroll
        for (int off = 32; off >= G; off >>= 1) part[k] += shfl_xor_d(part[k], off);
    }
    if (lane < G) {
#pragma unroll
        for (int k = 0; k < NR; ++k) sred[wave][lane * NR + k] = part[k];
    }
    __syncthreads();
    if (wave != 0) return false;
    if (lane < NRHS) {
        double s = 0;
        for (int w = 0; w < nwaves; ++w) s += sred[w][lane];
        store_coherent(&red[(size_t)bid * NRHS + lane], s);
    }
    wait_memory();
    const int grp = bid / kRedGroup;
    const int gn = min(kRedGroup, nblk - grp * kRedGroup);
    uint32_t prev = 0;
    if (lane == 0) prev = add_coherent(&cnt[1 + grp], 1u);
    prev = __shfl(prev, 0, 64);
    return prev == (uint32_t)(gn - 1);
}

// Stages 2 and 3, in wave 0 of a work-group for which grid_reduce_post
// returned true: returns true in the one work-group that finished the grid,
// where lane k < NRHS then holds the total of rhs k in *total.
template <int NRHS>
__device__ bool grid_reduce_finish(double* red, uint32_t* cnt, int nblk, int bid, double* total)
{
    const int lane = threadIdx.x & 63;
    const int ngroups = (nblk + kRedGroup - 1) / kRedGroup;
    double* gsum = red + (size_t)nblk * NRHS;
    const int grp = bid / kRedGroup;
    const int g0 = grp * kRedGroup;
    const int gn = min(kRedGroup, nblk - g0);
    acquire_agent();

    // stage 2: the last work-group of the group
    double acc[NRHS];
    const double* row = &red[(size_t)(g0 + (lane < gn ? lane : 0)) * NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) acc[k] = load_coherent(row + k);  // all loads in flight
    double mine = 0;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        acc[k] = wave_sum(lane < gn ? acc[k] : 0.0);
        if (lane == k) mine = acc[k];
    }
    if (lane < NRHS) store_coherent(&gsum[(size_t)grp * NRHS + lane], mine);
    if (lane == 0) store_coherent(&cnt[1 + grp], 0u);
    wait_memory();
    uint32_t prev = 0;
    if (lane == 0) prev = add_coherent(&cnt[0], 1u);
    prev = __shfl(prev, 0, 64);
    if (prev != (uint32_t)(ngroups - 1)) return false;
    acquire_agent();

    // stage 3: the last group
#pragma unroll
    for (int k = 0; k < NRHS; ++k) acc[k] = 0.0;
    for (int j = lane; j < ngroups; j += 64) {
        double v[NRHS];
#pragma unroll
        for (int k = 0; k < NRHS; ++k) v[k] = load_coherent(&gsum[(size_t)j * NRHS + k]);
#pragma unroll
        for (int k = 0; k < NRHS; ++k) acc[k] += v[k];
    }
    mine = 0;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        acc[k] = wave_sum(acc[k]);
        if (lane == k) mine = acc[k];
    }
    if (lane == 0) store_coherent(&cnt[0], 0u);
    *total = mine;
    return true;
}

template <int NRHS, int NR>
__device__ bool grid_reduce_rhs(double (&part)[NR], double* red, uint32_t* cnt, int nblk, int bid,
                                double* total)
{
    if (!grid_reduce_post<NRHS, NR>(part, red, cnt, nblk, bid)) return false;
    return grid_reduce_finish<NRHS>(red, cnt, nblk, bid, total);
}

__device__ inline bool finite_d(double v) { return v - v == 0.0; }

// Spinor field layouts, element (site i, colour c, rhs k) of an n-rhs field:
//   site-major   [Vh][3][n]  (CM = false, the canonical layout at the boundary)
//   colour-major [3][Vh][n]  (CM = true, the solver's internal layout)
// Both keep the rhs of a site innermost.  In colour-major order the lanes of a
// wave, which own consecutive sites, read one contiguous stretch per colour;
// in site-major order they stride by 3n complex numbers, and every load
// instruction touches about three times as many cache lines.
template <int NRHS, bool CM>
struct Layout {
    __device__ static __forceinline__ int site(int i) { return CM ? i * NRHS : i * 3 * NRHS; }
    __device__ static __forceinline__ int colour(int c, int Vh) { return CM ? c * Vh * NRHS : c * NRHS; }
};

// Loads and stores of NR consecutive complex numbers (rhs of one colour).
// NT: streamed data, read or written once per launch; the non-temporal hint
// keeps it from evicting the gathered neighbour field from L2.
template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int NR, bool NT = false>
__device__ __forceinline__ void load_rhs(const f2* __restrict__ p, f2 (&v)[NR])
{
    if constexpr (NR % 2 == 0) {
        const f4* q = reinterpret_cast<const f4*>(p);
#pragma unroll
        for (int k = 0; k < NR / 2; ++k) {
            f4 w = ld<NT>(q + k);
            v[2 * k] = f2{w.x, w.y};
            v[2 * k + 1] = f2{w.z, w.w};
        }
    } else {
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] = ld<NT>(p + k);
    }
}

template <int NR, bool NT = false>
__device__ __forceinline__ void load_rhs(const d2* __restrict__ p, d2 (&v)[NR])
{
#pragma unroll
    for (int k = 0; k < NR; ++k) v[k] = ld<NT>(p + k);
}

template <int NR, bool NT = false>
__device__ __forceinline__ void store_rhs(f2* __restrict__ p, const f2 (&v)[NR])
{
    if constexpr (NR % 2 == 0) {
        f4* q = reinterpret_cast<f4*>(p);
#pragma unroll
        for (int k = 0; k < NR / 2; ++k)
            st<NT>(q + k, f4{v[2 * k].x, v[2 * k].y, v[2 * k + 1].x, v[2 * k + 1].y});
    } else {
#pragma unroll
        for (int k = 0; k < NR; ++k) st<NT>(p + k, v[k]);
    }
}

template <int NR, bool NT = false>
__device__ __forceinline__ void store_rhs(d2* __restrict__ p, const d2 (&v)[NR])
{
#pragma unroll
    for (int k = 0; k < NR; ++k) st<NT>(p + k, v[k]);
}

// Masked stores for the CG updates: rhs k is written only if on[k] (converged
// rhs keep their values untouched in memory); a 16-byte FP32 pair with one rhs
// on stores that rhs alone.
template <int NR>
__device__ __forceinline__ void store_rhs_on(f2* __restrict__ p, const f2 (&v)[NR], const bool (&on)[NR])
{
    if constexpr (NR % 2 == 0) {
        f4* q = reinterpret_cast<f4*>(p);
#pragma unroll
        for (int k = 0; k < NR / 2; ++k) {
            if (on[2 * k] && on[2 * k + 1])
                q[k] = f4{v[2 * k].x, v[2 * k].y, v[2 * k + 1].x, v[2 * k + 1].y};
            else if (on[2 * k])
                p[2 * k] = v[2 * k];
            else if (on[2 * k + 1])
                p[2 * k + 1] = v[2 * k + 1];
        }
    } else {
#pragma unroll
        for (int k = 0; k < NR; ++k)
            if (on[k]) p[k] = v[k];
    }
}

template <int NR>
__device__ __forceinline__ void store_rhs_on(d2* __restrict__ p, const d2 (&v)[NR], const bool (&on)[NR])
{
#pragma unroll
    for (int k = 0; k < NR; ++k)
        if (on[k]) p[k] = v[k];
}

}  // namespace hisq
