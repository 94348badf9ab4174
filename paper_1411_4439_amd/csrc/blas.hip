// CG vector kernels for gfx950: the masked p-update with its fused |p|^2,
// precision conversions for the reliable updates, and FP64 reductions.
#include "hisq_device.h"

namespace hisq {

// ---------------------------------------------------------------------------
// p = r + beta_k p for every active rhs k; |p_k|^2 summed in FP64 -> pp[k].
// (site-tiled form, colour-major fields: bundles the streaming form does not cover)
template <typename T, int NRHS, int NR>
__device__ __forceinline__ void pupdate_tile(const PupdateArgs<T>& a, int tile, int nblk, int bid)
{
    using C = cplx<T>;
    constexpr int G = NRHS / NR;
    const int g = threadIdx.x % G;
    bool any_prob = false;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) any_prob = any_prob || (a.state->active[k] != 0);
    if (!any_prob) return;  // every rhs converged: nothing to do, nothing to reduce

    bool act[NR];
    T beta[NR];
    bool any_act = false;
    double part[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        act[k] = a.state->active[g * NR + k] != 0;
        beta[k] = (T)a.state->beta[g * NR + k];
        any_act = any_act || act[k];
        part[k] = 0.0;
    }
    const int i = (tile * (int)blockDim.x + (int)threadIdx.x) / G;
    const bool work = i < a.lat.Vh && any_act;
    using Lay = Layout<NRHS, true>;
    const int base = Lay::site(work ? i : 0) + g * NR;
    C pv[3][NR];
    if (work) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int off = base + Lay::colour(c, a.lat.Vh);
            C rv[NR];
            load_rhs<NR>(a.r + off, rv);
            load_rhs<NR>(a.p + off, pv[c]);
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                // beta = 0 starts (or restarts) the recursion: p = r exactly, even
                // if p held non-finite values
                pv[c][k] = beta[k] == T(0) ? rv[k]
                                           : C{rv[k].x + beta[k] * pv[c][k].x, rv[k].y + beta[k] * pv[c][k].y};
                if (act[k]) part[k] += (double)pv[c][k].x * pv[c][k].x + (double)pv[c][k].y * pv[c][k].y;
            }
        }
    }
    // partials first, then the stores (converged rhs are not written)
    const bool last = grid_reduce_post<NRHS, NR>(part, a.red, a.cnt, nblk, bid);
    if (work) {
#pragma unroll
        for (int c = 0; c < 3; ++c) store_rhs_on<NR>(a.p + base + Lay::colour(c, a.lat.Vh), pv[c], act);
    }
    double total;
    if (last && grid_reduce_finish<NRHS>(a.red, a.cnt, nblk, bid, &total)) {
        if (threadIdx.x < NRHS && !a.state->frozen) a.state->pp[threadIdx.x] = total;
    }
}

template <typename T, int NRHS, int NR>
__global__ __launch_bounds__(kMaxBlock) void k_pupdate(const PupdateArgs<T> a)
{
    pupdate_tile<T, NRHS, NR>(a, tile_of_block(blockIdx.x, gridDim.x, a.remap, a.lat, (int)blockDim.x / (NRHS / NR)), gridDim.x,
                              blockIdx.x);
}

template <typename T>
__global__ __launch_bounds__(kMaxBlock) void k_pupdate_batched(const BatchTable<T>* __restrict__ tab)
{
    int q = 0;
    for (int j = 1; j < tab->nprob; ++j)
        if ((int)blockIdx.x >= tab->p[j].block_start) q = j;
    const BatchProb<T>& bp = tab->p[q];
    const int bid = (int)blockIdx.x - bp.block_start;
    if (bid >= bp.nblocks) return;
    const int nb = bp.nblocks;
    const int tile = tile_of_block(bid, nb, bp.k1.remap, bp.k1.lat, (int)blockDim.x / (bp.n / bp.nr));
    switch (bp.n * 16 + bp.nr) {
    case 1 * 16 + 1: pupdate_tile<T, 1, 1>(bp.k1, tile, nb, bid); break;
    case 2 * 16 + 2: pupdate_tile<T, 2, 2>(bp.k1, tile, nb, bid); break;
    case 2 * 16 + 1: pupdate_tile<T, 2, 1>(bp.k1, tile, nb, bid); break;
    case 3 * 16 + 3: pupdate_tile<T, 3, 3>(bp.k1, tile, nb, bid); break;
    case 4 * 16 + 4: pupdate_tile<T, 4, 4>(bp.k1, tile, nb, bid); break;
    case 4 * 16 + 2: pupdate_tile<T, 4, 2>(bp.k1, tile, nb, bid); break;
    case 5 * 16 + 5: pupdate_tile<T, 5, 5>(bp.k1, tile, nb, bid); break;
    case 6 * 16 + 6: pupdate_tile<T, 6, 6>(bp.k1, tile, nb, bid); break;
    case 6 * 16 + 3: pupdate_tile<T, 6, 3>(bp.k1, tile, nb, bid); break;
    case 7 * 16 + 7: pupdate_tile<T, 7, 7>(bp.k1, tile, nb, bid); break;
    case 8 * 16 + 8: pupdate_tile<T, 8, 8>(bp.k1, tile, nb, bid); break;
    case 8 * 16 + 4: pupdate_tile<T, 8, 4>(bp.k1, tile, nb, bid); break;
    default: break;
    }
}

// Streaming form of the p-update for bundles of 1, 2, 4 or 8 rhs: the field is
// walked as a flat array of NRT-complex chunks with a stride that is a
// multiple of the rhs period, so every thread always touches the same NRT rhs
// (and the lanes of a wave with equal lane mod (NRHS/NRT) the same ones) while
// each load instruction covers a contiguous stretch of memory.
template <typename T, int NRHS, int NRT>
__global__ __launch_bounds__(kMaxBlock) void k_pupdate_flat(const PupdateArgs<T> a, long nchunks)
{
    using C = cplx<T>;
    constexpr int G = NRHS / NRT;
    bool any_prob = false;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) any_prob = any_prob || (a.state->active[k] != 0);
    if (!any_prob) return;
    const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;  // a multiple of 64, hence of G
    const int g = (int)(tid % G);
    bool act[NRT];
    T beta[NRT];
    double part[NRT];
    bool any_act = false;
#pragma unroll
    for (int k = 0; k < NRT; ++k) {
        act[k] = a.state->active[g * NRT + k] != 0;
        beta[k] = (T)a.state->beta[g * NRT + k];
        any_act = any_act || act[k];
        part[k] = 0.0;
    }
    if (any_act) {
        for (long j = tid; j < nchunks; j += stride) {
            C rv[NRT], pv[NRT];
            load_rhs<NRT>(a.r + j * NRT, rv);
            load_rhs<NRT>(a.p + j * NRT, pv);
#pragma unroll
            for (int k = 0; k < NRT; ++k) {
                pv[k] = beta[k] == T(0) ? rv[k]
                                        : C{rv[k].x + beta[k] * pv[k].x, rv[k].y + beta[k] * pv[k].y};
                if (act[k]) part[k] += (double)pv[k].x * pv[k].x + (double)pv[k].y * pv[k].y;
            }
            store_rhs_on<NRT>(a.p + j * NRT, pv, act);
        }
    }
    double total;
    if (grid_reduce_rhs<NRHS, NRT>(part, a.red, a.cnt, gridDim.x, blockIdx.x, &total)) {
        if (threadIdx.x < NRHS && !a.state->frozen) a.state->pp[threadIdx.x] = total;
    }
}

constexpr int kFlatMaxBlocks = 2048;

template <typename T, int NRHS, int NRT>
static hipError_t go_flat(PupdateArgs<T> a, hipStream_t s)
{
    const long nchunks = (long)a.lat.Vh * 3 * NRHS / NRT;
    const int bs = 256;
    long blocks = (nchunks + bs - 1) / bs;
    if (blocks > kFlatMaxBlocks) blocks = kFlatMaxBlocks;
    hipLaunchKernelGGL((k_pupdate_flat<T, NRHS, NRT>), dim3((int)blocks), dim3(bs), 0, s, a, nchunks);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_flat(int nrhs, const PupdateArgs<T>& a, hipStream_t s)
{
    switch (nrhs) {
    case 1: return go_flat<T, 1, 1>(a, s);
    case 2: return go_flat<T, 2, 2>(a, s);
    case 4: return go_flat<T, 4, 2>(a, s);
    case 8: return go_flat<T, 8, 2>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pupdate_flat_f64(int nrhs, const PupdateArgs<double>& a, hipStream_t s)
{
    return launch_flat<double>(nrhs, a, s);
}

hipError_t launch_pupdate_flat_f32(int nrhs, const PupdateArgs<float>& a, hipStream_t s)
{
    return launch_flat<float>(nrhs, a, s);
}

hipError_t launch_pupdate_batched_f64(const BatchTable<double>* tab, int total_blocks, int bs,
                                      hipStream_t s)
{
    if (bs < 64 || bs > kMaxBlock || bs % 64 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pupdate_batched<double>, dim3(total_blocks), dim3(bs), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_pupdate_batched_f32(const BatchTable<float>* tab, int total_blocks, int bs,
                                      hipStream_t s)
{
    if (bs < 64 || bs > kMaxBlock || bs % 64 != 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pupdate_batched<float>, dim3(total_blocks), dim3(bs), 0, s, tab);
    return hipGetLastError();
}

template <typename T, int NRHS, int NR>
static hipError_t go_pup(const Tile& t, PupdateArgs<T> a, hipStream_t s)
{
    constexpr int G = NRHS / NR;
    if (t.bs < 64 || t.bs > kMaxBlock || t.bs % 64 != 0) return hipErrorInvalidValue;
    const long threads = (long)a.lat.Vh * G;
    a.ntiles = (int)((threads + t.bs - 1) / t.bs);
    a.remap = t.remap;
    hipLaunchKernelGGL((k_pupdate<T, NRHS, NR>), dim3(a.ntiles), dim3(t.bs), 0, s, a);
    return hipGetLastError();
}

template <typename T, int NRHS>
static hipError_t pick_pup(const Tile& t, const PupdateArgs<T>& a, hipStream_t s)
{
    if (t.nr == NRHS) return go_pup<T, NRHS, NRHS>(t, a, s);
    if constexpr (NRHS % 2 == 0)
        if (t.nr == NRHS / 2) return go_pup<T, NRHS, NRHS / 2>(t, a, s);
    if constexpr (NRHS % 4 == 0)
        if (t.nr == NRHS / 4) return go_pup<T, NRHS, NRHS / 4>(t, a, s);
    if constexpr (NRHS % 8 == 0)
        if (t.nr == NRHS / 8) return go_pup<T, NRHS, NRHS / 8>(t, a, s);
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t launch_pupdate(int nrhs, const Tile& t, const PupdateArgs<T>& a, hipStream_t s)
{
    switch (nrhs) {
    case 1: return pick_pup<T, 1>(t, a, s);
    case 2: return pick_pup<T, 2>(t, a, s);
    case 3: return pick_pup<T, 3>(t, a, s);
    case 4: return pick_pup<T, 4>(t, a, s);
    case 5: return pick_pup<T, 5>(t, a, s);
    case 6: return pick_pup<T, 6>(t, a, s);
    case 7: return pick_pup<T, 7>(t, a, s);
    case 8: return pick_pup<T, 8>(t, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_pupdate_f64(int nrhs, const Tile& t, const PupdateArgs<double>& a, hipStream_t s)
{
    return launch_pupdate<double>(nrhs, t, a, s);
}

hipError_t launch_pupdate_f32(int nrhs, const Tile& t, const PupdateArgs<float>& a, hipStream_t s)
{
    return launch_pupdate<float>(nrhs, t, a, s);
}

// ---------------------------------------------------------------------------
// Elementwise kernels over complex arrays [Vh][3][n] (rhs index = element mod n).

static inline int blocks_for(size_t n, int bs)
{
    size_t b = (n + bs - 1) / bs;
    return (int)(b > 65535u * 16u ? 65535u * 16u : b);
}

__global__ void k_zero(uint32_t* p, size_t words)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < words;
         e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const size_t words = bytes / 4;  // every workspace region is 256-byte aligned
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words, 256)), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

__global__ void k_state_reset(CgState* st, int nrhs, int active)
{
    if (threadIdx.x == 0) {
        *st = CgState{};
        for (int k = 0; k < nrhs; ++k) {
            st->sel[k] = 1;
            st->active[k] = active;
        }
        st->frozen = active;  // armed for timing: the kernels run, the state stays put
    }
}

hipError_t launch_state_reset(CgState* st, int nrhs, int active, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(64), 0, s, st, nrhs, active);
    return hipGetLastError();
}

__global__ void k_to_f32_sel(const d2* __restrict__ src, f2* __restrict__ dst, size_t ncplx,
                             int nrhs, const CgState* st)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ncplx;
         e += (size_t)gridDim.x * blockDim.x) {
        if (st->sel[e % nrhs]) {
            const d2 v = src[e];
            dst[e] = f2{(float)v.x, (float)v.y};
        }
    }
}

hipError_t launch_to_f32_sel(const d2* src, f2* dst, size_t ncplx, int nrhs, const CgState* st,
                             hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32_sel, dim3(blocks_for(ncplx, 256)), dim3(256), 0, s, src, dst, ncplx,
                       nrhs, st);
    return hipGetLastError();
}

// x_hi += x_lo; x_lo = 0 for the selected rhs (solution accumulation of a
// reliable update).
__global__ void k_accum_sel(d2* __restrict__ xh, f2* __restrict__ xl, size_t ncplx, int nrhs,
                            const CgState* st)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ncplx;
         e += (size_t)gridDim.x * blockDim.x) {
        if (st->sel[e % nrhs]) {
            const f2 l = xl[e];
            d2 h = xh[e];
            h.x += (double)l.x;
            h.y += (double)l.y;
            xh[e] = h;
            xl[e] = f2{0.0f, 0.0f};
        }
    }
}

hipError_t launch_accum_sel(d2* xh, f2* xl, size_t ncplx, int nrhs, const CgState* st,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_accum_sel, dim3(blocks_for(ncplx, 256)), dim3(256), 0, s, xh, xl, ncplx,
                       nrhs, st);
    return hipGetLastError();
}

__global__ void k_copy_f64(const d2* __restrict__ src, d2* __restrict__ dst, size_t ncplx)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ncplx;
         e += (size_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

hipError_t launch_copy_f64(const d2* src, d2* dst, size_t ncplx, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_f64, dim3(blocks_for(ncplx, 256)), dim3(256), 0, s, src, dst, ncplx);
    return hipGetLastError();
}

__global__ void k_zero_sel(d2* __restrict__ v, size_t ncplx, int nrhs, const CgState* st)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < ncplx;
         e += (size_t)gridDim.x * blockDim.x)
        if (st->sel[e % nrhs]) v[e] = d2{0.0, 0.0};
}

hipError_t launch_zero_sel(d2* v, size_t ncplx, int nrhs, const CgState* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_sel, dim3(blocks_for(ncplx, 256)), dim3(256), 0, s, v, ncplx, nrhs, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Layout conversions between the canonical site-major field [Vh][3][n] and the
// solver's colour-major field [3][Vh][n] (FP64).
__global__ void k_to_colour_major(const d2* __restrict__ src, d2* __restrict__ dst, int Vh, int nrhs)
{
    const size_t total = (size_t)Vh * 3 * nrhs;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t k = e % nrhs, rest = e / nrhs;  // dst index = (c * Vh + i) * n + k
        const size_t i = rest % Vh, c = rest / Vh;
        dst[e] = src[(i * 3 + c) * nrhs + k];
    }
}

__global__ void k_to_site_major(const d2* __restrict__ src, d2* __restrict__ dst, int Vh, int nrhs)
{
    const size_t total = (size_t)Vh * 3 * nrhs;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t k = e % nrhs, rest = e / nrhs;  // dst index = (i * 3 + c) * n + k
        const size_t c = rest % 3, i = rest / 3;
        dst[e] = src[(c * Vh + i) * nrhs + k];
    }
}

hipError_t launch_layout(const d2* src, d2* dst, int Vh, int nrhs, bool to_colour_major, hipStream_t s)
{
    const size_t total = (size_t)Vh * 3 * nrhs;
    if (to_colour_major)
        hipLaunchKernelGGL(k_to_colour_major, dim3(blocks_for(total, 256)), dim3(256), 0, s, src, dst, Vh, nrhs);
    else
        hipLaunchKernelGGL(k_to_site_major, dim3(blocks_for(total, 256)), dim3(256), 0, s, src, dst, Vh, nrhs);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-rhs |v_k|^2 of an FP64 colour-major half field, one thread per site.
template <int NRHS>
__global__ __launch_bounds__(kMaxBlock) void k_norm2(const d2* __restrict__ v, int Vh, double* out,
                                                     double* red, uint32_t* cnt)
{
    double part[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) part[k] = 0.0;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Vh) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                const d2 e = v[((size_t)c * Vh + i) * NRHS + k];
                part[k] += e.x * e.x + e.y * e.y;
            }
    }
    double total;
    if (grid_reduce_rhs<NRHS, NRHS>(part, red, cnt, gridDim.x, blockIdx.x, &total)) {
        if (threadIdx.x < NRHS) out[threadIdx.x] = total;
    }
}

hipError_t launch_norm2_f64(const d2* v, int Vh, int nrhs, double* out, double* red,
                            uint32_t* cnt, hipStream_t s)
{
    const int bs = 256, grid = (Vh + bs - 1) / bs;
    switch (nrhs) {
#define HISQ_NORM_CASE(N)                                                                   \
    case N:                                                                                 \
        hipLaunchKernelGGL(k_norm2<N>, dim3(grid), dim3(bs), 0, s, v, Vh, out, red, cnt); \
        break;
        HISQ_NORM_CASE(1)
        HISQ_NORM_CASE(2)
        HISQ_NORM_CASE(3)
        HISQ_NORM_CASE(4)
        HISQ_NORM_CASE(5)
        HISQ_NORM_CASE(6)
        HISQ_NORM_CASE(7)
        HISQ_NORM_CASE(8)
#undef HISQ_NORM_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// out = scale * sum over sites, colours and rhs of Re(conj(y) x).
__global__ __launch_bounds__(kMaxBlock) void k_redot(const d2* __restrict__ y,
                                                     const d2* __restrict__ x, int Vh, int nrhs,
                                                     double scale, double* out, double* red,
                                                     uint32_t* cnt)
{
    double part[1] = {0.0};
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Vh) {
        for (int e = 0; e < 3 * nrhs; ++e) {
            const d2 a = y[(size_t)i * 3 * nrhs + e];
            const d2 b = x[(size_t)i * 3 * nrhs + e];
            part[0] += a.x * b.x + a.y * b.y;
        }
    }
    double total;
    if (grid_reduce_rhs<1, 1>(part, red, cnt, gridDim.x, blockIdx.x, &total)) {
        if (threadIdx.x == 0) *out = scale * total;
    }
}

hipError_t launch_redot(const d2* y, const d2* x, int Vh, int nrhs, double scale, double* out,
                        double* red, uint32_t* cnt, hipStream_t s)
{
    const int bs = 256, grid = (Vh + bs - 1) / bs;
    hipLaunchKernelGGL(k_redot, dim3(grid), dim3(bs), 0, s, y, x, Vh, nrhs, scale, out, red, cnt);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out = alpha a + beta b over n complex numbers (real scalars).
__global__ void k_axpby(const d2* __restrict__ a, const d2* __restrict__ b, d2* __restrict__ out,
                        size_t n, double alpha, double beta)
{
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const d2 x = a[e], y = b[e];
        out[e] = d2{alpha * x.x + beta * y.x, alpha * x.y + beta * y.y};
    }
}

hipError_t launch_axpby(const d2* a, const d2* b, d2* out, size_t n, double alpha, double beta,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, b, out, n, alpha, beta);
    return hipGetLastError();
}

// Per-rhs complex dot products sum_i conj(a_i) b_i over an even and an odd half
// field (site-major, n rhs), in a fixed order: stage 1 writes one partial per
// work-group and rhs (re, im), stage 2 sums the partials in work-group order.
template <int NRHS>
__global__ __launch_bounds__(256) void k_cdot_partial(const d2* __restrict__ ae, const d2* __restrict__ be,
                                                      const d2* __restrict__ ao, const d2* __restrict__ bo,
                                                      int Vh, double* __restrict__ part)
{
    __shared__ double sh[4][2 * NRHS];
    double re[NRHS], im[NRHS];
#pragma unroll
    for (int k = 0; k < NRHS; ++k) re[k] = im[k] = 0.0;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < 2 * Vh) {
        const bool even = j < Vh;
        const size_t i = even ? j : j - Vh;
        const d2* a = even ? ae : ao;
        const d2* b = even ? be : bo;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < NRHS; ++k) {
                const d2 x = a[(i * 3 + c) * NRHS + k], y = b[(i * 3 + c) * NRHS + k];
                re[k] += x.x * y.x + x.y * y.y;
                im[k] += x.x * y.y - x.y * y.x;
            }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NRHS; ++k) {
        re[k] = wave_sum(re[k]);
        im[k] = wave_sum(im[k]);
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NRHS; ++k) {
            sh[wave][2 * k] = re[k];
            sh[wave][2 * k + 1] = im[k];
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * NRHS) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w][threadIdx.x];
        part[(size_t)blockIdx.x * 2 * NRHS + threadIdx.x] = t;
    }
}

__global__ void k_cdot_final(const double* __restrict__ part, int nblk, int m2, double* __restrict__ out)
{
    const int k = threadIdx.x;
    if (k >= m2) return;
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += part[(size_t)b * m2 + k];
    out[k] = t;
}

size_t cdot_scratch_doubles(int Vh, int nrhs) { return (size_t)((2 * Vh + 255) / 256) * 2 * nrhs; }

hipError_t launch_cdot(const d2* ae, const d2* be, const d2* ao, const d2* bo, int Vh, int nrhs,
                       double* scratch, double* out, hipStream_t s)
{
    const int nblk = (2 * Vh + 255) / 256;
    switch (nrhs) {
#define HISQ_CDOT_CASE(N)                                                                      \
    case N:                                                                                    \
        hipLaunchKernelGGL(k_cdot_partial<N>, dim3(nblk), dim3(256), 0, s, ae, be, ao, bo, Vh, \
                           scratch);                                                           \
        break;
        HISQ_CDOT_CASE(1)
        HISQ_CDOT_CASE(2)
        HISQ_CDOT_CASE(3)
        HISQ_CDOT_CASE(4)
        HISQ_CDOT_CASE(5)
        HISQ_CDOT_CASE(6)
        HISQ_CDOT_CASE(7)
        HISQ_CDOT_CASE(8)
#undef HISQ_CDOT_CASE
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_cdot_final, dim3(1), dim3(64), 0, s, scratch, nblk, 2 * nrhs, out);
    return hipGetLastError();
}

}  // namespace hisq
