// Internal declarations shared by the HIP kernels and the host driver of libhisq.
//
// Data layout in HBM (all sizes in complex elements of the storage precision):
//
//  * Spinor fields: [Vh][3][n], rhs innermost, one parity.  A thread that owns
//    `NR` rhs of a site reads NR contiguous complex numbers per colour.
//
//  * Packed links: a 256-byte header, then one block per OUTPUT parity P.  The
//    block of parity P holds, for every site z of parity P (index i = s/2), the
//    sixteen matrices that the Dslash of Sec. 1 eq. (3) applies at z:
//        slot  0..3   U_{z,mu}                    (forward one-hop)
//        slot  4..7  -U^dag_{z-mu,mu}              (backward one-hop)
//        slot  8..11  N_{z,mu}                    (forward three-hop, Naik)
//        slot 12..15 -N^dag_{z-3mu,mu}             (backward three-hop)
//    so that w_z = sum_slot W_slot v_{neighbour(slot)}, and every half-Dslash
//    streams exactly one block (each link once, as eq. (3) needs), perfectly
//    coalesced: slot-major, then matrix element, then site ([slot][elem][Vh]).
//    Each link is therefore stored twice (once per parity block) -- memory is
//    traded for contiguous reads, the byte count per half-Dslash is unchanged.
//    Naik slots in r14 storage keep 7 complex: rows 0 and 1 and c, with
//    row2 = c * conj(row0 x row1)  (14 reals, Table 1 "r14").
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "hisq.h"

namespace hisq {

typedef float f2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

template <typename T>
struct CplxOf;
template <>
struct CplxOf<float> {
    using type = f2;
};
template <>
struct CplxOf<double> {
    using type = d2;
};
template <typename T>
using cplx = typename CplxOf<T>::type;

constexpr int kMaxRhs = HISQ_MAX_RHS;
constexpr size_t kLinkHeaderBytes = 256;
constexpr uint32_t kLinkMagic = 0x51534948u;  // "HISQ"
constexpr int kMaxBlock = 256;
// LDS-staged Dslash: up to 512 threads per work-group, up to 64 KB of staged
// neighbour rows.
constexpr int kMaxBlockLds = 512;
constexpr int kMaxStageBytes = 64 * 1024;
// r14 / r13: bound on the relative error of the FP64 fit row2 = c conj(row0 x row1)
// (before rounding to FP32); exact fits of s*U(3) links stay near 1e-15
constexpr float kNaikTolerance = 1e-10f;
constexpr float kR9Tolerance = 4e-6f;    // r9: bounded by the FP32 rounding of H
constexpr float kR9ScaleSpread = 1e-6f;  // r9: relative spread of the Naik scales

struct LinkHeader {
    uint32_t magic;
    int32_t L[4];
    int32_t prec;
    int32_t naik;
    uint32_t naik_err_bits;  // r14 / r13 / r9: max relative round-trip error, float bits (atomicMax)
    uint32_t scale_min_bits;  // r9: smallest and largest Naik scale |det N|^(1/3), float bits
    uint32_t scale_max_bits;
    float naik_scale;         // r9: the scale the kernels apply (set after packing)
};

// Lattice description as the kernels see it.
struct Lat {
    int32_t L[4];
    int32_t Lh0;  // L0 / 2
    int32_t Vh;   // sites per parity
    int32_t sy, sz, st;  // index strides of x1, x2, x3 within a parity
};

inline Lat make_lat(const hisq_geom& g)
{
    Lat l;
    for (int mu = 0; mu < 4; ++mu) l.L[mu] = g.L[mu];
    l.Lh0 = g.L[0] / 2;
    l.sy = l.Lh0;
    l.sz = l.Lh0 * g.L[1];
    l.st = l.sz * g.L[2];
    l.Vh = l.st * g.L[3];
    return l;
}

// Packed link block of one output parity: 16 slots (U fwd, -U^dag bwd, N fwd,
// -N^dag bwd per direction), each one matrix per site.  Sizes in reals (float or
// double).  U slots hold 18 reals; a Naik slot holds 18 (FULL), 14 (R14: rows 0
// and 1 and one complex c with row2 = c conj(row0 x row1)) or 13 (R13: rows 0
// and 1 and the phase phi of c = exp(i phi) / |row0|) or 9 (R9: Hermitian H,
// N = s exp(iH) with s in the header).  R14, R13 and R9 are FP32.
__host__ __device__ constexpr int naik_reals(int nk)
{
    return nk == HISQ_NAIK_R14 ? 14 : nk == HISQ_NAIK_R13 ? 13 : nk == HISQ_NAIK_R9 ? 9 : 18;
}

__host__ __device__ constexpr int slot_reals(int slot, int nk) { return slot < 8 ? 18 : naik_reals(nk); }

__host__ __device__ constexpr int slot_real_start(int slot, int nk)
{
    return slot < 8 ? 18 * slot : 144 + naik_reals(nk) * (slot - 8);
}

__host__ __device__ inline size_t link_block_reals(int Vh, int nk)
{
    return size_t(144 + 8 * naik_reals(nk)) * size_t(Vh);
}

// FP32: position (in floats, from the slot's start) of real r (0 <= r < nr) of
// site i's matrix.  Reals group into 16-byte words, [r/4][Vh][4], so that one
// load brings two complex numbers; the nr % 4 remaining reals follow as a plane
// [Vh][nr % 4].  FP64 slots are [element][Vh] complex.  Slot starts stay 16-byte
// aligned because Vh is a multiple of 8.
__host__ __device__ inline size_t slot_real_offset32(int r, int nr, int Vh, int i)
{
    const int nw = nr / 4, rem = nr % 4;
    if (r < 4 * nw) return ((size_t)(r >> 2) * Vh + i) * 4 + (r & 3);
    return (size_t)4 * nw * Vh + (size_t)i * rem + (r - 4 * nw);
}

// Per-problem CG scalars, in device memory (FP64).
struct CgState {
    double rr[kMaxRhs];      // current (iterated) |r|^2
    double pp[kMaxRhs];      // |p|^2 of this iteration
    double tt[kMaxRhs];      // |D_oe p|^2 of this iteration
    double alpha[kMaxRhs];
    double beta[kMaxRhs];
    double thresh[kMaxRhs];  // device-side masking threshold on rr
    double rr_true[kMaxRhs]; // |b - A x|^2 of the last true-residual pass
    double aux[kMaxRhs];     // |b|^2
    double rrmax[kMaxRhs];   // largest iterated |r|^2 since the last true-residual pass
    int32_t active[kMaxRhs];
    int32_t status[kMaxRhs];
    int32_t iters[kMaxRhs];
    int32_t sel[kMaxRhs];    // rhs selected for the next true-residual pass
    int32_t maxiter;
    int32_t frozen;          // 1 while the autotuner times kernels: finishers write nothing
    int32_t pad[6];
};

enum Epi {
    EPI_PLAIN = 0,  // out = D in
    EPI_NORM = 1,   // t = D_oe p; |t|^2 -> tt, alpha
    EPI_CG = 2,     // u = D_eo t; q = 4m^2 p - u; x += alpha p; r -= alpha q; |r|^2 -> rr, beta
    EPI_RESID = 3   // (FP64) r = b - (4m^2 x - D_eo t) for selected rhs; |r|^2 -> rr_true
};

// Arguments of one Dslash launch (one problem).
template <typename T>
struct DslashArgs {
    Lat lat;
    int parity;  // output parity
    const cplx<T>* links;  // link block of the output parity
    const cplx<T>* in;
    cplx<T>* out;
    // CG epilogue
    const cplx<T>* p;
    cplx<T>* x;
    cplx<T>* r;
    // residual epilogue (FP64 b, x)
    const d2* b;
    const d2* xh;
    double mass4;  // 4 m^2
    CgState* state;
    double* red;    // reduction scratch: partials + group sums
    uint32_t* cnt;  // reduction counters (zero between launches)
    int ntiles;
    int remap;
    int rows;  // LDS-staged x-rows per tile (0: unstaged)
    const float* naik_scale;  // r9 links: the scale in their header
};

template <typename T>
struct PupdateArgs {
    Lat lat;
    const cplx<T>* r;
    cplx<T>* p;
    CgState* state;
    double* red;
    uint32_t* cnt;
    int ntiles;
    int remap;
};

// One problem of a batched launch: the arguments of its three CG phases and
// its range of work-groups in the flattened (problem, tile) grid.
template <typename T>
struct BatchProb {
    PupdateArgs<T> k1;
    DslashArgs<T> k2;
    DslashArgs<T> k3;
    int n;
    int nr;
    int block_start;
    int nblocks;
};

template <typename T>
struct BatchTable {
    BatchProb<T> p[HISQ_MAX_PROBLEMS];
    int nprob;
    int total_blocks;
};

// Launch shape: rhs per thread, work-group size (one tile of bs threads per
// work-group), XCD-contiguous tile order.
struct Tile {
    int nr;
    int bs;
    int remap;
    int rows = 0;  // > 0: LDS-staged Dslash, the work-group covers `rows` x-rows
};

// Reduction scratch for a grid of up to `blocks` work-groups.
inline size_t red_doubles(size_t blocks) { return (blocks + (blocks + 63) / 64) * kMaxRhs; }
inline size_t red_counters(size_t blocks) { return 1 + (blocks + 63) / 64; }

// Launchers, defined in the per-precision kernel objects.  cm selects the
// colour-major field layout [3][Vh][n] (the solver's); the plain Dslash also
// exists for the site-major canonical layout [Vh][3][n].
hipError_t launch_dslash_f64(int epi, int nrhs, const Tile& t, const DslashArgs<double>& a,
                             hipStream_t s, bool cm);
// nk: Naik storage of the FP32 links (HISQ_NAIK_FULL, _R14, _R13)
hipError_t launch_dslash_f32(int epi, int nk, int nrhs, const Tile& t, const DslashArgs<float>& a,
                             hipStream_t s, bool cm);
hipError_t launch_dslash_batched_f64(int epi, const BatchTable<double>* tab, int total_blocks,
                                     int bs, hipStream_t s);
hipError_t launch_dslash_batched_f32(int epi, int nk, const BatchTable<float>* tab,
                                     int total_blocks, int bs, hipStream_t s);
hipError_t launch_pupdate_batched_f64(const BatchTable<double>* tab, int total_blocks, int bs,
                                      hipStream_t s);
hipError_t launch_pupdate_batched_f32(const BatchTable<float>* tab, int total_blocks, int bs,
                                      hipStream_t s);
// rhs-per-thread tiles the batched kernels are built for
inline bool batched_nr_ok(int n, int nr) { return nr == n || (n % 2 == 0 && nr == n / 2); }
// Streaming p-update for bundles of 1, 2, 4 or 8 rhs (any tile).
inline bool pupdate_flat_ok(int n) { return n == 1 || n == 2 || n == 4 || n == 8; }
hipError_t launch_pupdate_flat_f64(int nrhs, const PupdateArgs<double>& a, hipStream_t s);
hipError_t launch_pupdate_flat_f32(int nrhs, const PupdateArgs<float>& a, hipStream_t s);
hipError_t launch_pupdate_f64(int nrhs, const Tile& t, const PupdateArgs<double>& a,
                              hipStream_t s);
hipError_t launch_pupdate_f32(int nrhs, const Tile& t, const PupdateArgs<float>& a,
                              hipStream_t s);

// Elementwise and reduction helpers (blas.hip).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_state_reset(CgState* st, int nrhs, int active, hipStream_t s);
// per-rhs |v|^2 of a colour-major FP64 field
hipError_t launch_norm2_f64(const d2* v, int Vh, int nrhs, double* out, double* red,
                            uint32_t* cnt, hipStream_t s);
hipError_t launch_to_f32_sel(const d2* src, f2* dst, size_t ncplx, int nrhs, const CgState* st,
                             hipStream_t s);
hipError_t launch_accum_sel(d2* xh, f2* xl, size_t ncplx, int nrhs, const CgState* st,
                            hipStream_t s);
hipError_t launch_copy_f64(const d2* src, d2* dst, size_t ncplx, hipStream_t s);
hipError_t launch_layout(const d2* src, d2* dst, int Vh, int nrhs, bool to_colour_major, hipStream_t s);
hipError_t launch_axpby(const d2* a, const d2* b, d2* out, size_t n, double alpha, double beta,
                        hipStream_t s);
size_t cdot_scratch_doubles(int Vh, int nrhs);
// out[2k], out[2k+1] = re, im of sum conj(a) b over both half fields, rhs k
hipError_t launch_cdot(const d2* ae, const d2* be, const d2* ao, const d2* bo, int Vh, int nrhs,
                       double* scratch, double* out, hipStream_t s);
// d^n D / d mu^n at mu = 0 (n >= 1), FP64 links of the output parity, site-major
hipError_t launch_dslash_dmu(const Lat& lat, int parity, int nrhs, int nder, const d2* lk,
                             const d2* in, d2* out, hipStream_t s);
hipError_t launch_zero_sel(d2* v, size_t ncplx, int nrhs, const CgState* st, hipStream_t s);
hipError_t launch_redot(const d2* y, const d2* x, int Vh, int nrhs, double scale, double* out,
                        double* red, uint32_t* cnt, hipStream_t s);

// The solve of hisq_cg_solve over a workspace region (api.cpp); host_buf, if
// not NULL, holds HISQ_MAX_PROBLEMS host copies of the CG state in place of
// the calling thread's pinned buffer.
int cg_solve_on(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                const void* links64, const void* links32, const double* b_e, double* x_e,
                void* ws, size_t ws_bytes, hisq_info* info, void* stream, CgState* host_buf);
size_t cg_workspace_bytes(const Lat& lat, int nrhs, int mode);
// Sets the message of hisq_last_error() for this thread; returns code.
int report_error(int code, const char* fmt, ...);

// Link packing (pack.hip) and the link force (force.hip).
hipError_t launch_pack(const Lat& lat, const d2* U, const d2* N, int prec, int naik,
                       void* packed, hipStream_t s);
// link force from colour-major FP64 fields x, y (even) and D_oe x, D_oe y (odd)
hipError_t launch_force(const Lat& lat, int nrhs, const d2* xc, const d2* yc, const d2* txc,
                        const d2* syc, d2* GU, d2* GN, hipStream_t s);

}  // namespace hisq
