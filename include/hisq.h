/*
 * hisq.h -- C ABI of libhisq, an MI355X (gfx950) library for the even-odd
 * preconditioned HISQ staggered-fermion system
 *
 *     A x_e = b_e,   A = 4 m^2 - D_eo D_oe,
 *
 * solved by conjugate gradient on bundles of 1..8 right-hand sides.
 *
 * Source: O. Kaczmarek, C. Schmidt, P. Steinbrecher, M. Wagner, "Conjugate
 * gradient solvers on Intel Xeon Phi and NVIDIA GPUs", GPUHEP2014.
 *   - D is the HISQ Dslash of Sec. 1, eq. (3): one-hop smeared links U and
 *     three-hop Naik links N, summed over the four directions mu = 0..3 of a
 *     periodic 4-D lattice; U, N are complex 3x3, fields complex 3-vectors.
 *   - A bundle of n rhs is n independent applications of D sharing each link
 *     load (eq. (4)).
 *   - Naik links may be stored with 14 reals ("r14", Table 1), 13 or 9.
 *   - The fermion matrix is read as M = 2m + D; D is anti-Hermitian and only
 *     couples opposite parities, so the even block of M^dag M is
 *     A = 4 m^2 - D_eo D_oe, Hermitian positive definite (lambda_min >= 4 m^2).
 *   - The solver serves stochastic trace estimation (Sec. 1, eq. (2)): many
 *     inversions on one fixed gauge field.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Geometry   hisq_geom.L = (L0, L1, L2, L3); every L_mu must be even and >= 4,
 *            and Vh * 144 < 2^31 (packed links use 32-bit offsets within a
 *            parity block: up to about 96^3 x 24), else HISQ_EGEOM.
 *            V = L0 L1 L2 L3, Vh = V/2.
 * Sites      s = x0 + L0*(x1 + L1*(x2 + L2*x3)); parity of s = (x0+x1+x2+x3) mod 2;
 *            even means parity 0.
 * Links      canonical input: [4][V][3][3] complex128 (mu, site, row, col),
 *            interleaved (re, im), row-major 3x3.  Staggered phases and boundary
 *            signs must already be folded in.  Packed links are opaque.
 * Fields     half-lattice, one parity: [Vh][3][n] complex, rhs innermost; the row
 *            of site s is s/2 ("site-major").  Complex128 at the solver
 *            boundary; in the storage precision (complex64 or complex128) for
 *            hisq_dslash, which also accepts the colour-major order [3][Vh][n]
 *            that the solvers iterate on internally.
 * Memory     every data pointer is a DEVICE pointer owned by the caller, except
 *            hisq_info / hisq_params / hisq_problem structs, which are host memory.
 *            Field, link and workspace buffers must be 16-byte aligned (they are
 *            read with 16-byte vector loads); HISQ_EINVAL otherwise.
 *            No entry point allocates device memory: the solvers take a
 *            workspace sized by the *_workspace_bytes() queries
 *            (hisq_cg_solve_noalloc uses a static device array instead).
 *            Buffers must not overlap.
 * Streams    `stream` is a hipStream_t passed as void* (NULL = default stream).
 *            hisq_dslash and hisq_pack_links (FULL Naik) are asynchronous.  The
 *            solvers block the calling host thread until the solve ends, because
 *            convergence decisions are taken on the host, but run all device
 *            work on `stream`.
 * Errors     0 = HISQ_OK.  Negative = nothing was launched (bad argument,
 *            geometry, workspace, packing, or a HIP error); the message is
 *            available from hisq_last_error() (thread-local).  Positive = a
 *            numerical outcome of a solve whose x holds the last iterate.
 * Threads    entry points are thread-safe; calls that share buffers race.
 */
#ifndef HISQ_H
#define HISQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HISQ_OK 0
#define HISQ_EINVAL (-1)      /* null pointer, n outside 1..8, tol <= 0, bad enum   */
#define HISQ_EGEOM (-2)       /* an extent odd or < 4, or the lattice too large     */
#define HISQ_EWORKSPACE (-3)  /* workspace smaller than hisq_workspace_bytes()      */
#define HISQ_EPACK (-4)       /* r14/r13 fit error above 1e-10 |N| (not s*U(3))      */
#define HISQ_EHIP (-5)        /* a HIP runtime call failed                           */
#define HISQ_NOT_CONVERGED 1  /* maxiter reached before the true residual passed    */
#define HISQ_BREAKDOWN 2      /* <p, A p> <= 0 or not finite                         */

#define HISQ_MAX_RHS 8
#define HISQ_MAX_PROBLEMS 16
#define HISQ_MAX_DERIVATIVE 8   /* highest mu-derivative order of hisq_dslash_dmu     */
#define HISQ_MAX_INSERTIONS 8   /* operator insertions per hisq_trace_estimate term   */

enum hisq_prec { HISQ_PREC_F64 = 0, HISQ_PREC_F32 = 1 };
/* Naik link storage (Sec. 1: reconstruction from 9 or 13/14 floats, Table 1 "r14"):
 * FULL 18 reals; R14 rows 0, 1 and one complex c with row2 = c conj(row0 x row1);
 * R13 rows 0, 1 and the phase phi of c, |c| = 1 / |row0|; R9 one Hermitian H
 * with N = s exp(iH), s one scale for the whole field.  R14, R13 and R9 are
 * exact for N = s V with V in U(3), s > 0 (R9: the same s everywhere), and FP32
 * only. */
enum hisq_naik { HISQ_NAIK_FULL = 0, HISQ_NAIK_R14 = 1, HISQ_NAIK_R13 = 2, HISQ_NAIK_R9 = 3 };
enum hisq_mode { HISQ_MODE_FP64 = 0, HISQ_MODE_MIXED = 1 };
/* field order: [Vh][3][n] (site-major, the default) or [3][Vh][n] */
enum hisq_layout { HISQ_LAYOUT_SITE = 0, HISQ_LAYOUT_COLOUR = 1 };

typedef struct {
    int32_t L[4];
} hisq_geom;

/* Solver controls.  hisq_default_params() fills the defaults noted here. */
typedef struct {
    int32_t mode;        /* HISQ_MODE_FP64 (default) or HISQ_MODE_MIXED                */
    int32_t naik;        /* Naik storage of links32 in MIXED mode (HISQ_NAIK_FULL)      */
    double tol;          /* stop when ||b_k - A x_k|| <= tol ||b_k|| in FP64 (1e-10)    */
    int32_t maxiter;     /* per-rhs iteration cap (20000)                               */
    double delta;        /* MIXED: reliable update when ||r|| < delta * max ||r|| (0.1) */
    int32_t poll_every;  /* iterations between host polls; 0 = chosen from the volume   */
    int32_t use_x0;      /* 1: x_e holds the start vector on entry (0: start from 0)   */
    int32_t use_graph;   /* 1: each poll block of iterations is one hipGraph (1)        */
    int32_t profile;     /* 1: time every Dslash launch with HIP events into info (0)   */
} hisq_params;

/* Kernel classes timed when hisq_params.profile = 1. */
enum hisq_kclass {
    HISQ_K_PUPDATE = 0,   /* p = r + beta p, |p|^2                           */
    HISQ_K_DSLASH_OE = 1, /* t = D_oe p, |t|^2                               */
    HISQ_K_DSLASH_EO = 2, /* D_eo t + CG epilogue: x, r updates, |r|^2       */
    HISQ_K_RELIABLE = 3,  /* FP64 true residual (two FP64 half-Dslash + BLAS) */
    HISQ_K_FORCE = 4,     /* hisq_cg_solve_backward: the link-force kernel    */
    HISQ_K_COUNT = 5
};

typedef struct {
    int32_t iters[HISQ_MAX_RHS];         /* CG iterations per rhs                       */
    int32_t status[HISQ_MAX_RHS];        /* HISQ_OK / HISQ_NOT_CONVERGED / HISQ_BREAKDOWN */
    double rel_true_res[HISQ_MAX_RHS];   /* ||b - A x|| / ||b||, FP64, from returned x  */
    double rel_iter_res[HISQ_MAX_RHS];   /* last iterated residual / ||b||             */
    int32_t reliable_updates;            /* FP64 true-residual recomputations           */
    int32_t polls;                       /* host polls                                  */
    int32_t total_iters;                 /* iterations of the bundle (max over rhs)     */
    int32_t block_size;                  /* tuned work-group size of the D_oe Dslash    */
    int32_t rhs_per_thread;              /* tuned rhs tile of the D_oe Dslash           */
    int32_t tile_order;                  /* tuned work-group -> tile order (0..3)       */
    int32_t stage_rows;                  /* tuned LDS-staged x-rows per tile (0: none)  */
    int32_t eo_block_size;               /* the same four for the D_eo Dslash with the  */
    int32_t eo_rhs_per_thread;           /* CG epilogue (equal to the above in batched  */
    int32_t eo_tile_order;               /* solves)                                     */
    int32_t eo_stage_rows;
    int32_t reserved;
    double seconds;                      /* host wall time of the solve                 */
    double kernel_ms[HISQ_K_COUNT];      /* profile = 1: summed event time per class    */
    int32_t kernel_launches[HISQ_K_COUNT];
} hisq_info;

/* One independent solve of a batch (hisq_cg_solve_batched). */
typedef struct {
    hisq_geom geom;
    double mass;
    int32_t nrhs;
    const void* links64; /* packed FP64 links (FULL Naik)                     */
    const void* links32; /* packed FP32 links (params->naik), MIXED mode only */
    const double* b;     /* [Vh][3][nrhs] complex128, even sites               */
    double* x;           /* [Vh][3][nrhs] complex128, solution (start if use_x0) */
} hisq_problem;

/* Fill *p with the defaults listed in hisq_params. */
void hisq_default_params(hisq_params* p);

/*
 * Size in bytes of a packed link buffer for `prec` (HISQ_PREC_*) and Naik
 * storage `naik` (HISQ_NAIK_*; R14, R13 and R9 only with F32).  0 on invalid input.
 */
size_t hisq_links_bytes(const hisq_geom* g, int prec, int naik);

/*
 * Workspace bytes needed by hisq_cg_solve for nrhs rhs in `mode`
 * (HISQ_MODE_*).  0 on invalid input.  The workspace is caller-owned device
 * memory, needs no initialisation and holds nothing between calls.
 */
size_t hisq_workspace_bytes(const hisq_geom* g, int nrhs, int mode);

/* Workspace bytes needed by hisq_cg_solve_backward (more than the forward). */
size_t hisq_backward_workspace_bytes(const hisq_geom* g, int nrhs, int mode);

/* Workspace bytes for hisq_cg_solve_batched over nprob problems. */
size_t hisq_batched_workspace_bytes(int nprob, const hisq_problem* probs, int mode);

/* Workspace bytes for hisq_solve_full and hisq_trace_estimate. */
size_t hisq_full_workspace_bytes(const hisq_geom* g, int nrhs, int mode);
size_t hisq_trace_workspace_bytes(const hisq_geom* g, int nrhs, int mode);

/*
 * Pack canonical links U, N ([4][V][3][3] complex128, device) into `packed`
 * (device, hisq_links_bytes(g, prec, naik) bytes) for the Dslash of eq. (3).
 * For naik = R14 every Naik link (and its adjoint) is stored as rows 0, 1 and
 * one complex c with row2 = c conj(row0 x row1); for R13 as rows 0, 1 and the
 * phase of c, whose modulus 1/|row0| follows from N = s V, V in U(3); for R9
 * as the 9 reals of H = -i log(N / s) with s = |det N|^(1/3).  These calls then
 * synchronize `stream` and return HISQ_EPACK if, for R14 and R13, the FP64 fit
 * of row 2 from rows 0 and 1 misses by more than 1e-10 of the link's norm (N is
 * not a positive multiple of a U(3) matrix), or, for R9, if the FP32 decode
 * misses by more than 4e-6 (the FP32 rounding of H is at that level) or the
 * scales s of the Naik links differ by more than 1e-6 (not one multiple
 * throughout).  A buffer that fails is left with an invalid header, which
 * every other entry point rejects.
 *
 * Every entry point that takes packed links checks the buffer's header against
 * its arguments (lattice, precision, Naik storage; FP64/FULL for links64) and
 * returns HISQ_EINVAL on a mismatch, before launching anything.  The blocking
 * solvers read the header back with a 256-byte copy on `stream`; hisq_dslash
 * and hisq_dslash_dmu use what this process recorded when it packed (or last
 * read) the buffer, and read it back only for a buffer they have not seen.
 */
int hisq_pack_links(const hisq_geom* g, const double* U, const double* N, int prec, int naik,
                    void* packed, void* stream);

/*
 * out = D_{out_parity, 1-out_parity} in  (Sec. 1 eqs. (3)-(4)): the HISQ Dslash
 * from the fields of parity 1-out_parity to those of parity out_parity, for
 * nrhs independent rhs sharing every link load.  `in`, `out`: complex in the
 * storage precision `prec` of `packed`, in the order `layout` (HISQ_LAYOUT_*):
 * [Vh][3][nrhs] or [3][Vh][nrhs].  The colour-major order lets the 64 lanes of
 * a wavefront read one contiguous stretch per colour; the solvers use it.
 * Asynchronous.
 */
int hisq_dslash(const hisq_geom* g, int out_parity, int nrhs, int prec, int naik, int layout,
                const void* packed, const void* in, void* out, void* stream);

/*
 * Solve (4 m^2 - D_eo D_oe) x_k = b_k for each rhs k of the bundle by CG.
 * links64: packed FP64/FULL links (always needed: FP64 mode iterates on them,
 * MIXED mode uses them for the true residual).  links32: packed FP32 links
 * with Naik storage params->naik (MIXED only; may be NULL in FP64 mode).
 * b_e, x_e: [Vh][3][nrhs] complex128 device buffers (copied into the
 * colour-major working order inside the workspace).  Ends when every rhs has
 * ||b_k - A x_k|| <= tol ||b_k|| recomputed in FP64 from x, or failed.  Returns
 * HISQ_OK, or the worst per-rhs status (NOT_CONVERGED < BREAKDOWN), or < 0.
 */
int hisq_cg_solve(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                  const void* links64, const void* links32, const double* b_e, double* x_e,
                  void* ws, size_t ws_bytes, hisq_info* info, void* stream);

/*
 * Backward of x = A^{-1} b for the loss L = sum_k Re(grad_x_k^dag x_k):
 * solves A y = grad_x with the same operator (A is Hermitian), then with
 * t = D_oe x and s = D_oe y writes, in PyTorch's complex-gradient convention
 * G = dL/dRe + i dL/dIm:
 *   grad_U[mu][a] =  sum_k (y_a t_{a+mu}^dag + x_a s_{a+mu}^dag)   a even
 *   grad_U[mu][a] = -sum_k (t_a y_{a+mu}^dag + s_a x_{a+mu}^dag)   a odd
 *   grad_N: the same with a + 3 mu;   grad_m = -8 m sum_k Re(y_k^dag x_k);
 *   grad_b = y (if grad_b is not NULL).
 * grad_U, grad_N: [4][V][3][3] complex128 (device); grad_m: one double (device).
 * U and N are treated as independent inputs.  x_e is the forward solution.
 */
int hisq_cg_solve_backward(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                           const void* links64, const void* links32, const double* x_e,
                           const double* grad_x, double* grad_U, double* grad_N,
                           double* grad_m, double* grad_b, void* ws, size_t ws_bytes,
                           hisq_info* info, void* stream);

/*
 * Solve nprob independent problems (different lattices, masses and bundle
 * sizes) together: every CG phase is one launch over the work of all problems,
 * with per-problem coefficients and per-rhs masking.  infos: nprob entries.
 */
int hisq_cg_solve_batched(int nprob, const hisq_problem* probs, const hisq_params* p, void* ws,
                          size_t ws_bytes, hisq_info* infos, void* stream);

/*
 * out = d^nder D / d mu^nder in, at mu = 0, from the fields of parity
 * 1-out_parity to those of parity out_parity: the derivative operators of the
 * trace formula Sec. 1 eq. (2).  The paper does not write M(mu) out; this
 * library reads it as the usual one: a temporal hop of h steps (h = +-1 for U,
 * +-3 for N) carries exp(h mu), spatial hops carry none.  So for nder >= 1 only
 * the time-direction terms of eq. (3) remain, weighted by h^nder; nder = 0 is
 * the Dslash itself.  links64: packed FP64/FULL links.  in, out: site-major
 * [Vh][3][nrhs] complex128.  0 <= nder <= HISQ_MAX_DERIVATIVE.  Asynchronous.
 */
int hisq_dslash_dmu(const hisq_geom* g, int out_parity, int nrhs, int nder, const void* links64,
                    const double* in, double* out, void* stream);

/*
 * Solve M x = b on the full lattice, M = 2m + D (the reading of the fermion
 * matrix; Sec. 1 eq. (3) gives D), through the even-odd reduction:
 * (4m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o by the CG of hisq_cg_solve (same
 * params, start vector zero), then x_o = (b_o - D_oe x_e) / (2m).
 * b_e, b_o, x_e, x_o: site-major [Vh][3][nrhs] complex128 device buffers.
 * mass must be finite and nonzero.  info and the return value are those of the
 * even solve.  Blocks until done.
 */
int hisq_solve_full(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                    const void* links64, const void* links32, const double* b_e, const double* b_o,
                    double* x_e, double* x_o, void* ws, size_t ws_bytes, hisq_info* info,
                    void* stream);

/*
 * One bundle of terms of the stochastic trace estimator, Sec. 1 eq. (2):
 *   est_k = eta_k^dag M^(n_1) M^-1 M^(n_2) M^-1 ... M^(n_j) M^-1 eta_k
 * for orders = (n_1 .. n_j) (host array, j = ninsert), M^(n) = d^n M / d mu^n
 * at mu = 0 (hisq_dslash_dmu; n = 0 is M).  Evaluated right to left with
 * hisq_solve_full for each M^-1.  eta_e, eta_o: the caller's noise vectors
 * (site-major [Vh][3][nrhs] complex128; the library draws no random numbers).
 * est: device, [nrhs][2] doubles (re, im).  The mean of est_k over many
 * vectors estimates the trace.  info: total iterations, reliable updates and
 * seconds summed over the j solves; the rest from the last solve.  Returns the
 * worst solve status, or < 0.  Blocks until done.
 */
int hisq_trace_estimate(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                        const void* links64, const void* links32, int ninsert, const int* orders,
                        const double* eta_e, const double* eta_o, double* est, void* ws,
                        size_t ws_bytes, hisq_info* info, void* stream);

/*
 * Autotuner control (process-wide).  mode 0: time the candidate tiles on first
 * use of a (lattice, nrhs, precision, Naik, kernel) key and cache the fastest
 * (default); mode 1: always use rhs_per_thread / block_size / tile_order /
 * stage_rows;
 * mode 2: built-in default, no timing.  rhs_per_thread must divide the bundle
 * with a power-of-two quotient (otherwise the forced tile is ignored for that
 * bundle), block_size is 64, 128 or 256, tile_order is 0 (canonical site
 * order), 1 (a contiguous slab of tiles per XCD), 2 (per XCD, the time
 * slices of one slice position back to back; falls back to 1 where tiles
 * would straddle a time slice) or 3 (XCD j owns z-chunk j of L2/8 planes and
 * walks it x-y position outermost, then t, then z; falls back to 1 unless
 * L2 % 8 == 0 and a tile divides an x-y plane).  stage_rows > 0 selects the
 * LDS-staged Dslash on colour-major fields: a work-group covers stage_rows
 * whole x-rows of one (z, t) plane (block size stage_rows * L0/2 * n /
 * rhs_per_thread, which then replaces block_size) and reads its x and y
 * neighbours from LDS; where that shape is not possible (block not a multiple
 * of 64 or above 512 threads, L1 % stage_rows != 0, staged rows above 64 KB,
 * site-major fields) the unstaged kernel runs.  Neither the order nor the
 * staging changes results.  Returns HISQ_EINVAL for an unknown mode or
 * out-of-range values.
 */
int hisq_set_tuning(int mode, int rhs_per_thread, int block_size, int tile_order, int stage_rows);

/*
 * In a single solve the D_eo half-Dslash with the CG epilogue (it also reads
 * p, x, r and writes x, r) is tuned on its own, separately from D_oe, whose
 * tile the p-update, the batched kernels and the FP64 residual share; both
 * tiles are reported in hisq_info.  This call gives the D_eo kernel its own
 * tile under tuning mode 1, with the arguments of hisq_set_tuning; until it is
 * called, after rhs_per_thread = 0, and after every hisq_set_tuning call, that
 * kernel takes the mode-1 tile of hisq_set_tuning.  Returns HISQ_EINVAL for
 * out-of-range values.
 */
int hisq_set_tuning_eo(int rhs_per_thread, int block_size, int tile_order, int stage_rows);

/*
 * For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc) and so cannot provide
 * the workspace of hisq_cg_solve: the same solve, with the same arguments
 * except the workspace, whose scratch (CG scalars, reduction partials and
 * counters, working fields) lives in a static device array of
 * HISQ_NOALLOC_SCRATCH_BYTES per GPU, held from library load to process end.
 * A solve whose hisq_workspace_bytes() exceeds that returns HISQ_EWORKSPACE
 * (64 MiB: e.g. 24^3 x 6 with up to 5 rhs in MIXED mode, 32^3 x 8 with one).
 * It calls no hipMalloc, hipFree or other allocating routine: poll blocks run
 * without a hipGraph (params->use_graph and ->profile are ignored) and the
 * host copies of the CG state are the calling thread's ordinary memory.  All
 * calls on one GPU share its array: calls that overlap in time on one GPU
 * (from several threads or streams) race and must be serialised by the
 * caller.  Every region that must start at zero is cleared by each call.
 */
#define HISQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hisq_cg_solve_noalloc(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                          const void* links64, const void* links32, const double* b_e,
                          double* x_e, hisq_info* info, void* stream);

/* Message of the last failing call on this thread ("" if none). */
const char* hisq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HISQ_H */
