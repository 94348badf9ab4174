// Host side of libhisq: argument checks, workspace layout, the autotuner, the
// CG driver (polling, reliable updates, hipGraph capture) and the C ABI.
//
// The solver is the even-odd CG for A x = b with A = 4m^2 - D_eo D_oe and the
// HISQ Dslash of Sec. 1 eq. (3), run on bundles of n rhs (eq. (4)); every rhs
// has its own alpha, beta and convergence flag.  Per iteration three kernels
// run: p = r + beta p (|p|^2), t = D_oe p (|t|^2, alpha), and
// D_eo t fused with x += alpha p, r -= alpha (4m^2 p - D_eo t) (|r|^2, beta).
// alpha uses <p, A p> = 4m^2 |p|^2 + |D_oe p|^2, which holds because D is
// anti-Hermitian (D_eo^dag = -D_oe).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "hisq_internal.h"

using namespace hisq;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess) return fail(HISQ_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Runs f when the scope ends, also on an early error return: releases HIP
// events and graphs on every path.
template <typename F>
struct ScopeExit {
    F f;
    ~ScopeExit() { f(); }
};
template <typename F>
ScopeExit<F> on_scope_exit(F f)
{
    return ScopeExit<F>{f};
}
void destroy_events(hipEvent_t* e, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (e[i]) {
            hipEventDestroy(e[i]);
            e[i] = nullptr;
        }
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int check_geom(const hisq_geom* g, Lat* lat)
{
    if (!g) return fail(HISQ_EINVAL, "geometry is NULL");
    long long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        if (g->L[mu] < 4 || (g->L[mu] % 2) != 0)
            return fail(HISQ_EGEOM, "extent L[%d] = %d must be even and >= 4", mu, g->L[mu]);
        V *= g->L[mu];
    }
    // 32-bit indexing of the packed link blocks: 144 complex per site and parity
    if (V / 2 * 144 >= (1LL << 31)) return fail(HISQ_EGEOM, "lattice too large (V = %lld)", V);
    *lat = make_lat(*g);
    return HISQ_OK;
}

// Field, link and workspace buffers are read with 16-byte vector loads.
bool misaligned(std::initializer_list<const void*> ptrs)
{
    for (const void* q : ptrs)
        if (q && (reinterpret_cast<uintptr_t>(q) & 15u) != 0) return true;
    return false;
}

#define HISQ_CHECK_ALIGNED(...)                                                     \
    do {                                                                            \
        if (misaligned({__VA_ARGS__}))                                              \
            return fail(HISQ_EINVAL, "device buffers must be 16-byte aligned");     \
    } while (0)

bool valid_naik(int nk)
{
    return nk == HISQ_NAIK_FULL || nk == HISQ_NAIK_R14 || nk == HISQ_NAIK_R13 || nk == HISQ_NAIK_R9;
}

// r9 links: the Naik scale the kernels read, in the buffer's header
const float* naik_scale_of(const void* packed)
{
    return packed ? &reinterpret_cast<const LinkHeader*>(packed)->naik_scale : nullptr;
}

// ---------------------------------------------------------------------------
// Packed-link headers.  A buffer is only valid for the lattice, precision and
// Naik storage it was packed for: a Dslash that took an r14 block for a full
// one, or links of a smaller lattice, would read past the allocation.  Every
// entry point compares the header with its arguments before launching.
// hisq_pack_links records what it wrote; a buffer the library has not seen in
// this process (or, for the blocking solvers, any buffer) has its 256-byte
// header read back once with a device-to-host copy on the caller's stream.
struct LinkKey {
    int32_t L[4];
    int32_t prec;
    int32_t naik;
};
std::mutex g_links_mu;
std::map<const void*, LinkKey> g_links;

void remember_links(const void* packed, const Lat& lat, int prec, int naik)
{
    LinkKey k{{lat.L[0], lat.L[1], lat.L[2], lat.L[3]}, prec, naik};
    std::lock_guard<std::mutex> lk(g_links_mu);
    g_links[packed] = k;
}

void forget_links(const void* packed)
{
    std::lock_guard<std::mutex> lk(g_links_mu);
    g_links.erase(packed);
}

// HISQ_OK if `packed` holds links packed for (lat, prec, naik); re_read: read
// the header from the device even if this process packed the buffer.
int check_links(const char* what, const void* packed, const Lat& lat, int prec, int naik,
                hipStream_t s, bool re_read)
{
    LinkKey k{};
    bool known = false;
    if (!re_read) {
        std::lock_guard<std::mutex> lk(g_links_mu);
        auto it = g_links.find(packed);
        if (it != g_links.end()) {
            k = it->second;
            known = true;
        }
    }
    if (!known) {
        LinkHeader h{};
        HIP_TRY(hipMemcpyAsync(&h, packed, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h.magic != kLinkMagic)
            return fail(HISQ_EINVAL, "%s: not a packed link buffer (bad header)", what);
        for (int mu = 0; mu < 4; ++mu) k.L[mu] = h.L[mu];
        k.prec = h.prec;
        k.naik = h.naik;
        std::lock_guard<std::mutex> lk(g_links_mu);
        g_links[packed] = k;
    }
    for (int mu = 0; mu < 4; ++mu)
        if (k.L[mu] != lat.L[mu])
            return fail(HISQ_EINVAL, "%s: packed for lattice %dx%dx%dx%d, called with %dx%dx%dx%d",
                        what, k.L[0], k.L[1], k.L[2], k.L[3], lat.L[0], lat.L[1], lat.L[2],
                        lat.L[3]);
    if (k.prec != prec || k.naik != naik)
        return fail(HISQ_EINVAL, "%s: packed with prec %d, naik %d; called with prec %d, naik %d",
                    what, k.prec, k.naik, prec, naik);
    return HISQ_OK;
}

// The two link buffers of a solve: FP64/FULL, and in MIXED mode FP32 with the
// params' Naik storage.
int check_solve_links(const void* links64, const void* links32, const Lat& lat, int mode,
                      int naik, hipStream_t s)
{
    int rc = check_links("links64", links64, lat, HISQ_PREC_F64, HISQ_NAIK_FULL, s, true);
    if (rc == HISQ_OK && mode == HISQ_MODE_MIXED)
        rc = check_links("links32", links32, lat, HISQ_PREC_F32, naik, s, true);
    return rc;
}

bool valid_nr(int n, int nr)
{
    if (nr < 1 || nr > n || n % nr != 0) return false;
    const int G = n / nr;
    return G == 1 || G == 2 || G == 4 || G == 8;
}

// ---------------------------------------------------------------------------
// Workspace layout (every region 256-byte aligned).
struct Ws {
    CgState* st = nullptr;
    double* red = nullptr;
    uint32_t* cnt = nullptr;
    size_t cnt_bytes = 0;
    d2* r64 = nullptr;  // FP64 residual (the iteration r in FP64 mode)
    d2* t64 = nullptr;  // FP64 odd temporary (the iteration t in FP64 mode)
    d2* p64 = nullptr;  // FP64 mode: search direction
    f2* r32 = nullptr;  // MIXED: FP32 r, p, t, x_lo
    f2* p32 = nullptr;
    f2* t32 = nullptr;
    f2* x32 = nullptr;
    d2* xc = nullptr;  // colour-major copies of x and b (the solver's layout)
    d2* bc = nullptr;
    d2* y = nullptr;  // backward: adjoint solution, D_oe x, D_oe y
    d2* tx = nullptr;
    d2* sy = nullptr;
    d2* bp = nullptr;  // full solve: reduced source 2m b_e - D_eo b_o, a Dslash output
    d2* fo = nullptr;
    d2* ve = nullptr;  // trace estimator: M^(n) applied (even, odd), M^-1 applied
    d2* vo = nullptr;
    d2* xe = nullptr;
    d2* xo = nullptr;
    double* dot = nullptr;  // per-work-group partials of the final dot products
};

// What a workspace serves: the extra regions beyond the solver's own.
enum WsKind { WS_SOLVE = 0, WS_BACKWARD = 1, WS_FULL = 2, WS_TRACE = 3 };

size_t ws_layout(const Lat& lat, int n, int mode, int kind, char* base, Ws* w)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        const size_t o = off;
        off = align256(off + bytes);
        return base ? base + o : nullptr;
    };
    const size_t f64 = (size_t)lat.Vh * 3 * n * sizeof(d2);
    const size_t f32 = (size_t)lat.Vh * 3 * n * sizeof(f2);
    const size_t maxblocks = (size_t)lat.Vh * 8 / 64 + 1;  // block >= 64 threads, <= 8 per site
    w->st = (CgState*)take(sizeof(CgState));
    w->red = (double*)take(red_doubles(maxblocks) * sizeof(double));
    w->cnt_bytes = align256(red_counters(maxblocks) * sizeof(uint32_t));
    w->cnt = (uint32_t*)take(w->cnt_bytes);
    w->r64 = (d2*)take(f64);
    w->t64 = (d2*)take(f64);
    w->xc = (d2*)take(f64);
    w->bc = (d2*)take(f64);
    if (mode == HISQ_MODE_FP64) {
        w->p64 = (d2*)take(f64);
    } else {
        w->r32 = (f2*)take(f32);
        w->p32 = (f2*)take(f32);
        w->t32 = (f2*)take(f32);
        w->x32 = (f2*)take(f32);
    }
    if (kind == WS_BACKWARD) {
        w->y = (d2*)take(f64);
        w->tx = (d2*)take(f64);
        w->sy = (d2*)take(f64);
    }
    if (kind == WS_FULL || kind == WS_TRACE) {
        w->bp = (d2*)take(f64);
        w->fo = (d2*)take(f64);
    }
    if (kind == WS_TRACE) {
        w->ve = (d2*)take(f64);
        w->vo = (d2*)take(f64);
        w->xe = (d2*)take(f64);
        w->xo = (d2*)take(f64);
        w->dot = (double*)take((cdot_scratch_doubles(lat.Vh, n) + 2 * kMaxRhs) * sizeof(double));
    }
    return off;
}

// ---------------------------------------------------------------------------
// Packed link access.
template <typename T>
const cplx<T>* link_block(const void* packed, int Vh, int nk, int parity)
{
    const char* b = reinterpret_cast<const char*>(packed) + kLinkHeaderBytes;
    return reinterpret_cast<const cplx<T>*>(reinterpret_cast<const T*>(b) +
                                            (size_t)parity * link_block_reals(Vh, nk));
}

// cm: colour-major fields (every solver launch); false only for the plain
// Dslash on canonical site-major fields.
hipError_t launch_ds(int epi, int n, int nk, const Tile& t, const DslashArgs<double>& a,
                     hipStream_t s, bool cm = true)
{
    (void)nk;
    return launch_dslash_f64(epi, n, t, a, s, cm);
}

hipError_t launch_ds(int epi, int n, int nk, const Tile& t, const DslashArgs<float>& a,
                     hipStream_t s, bool cm = true)
{
    return launch_dslash_f32(epi, nk, n, t, a, s, cm);
}

bool t_order_ok(const Lat& lat, int G, int bs, int order);

// The tile of a kernel without LDS staging (the p-update, the batched
// kernels): a staged Dslash tile may hold up to kMaxBlockLds threads, more
// than those kernels are built for, so it falls back to 128 threads.
Tile unstaged(const Tile& t)
{
    if (t.rows == 0 && t.bs <= kMaxBlock) return t;
    return Tile{t.nr, 128, t.remap, 0};
}

hipError_t launch_pup(int n, const Tile& t, const PupdateArgs<double>& a, hipStream_t s)
{
    if (pupdate_flat_ok(n)) return launch_pupdate_flat_f64(n, a, s);
    Tile u = unstaged(t);
    if (!t_order_ok(a.lat, n / u.nr, u.bs, u.remap)) u.remap = 1;
    return launch_pupdate_f64(n, u, a, s);
}

hipError_t launch_pup(int n, const Tile& t, const PupdateArgs<float>& a, hipStream_t s)
{
    if (pupdate_flat_ok(n)) return launch_pupdate_flat_f32(n, a, s);
    Tile u = unstaged(t);
    if (!t_order_ok(a.lat, n / u.nr, u.bs, u.remap)) u.remap = 1;
    return launch_pupdate_f32(n, u, a, s);
}

// ---------------------------------------------------------------------------
// Autotuner: times the candidate tiles with the plain Dslash on the caller's
// buffers and caches the fastest per (lattice, nrhs, precision, Naik storage).
std::mutex g_tune_mu;
std::map<std::string, Tile> g_tune_cache;
int g_tune_mode = 0;
int g_force_nr = 0, g_force_bs = 0, g_force_order = 1, g_force_rows = 0;
// mode 1: a tile of its own for the D_eo kernel with the CG epilogue (nr 0: none)
int g_force_eo_nr = 0, g_force_eo_bs = 0, g_force_eo_order = 1, g_force_eo_rows = 0;

// Tile order 2 needs tiles that never straddle a time slice; order 3 needs
// z-chunks of whole planes for each of the 8 XCDs and tiles that divide an x-y
// plane.
bool t_order_ok(const Lat& lat, int G, int bs, int order)
{
    if (order == 2) {
        const long slice_threads = (long)lat.Vh / lat.L[3] * G;
        return slice_threads % bs == 0;
    }
    if (order == 3) {
        const int tile_sites = bs / G;
        const int plane = lat.L[0] * lat.L[1] / 2;
        return bs % G == 0 && lat.L[2] % 8 == 0 && plane % tile_sites == 0;
    }
    return order == 0 || order == 1;
}

// Block size of the LDS-staged Dslash with R x-rows per tile and G lanes per
// site, or 0 where that tile is not possible: whole waves, at most
// kMaxBlockLds threads, tiles that never straddle a plane, staged rows within
// kMaxStageBytes.
int staged_block(const Lat& lat, int n, int G, int R, int prec)
{
    if (R < 1) return 0;
    const long bs = (long)R * lat.Lh0 * G;
    const size_t elt = prec == HISQ_PREC_F64 ? 16 : 8;
    const size_t lds = (size_t)3 * (R + 6) * lat.Lh0 * n * elt;
    if (bs % 64 != 0 || bs > kMaxBlockLds || lat.L[1] % R != 0 || lds > (size_t)kMaxStageBytes)
        return 0;
    return (int)bs;
}

Tile default_tile(int n, int prec)
{
    Tile t{n, 128, 1};
    if (prec == HISQ_PREC_F64 && n > 4) {
        for (int nr = 4; nr >= 1; --nr)
            if (valid_nr(n, nr)) {
                t.nr = nr;
                break;
            }
    }
    return t;
}

std::string tune_key(const Lat& lat, int n, int prec, int naik, int epi, bool cm)
{
    char buf[128];
    snprintf(buf, sizeof(buf), "%dx%dx%dx%d/n%d/p%d/k%d/e%d/c%d", lat.L[0], lat.L[1], lat.L[2],
             lat.L[3], n, prec, naik, epi, cm ? 1 : 0);
    return buf;
}

// epi: EPI_PLAIN times the bare Dslash (hisq_dslash); EPI_NORM times the
// solver's reducing kernel, whose per-work-group reduction cost depends on the
// tile (probe.state/red/cnt must then be valid, counters zero, rhs active).
template <typename T>
int get_tile(const Lat& lat, int n, int prec, int nk, const DslashArgs<T>& probe, hipStream_t s,
             Tile* out, int epi = EPI_PLAIN, bool cm = true)
{
    int mode, fnr, fbs, ford, frows;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        mode = g_tune_mode;
        const bool eo = epi == EPI_CG && g_force_eo_nr > 0;
        fnr = eo ? g_force_eo_nr : g_force_nr;
        fbs = eo ? g_force_eo_bs : g_force_bs;
        ford = eo ? g_force_eo_order : g_force_order;
        frows = eo ? g_force_eo_rows : g_force_rows;
    }
    if (mode == 1 && valid_nr(n, fnr)) {
        const int sbs = cm ? staged_block(lat, n, n / fnr, frows, prec) : 0;
        Tile t{fnr, sbs ? sbs : fbs, ford, sbs ? frows : 0};
        if (!t_order_ok(lat, n / fnr, t.bs, t.remap)) t.remap = 1;
        *out = t;
        return HISQ_OK;
    }
    if (mode != 0) {
        *out = default_tile(n, prec);
        return HISQ_OK;
    }
    const std::string key = tune_key(lat, n, prec, nk, epi, cm);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return HISQ_OK;
        }
    }
    hipEvent_t tev[2] = {nullptr, nullptr};
    auto release = on_scope_exit([&] { destroy_events(tev, 2); });
    HIP_TRY(hipEventCreate(&tev[0]));
    HIP_TRY(hipEventCreate(&tev[1]));
    hipEvent_t e0 = tev[0], e1 = tev[1];
    Tile best = default_tile(n, prec);
    float best_ms = 1e30f;
    // candidates: unstaged tiles of 64, 128, 256 threads, then (colour-major
    // only) LDS-staged tiles of 1..16 rows
    std::vector<Tile> cand;
    for (int G = 1; G <= 8; G *= 2) {
        if (n % G != 0) continue;
        for (int bs : {64, 128, 256}) cand.push_back(Tile{n / G, bs, 0, 0});
        if (cm)
            for (int R = 1; R <= 16; ++R) {
                const int sbs = staged_block(lat, n, G, R, prec);
                if (sbs) cand.push_back(Tile{n / G, sbs, 0, R});
            }
    }
    for (const Tile& base : cand) {
        const int G = n / base.nr;
        for (int remap = 0; remap < 4; ++remap) {
                Tile c = base;
                c.remap = remap;
                if (!t_order_ok(lat, G, c.bs, remap)) continue;
                if (launch_ds(epi, n, nk, c, probe, s, cm) != hipSuccess) continue;
                HIP_TRY(hipEventRecord(e0, s));
                for (int rep = 0; rep < 3; ++rep) HIP_TRY(launch_ds(epi, n, nk, c, probe, s, cm));
                HIP_TRY(hipEventRecord(e1, s));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    *out = best;
    return HISQ_OK;
}

// ---------------------------------------------------------------------------
// Per-thread resources: pinned host copy of the CG state and a capture stream.
struct ThreadRes {
    CgState* host_state = nullptr;
    std::map<int, hipStream_t> capture;
    ~ThreadRes()
    {
        // Process teardown: the runtime may already be gone; release nothing.
    }
};
thread_local ThreadRes g_res;

int host_state(CgState** out)
{
    if (!g_res.host_state) {
        void* p = nullptr;
        HIP_TRY(hipHostMalloc(&p, sizeof(CgState) * HISQ_MAX_PROBLEMS, hipHostMallocDefault));
        g_res.host_state = (CgState*)p;
    }
    *out = g_res.host_state;
    return HISQ_OK;
}

int capture_stream(hipStream_t* out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto it = g_res.capture.find(dev);
    if (it == g_res.capture.end()) {
        hipStream_t s;
        HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        it = g_res.capture.emplace(dev, s).first;
    }
    *out = it->second;
    return HISQ_OK;
}

// ---------------------------------------------------------------------------
// The CG driver.  A solve is a set of problems (one bundle each); with a single
// problem the iteration kernels are specialised for its bundle and tile, with
// several every CG phase is one batched launch over all of them.
struct Prob {
    Lat lat{};
    int n = 0;
    double mass = 0, m4 = 0;
    const void* links64 = nullptr;
    const void* links32 = nullptr;
    const d2* ub = nullptr;  // caller's b and x, site-major [Vh][3][n]
    d2* ux = nullptr;
    const d2* b = nullptr;  // colour-major working copies [3][Vh][n]
    d2* x = nullptr;
    Ws w;
    Tile t64{}, t32{};    // D_oe with |t|^2 (tuned), the p-update, the FP64 residual
    Tile t64e{}, t32e{};  // D_eo with the CG epilogue (tuned on its own)
    int bnr = 0;          // rhs per thread in the batched kernels (tuned with the batch)
    CgState* hs = nullptr;  // pinned host copy
    double bb[kMaxRhs] = {};
    bool fin[kMaxRhs] = {};
    int restarts[kMaxRhs] = {};
    double rr_iter[kMaxRhs] = {};
    int st_final[kMaxRhs] = {};
    size_t ncplx() const { return (size_t)lat.Vh * 3 * n; }
};

struct Engine {
    std::vector<Prob> P;
    hisq_params prm{};
    bool mixed = false;
    int nk = HISQ_NAIK_FULL;  // Naik storage of the FP32 links (MIXED)
    hipStream_t s = nullptr;
    CgState* states = nullptr;  // device, contiguous, one per problem
    void* table = nullptr;      // device BatchTable (several problems)
    int batch_bs = 128, batch_blocks = 0;
    CgState* host_buf = nullptr;  // host copy of the states (NULL: the thread's pinned buffer)
    std::vector<hipEvent_t> ev;
    double kms[HISQ_K_COUNT] = {};
    int klaunch[HISQ_K_COUNT] = {};
    int updates = 0, polls = 0;

    DslashArgs<double> args64(const Prob& q, int parity) const
    {
        DslashArgs<double> a{};
        a.lat = q.lat;
        a.parity = parity;
        a.links = link_block<double>(q.links64, q.lat.Vh, HISQ_NAIK_FULL, parity);
        a.mass4 = q.m4;
        a.state = q.w.st;
        a.red = q.w.red;
        a.cnt = q.w.cnt;
        return a;
    }

    // r64 = b - A x for the selected rhs of q (FP64 links); |r|^2 -> rr_true.
    int true_residual(const Prob& q)
    {
        DslashArgs<double> a = args64(q, 1);
        a.in = q.x;
        a.out = q.w.t64;
        HIP_TRY(launch_ds(EPI_PLAIN, q.n, HISQ_NAIK_FULL, q.t64, a, s));
        DslashArgs<double> c = args64(q, 0);
        c.in = q.w.t64;
        c.out = q.w.r64;
        c.b = q.b;
        c.xh = q.x;
        HIP_TRY(launch_ds(EPI_RESID, q.n, HISQ_NAIK_FULL, q.t64, c, s));
        return HISQ_OK;
    }

    template <typename T>
    void iter_args(const Prob& q, PupdateArgs<T>& k1, DslashArgs<T>& k2, DslashArgs<T>& k3) const
    {
        const void* L = std::is_same<T, float>::value ? q.links32 : q.links64;
        const int rr = std::is_same<T, float>::value ? nk : HISQ_NAIK_FULL;
        cplx<T>* r;
        cplx<T>* p;
        cplx<T>* t;
        cplx<T>* x;
        if constexpr (std::is_same<T, float>::value) {
            r = q.w.r32;
            p = q.w.p32;
            t = q.w.t32;
            x = q.w.x32;
        } else {
            r = q.w.r64;
            p = q.w.p64;
            t = q.w.t64;
            x = q.x;
        }
        const Tile& tile = std::is_same<T, float>::value ? q.t32 : q.t64;
        k1 = PupdateArgs<T>{};
        k1.lat = q.lat;
        k1.r = r;
        k1.p = p;
        k1.state = q.w.st;
        k1.red = q.w.red;
        k1.cnt = q.w.cnt;
        k1.remap = tile.remap;
        k2 = DslashArgs<T>{};
        k2.lat = q.lat;
        k2.parity = 1;
        k2.links = link_block<T>(L, q.lat.Vh, rr, 1);
        k2.naik_scale = naik_scale_of(L);
        k2.in = p;
        k2.out = t;
        k2.mass4 = q.m4;
        k2.state = q.w.st;
        k2.red = q.w.red;
        k2.cnt = q.w.cnt;
        k2.remap = tile.remap;
        k3 = k2;
        k3.parity = 0;
        k3.links = link_block<T>(L, q.lat.Vh, rr, 0);
        k3.in = t;
        k3.out = nullptr;
        k3.p = p;
        k3.x = x;
        k3.r = r;
    }

    template <typename T>
    int emit_single(hipStream_t st, hipEvent_t* evs)
    {
        const Prob& q = P[0];
        PupdateArgs<T> k1;
        DslashArgs<T> k2, k3;
        iter_args<T>(q, k1, k2, k3);
        const Tile& tile = std::is_same<T, float>::value ? q.t32 : q.t64;
        const Tile& tile_e = std::is_same<T, float>::value ? q.t32e : q.t64e;
        const int rr = std::is_same<T, float>::value ? nk : HISQ_NAIK_FULL;
        if (evs) HIP_TRY(hipEventRecord(evs[0], st));
        HIP_TRY(launch_pup(q.n, tile, k1, st));
        if (evs) HIP_TRY(hipEventRecord(evs[1], st));
        HIP_TRY(launch_ds(EPI_NORM, q.n, rr, tile, k2, st));
        if (evs) HIP_TRY(hipEventRecord(evs[2], st));
        HIP_TRY(launch_ds(EPI_CG, q.n, rr, tile_e, k3, st));
        if (evs) HIP_TRY(hipEventRecord(evs[3], st));
        return HISQ_OK;
    }

    template <typename T>
    int emit_batched(hipStream_t st, hipEvent_t* evs)
    {
        const BatchTable<T>* tab = reinterpret_cast<const BatchTable<T>*>(table);
        if (evs) HIP_TRY(hipEventRecord(evs[0], st));
        if constexpr (std::is_same<T, float>::value) {
            HIP_TRY(launch_pupdate_batched_f32(tab, batch_blocks, batch_bs, st));
            if (evs) HIP_TRY(hipEventRecord(evs[1], st));
            HIP_TRY(launch_dslash_batched_f32(EPI_NORM, nk, tab, batch_blocks, batch_bs, st));
            if (evs) HIP_TRY(hipEventRecord(evs[2], st));
            HIP_TRY(launch_dslash_batched_f32(EPI_CG, nk, tab, batch_blocks, batch_bs, st));
        } else {
            HIP_TRY(launch_pupdate_batched_f64(tab, batch_blocks, batch_bs, st));
            if (evs) HIP_TRY(hipEventRecord(evs[1], st));
            HIP_TRY(launch_dslash_batched_f64(EPI_NORM, tab, batch_blocks, batch_bs, st));
            if (evs) HIP_TRY(hipEventRecord(evs[2], st));
            HIP_TRY(launch_dslash_batched_f64(EPI_CG, tab, batch_blocks, batch_bs, st));
        }
        if (evs) HIP_TRY(hipEventRecord(evs[3], st));
        return HISQ_OK;
    }

    int emit_block(hipStream_t st, int iters, bool with_events)
    {
        for (int j = 0; j < iters; ++j) {
            hipEvent_t* evs = with_events ? &ev[4 * j] : nullptr;
            int rc;
            if (P.size() == 1)
                rc = mixed ? emit_single<float>(st, evs) : emit_single<double>(st, evs);
            else
                rc = mixed ? emit_batched<float>(st, evs) : emit_batched<double>(st, evs);
            if (rc) return rc;
        }
        return HISQ_OK;
    }

    // Batch table over the problems `which` (all if empty), each with its own
    // rhs tile bnr, for work-groups of bs threads; uploads it and sets
    // batch_blocks.
    template <typename T>
    int upload_table(void* host_buf, const std::vector<int>& which, int bs)
    {
        BatchTable<T>* tab = reinterpret_cast<BatchTable<T>*>(host_buf);
        std::memset(tab, 0, sizeof(*tab));
        int start = 0;
        const int np = which.empty() ? (int)P.size() : (int)which.size();
        for (int jj = 0; jj < np; ++jj) {
            const Prob& q = P[which.empty() ? jj : which[jj]];
            BatchProb<T>& bp = tab->p[jj];
            iter_args<T>(q, bp.k1, bp.k2, bp.k3);
            bp.n = q.n;
            bp.nr = batched_nr_ok(q.n, q.bnr) ? q.bnr : q.n;
            // XCD-owned z-chunks where the problem's tiles allow, else one
            // contiguous slab per XCD
            const int G = q.n / bp.nr;
            bp.k1.remap = bp.k2.remap = bp.k3.remap = t_order_ok(q.lat, G, bs, 3) ? 3 : 1;
            const long threads = (long)q.lat.Vh * G;
            bp.nblocks = (int)((threads + bs - 1) / bs);
            bp.k1.ntiles = bp.k2.ntiles = bp.k3.ntiles = bp.nblocks;
            bp.block_start = start;
            start += bp.nblocks;
        }
        tab->nprob = np;
        tab->total_blocks = start;
        batch_blocks = start;
        batch_bs = bs;
        HIP_TRY(hipMemcpyAsync(table, tab, sizeof(BatchTable<T>), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return HISQ_OK;
    }

    // The batched autotuner: the rhs tile of every problem and the work-group
    // size of the batched launches, timed on the problems' own buffers with the
    // CG state frozen (every rhs active, alpha = 0: x and r keep their values;
    // setup() initialises everything afterwards).  Each problem's tile is timed
    // in a batch of its own, then the block size for the whole batch.  The
    // timed unit is one D_oe (|t|^2) plus one D_eo (CG epilogue) launch.
    template <typename T>
    int tune_batched(void* host_buf);

    int read_states(CgState* host)
    {
        HIP_TRY(hipMemcpyAsync(host, states, sizeof(CgState) * P.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return HISQ_OK;
    }

    int write_states(CgState* host)
    {
        HIP_TRY(hipMemcpyAsync(states, host, sizeof(CgState) * P.size(), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return HISQ_OK;
    }

    int poll_block_size() const
    {
        if (prm.poll_every > 0) return prm.poll_every;
        double bytes = 0;
        for (const Prob& q : P)
            bytes += (double)q.lat.Vh * (mixed ? (2304.0 + 264.0 * q.n) : (4608.0 + 528.0 * q.n));
        const double est = bytes / 4.0e12 + 3 * 4.0e-6;
        const int k = (int)std::ceil(2.0e-3 / est);
        return std::max(4, std::min(64, k));
    }

    int collect_events(int iters)
    {
        for (int j = 0; j < iters; ++j)
            for (int c = 0; c < 3; ++c) {
                float ms = 0;
                HIP_TRY(hipEventElapsedTime(&ms, ev[4 * j + c], ev[4 * j + c + 1]));
                kms[c] += ms;
                klaunch[c] += 1;
            }
        return HISQ_OK;
    }

    int batched_time(void* host_buf, const std::vector<int>& which, int bs, float* ms);
    int setup(CgState* host);
    int poll_and_update(CgState* host);
    int finish(CgState* host, hisq_info* infos, double seconds);
    int run(hisq_info* infos);
};

// Mean time of one D_oe + one D_eo batched launch over the problems `which`
// (states armed and frozen by the caller), work-groups of bs threads.
int Engine::batched_time(void* host_buf, const std::vector<int>& which, int bs, float* ms)
{
    int rc = mixed ? upload_table<float>(host_buf, which, bs) : upload_table<double>(host_buf, which, bs);
    if (rc) return rc;
    hipEvent_t tev[2] = {nullptr, nullptr};
    auto release = on_scope_exit([&] { destroy_events(tev, 2); });
    HIP_TRY(hipEventCreate(&tev[0]));
    HIP_TRY(hipEventCreate(&tev[1]));
    hipEvent_t e0 = tev[0], e1 = tev[1];
    auto pair = [&]() -> int {
        if (mixed) {
            const auto* tab = reinterpret_cast<const BatchTable<float>*>(table);
            HIP_TRY(launch_dslash_batched_f32(EPI_NORM, nk, tab, batch_blocks, bs, s));
            HIP_TRY(launch_dslash_batched_f32(EPI_CG, nk, tab, batch_blocks, bs, s));
        } else {
            const auto* tab = reinterpret_cast<const BatchTable<double>*>(table);
            HIP_TRY(launch_dslash_batched_f64(EPI_NORM, tab, batch_blocks, bs, s));
            HIP_TRY(launch_dslash_batched_f64(EPI_CG, tab, batch_blocks, bs, s));
        }
        return HISQ_OK;
    };
    constexpr int kReps = 3;
    if ((rc = pair())) return rc;
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < kReps; ++r)
        if ((rc = pair())) return rc;
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = t / kReps;
    return HISQ_OK;
}

std::map<std::string, std::pair<std::vector<int>, int>> g_batch_cache;  // key -> (tiles, block)

template <typename T>
int Engine::tune_batched(void* host_buf)
{
    std::string key = std::string("B/p") + (mixed ? "1" : "0") + "/k" + std::to_string(nk);
    for (const Prob& q : P) {
        char buf[64];
        snprintf(buf, sizeof(buf), "/%dx%dx%dx%d:%d", q.lat.L[0], q.lat.L[1], q.lat.L[2], q.lat.L[3],
                 q.n);
        key += buf;
    }
    int mode;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        mode = g_tune_mode;
        auto it = g_batch_cache.find(key);
        if (mode == 0 && it != g_batch_cache.end()) {
            for (size_t j = 0; j < P.size(); ++j) P[j].bnr = it->second.first[j];
            batch_bs = it->second.second;
            return HISQ_OK;
        }
    }
    if (mode != 0) {
        // fixed tiles (tuning modes 1 and 2): every rhs of a site in one thread
        for (Prob& q : P) q.bnr = q.n;
        batch_bs = 128;
        return HISQ_OK;
    }
    int rc;
    for (Prob& q : P) {
        HIP_TRY(launch_zero(q.w.cnt, q.w.cnt_bytes, s));
        HIP_TRY(launch_state_reset(q.w.st, q.n, 1, s));
    }
    const int sizes[3] = {64, 128, 256};
    for (size_t j = 0; j < P.size(); ++j) {
        Prob& q = P[j];
        int best_nr = q.n;
        float best = 1e30f;
        for (int nr : {q.n, q.n / 2}) {
            if (nr < 1 || !batched_nr_ok(q.n, nr)) continue;
            q.bnr = nr;
            for (int bs : sizes) {
                float ms;
                if ((rc = batched_time(host_buf, {(int)j}, bs, &ms))) return rc;
                if (ms < best) {
                    best = ms;
                    best_nr = nr;
                }
            }
        }
        q.bnr = best_nr;
    }
    float best = 1e30f;
    int best_bs = 128;
    for (int bs : sizes) {
        float ms;
        if ((rc = batched_time(host_buf, {}, bs, &ms))) return rc;
        if (ms < best) {
            best = ms;
            best_bs = bs;
        }
    }
    batch_bs = best_bs;
    std::vector<int> tiles;
    for (const Prob& q : P) tiles.push_back(q.bnr);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_batch_cache[key] = {tiles, batch_bs};
    return HISQ_OK;
}

int Engine::setup(CgState* host)
{
    int rc;
    for (Prob& q : P) {
        const size_t nc = q.ncplx();
        HIP_TRY(launch_zero(q.w.cnt, q.w.cnt_bytes, s));
        HIP_TRY(launch_state_reset(q.w.st, q.n, 0, s));
        HIP_TRY(launch_layout(q.ub, q.w.bc, q.lat.Vh, q.n, true, s));
        if (prm.use_x0)
            HIP_TRY(launch_layout(q.ux, q.w.xc, q.lat.Vh, q.n, true, s));
        else
            HIP_TRY(launch_zero(q.x, nc * sizeof(d2), s));
        HIP_TRY(launch_norm2_f64(q.b, q.lat.Vh, q.n, q.w.st->aux, q.w.red, q.w.cnt, s));
        if ((rc = true_residual(q))) return rc;
        if (mixed) {
            HIP_TRY(launch_to_f32_sel(q.w.r64, q.w.r32, nc, q.n, q.w.st, s));
            HIP_TRY(launch_zero(q.w.x32, nc * sizeof(f2), s));
            HIP_TRY(launch_zero(q.w.p32, nc * sizeof(f2), s));
        } else {
            HIP_TRY(launch_zero(q.w.p64, nc * sizeof(d2), s));
        }
    }
    if ((rc = read_states(host))) return rc;
    const double tol2 = prm.tol * prm.tol;
    bool any_zero_b = false;
    for (size_t j = 0; j < P.size(); ++j) {
        Prob& q = P[j];
        CgState* h = &host[j];
        q.hs = h;
        for (int k = 0; k < q.n; ++k) {
            q.bb[k] = h->aux[k];
            h->thresh[k] = tol2 * q.bb[k];
            h->rr[k] = h->rr_true[k];
            h->rrmax[k] = h->rr[k];
            h->beta[k] = 0.0;
            h->iters[k] = 0;
            h->status[k] = HISQ_OK;
            q.restarts[k] = 0;
            q.fin[k] = !(h->rr[k] > h->thresh[k]) || prm.maxiter == 0;
            h->active[k] = q.fin[k] ? 0 : 1;
            h->sel[k] = q.bb[k] == 0.0 ? 1 : 0;
            any_zero_b = any_zero_b || q.bb[k] == 0.0;
        }
        h->maxiter = prm.maxiter;
    }
    if ((rc = write_states(host))) return rc;
    if (any_zero_b) {
        // b_k = 0: the solution is exactly 0, whatever the start vector
        for (Prob& q : P) HIP_TRY(launch_zero_sel(q.x, q.ncplx(), q.n, q.w.st, s));
        for (size_t j = 0; j < P.size(); ++j)
            for (int k = 0; k < P[j].n; ++k) {
                host[j].sel[k] = 0;
                if (P[j].bb[k] == 0.0) {
                    P[j].fin[k] = true;
                    host[j].active[k] = 0;
                }
            }
        if ((rc = write_states(host))) return rc;
    }
    return HISQ_OK;
}

// After a poll: choose the rhs that need a true-residual pass, run it, and
// decide convergence, restarts and reliable updates.
int Engine::poll_and_update(CgState* host)
{
    int rc;
    bool any = false;
    for (Prob& q : P) {
        CgState* h = q.hs;
        bool any_q = false;
        for (int k = 0; k < q.n; ++k) {
            h->sel[k] = 0;
            if (q.fin[k]) continue;
            if (h->status[k] == HISQ_BREAKDOWN) {
                if (mixed && q.restarts[k] < 3) {
                    h->sel[k] = 1;  // recover: reliable update, restart with p = r
                } else {
                    q.fin[k] = true;
                    continue;
                }
            } else if (!h->active[k]) {
                h->sel[k] = 1;  // iterated residual passed (or maxiter): check the true one
            } else if (mixed && h->rr[k] < prm.delta * prm.delta * h->rrmax[k]) {
                h->sel[k] = 1;  // reliable update
            }
            any_q = any_q || h->sel[k];
        }
        if (any_q && mixed) {
            // one FP64 pass serves the whole bundle: update every running rhs
            for (int k = 0; k < q.n; ++k)
                if (!q.fin[k]) h->sel[k] = 1;
        }
        any = any || any_q;
    }
    if (!any) return HISQ_OK;
    if ((rc = write_states(host))) return rc;
    hipEvent_t tev[2] = {nullptr, nullptr};
    auto release = on_scope_exit([&] { destroy_events(tev, 2); });
    if (prm.profile) {
        HIP_TRY(hipEventCreate(&tev[0]));
        HIP_TRY(hipEventCreate(&tev[1]));
        HIP_TRY(hipEventRecord(tev[0], s));
    }
    hipEvent_t e0 = tev[0], e1 = tev[1];
    for (Prob& q : P) {
        bool any_q = false;
        for (int k = 0; k < q.n; ++k) any_q = any_q || q.hs->sel[k];
        if (!any_q) continue;
        if (mixed) HIP_TRY(launch_accum_sel(q.x, q.w.x32, q.ncplx(), q.n, q.w.st, s));
        if ((rc = true_residual(q))) return rc;
        if (mixed) HIP_TRY(launch_to_f32_sel(q.w.r64, q.w.r32, q.ncplx(), q.n, q.w.st, s));
    }
    if (prm.profile) HIP_TRY(hipEventRecord(e1, s));
    ++updates;
    if ((rc = read_states(host))) return rc;
    if (prm.profile) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        kms[HISQ_K_RELIABLE] += ms;
        klaunch[HISQ_K_RELIABLE] += 1;
    }
    for (Prob& q : P) {
        CgState* h = q.hs;
        for (int k = 0; k < q.n; ++k) {
            if (!h->sel[k]) continue;
            const double rt = h->rr_true[k];
            if (rt <= h->thresh[k] && h->status[k] != HISQ_BREAKDOWN) {
                q.fin[k] = true;
                h->active[k] = 0;
                h->status[k] = HISQ_OK;
                continue;
            }
            if (h->iters[k] >= prm.maxiter) {
                q.fin[k] = true;
                h->active[k] = 0;
                h->status[k] = HISQ_NOT_CONVERGED;
                continue;
            }
            if (h->status[k] == HISQ_BREAKDOWN) {
                q.restarts[k] += 1;
                h->status[k] = HISQ_OK;
                h->beta[k] = 0.0;  // restart: p = r
            } else if (!mixed || !h->active[k]) {
                h->beta[k] = 0.0;  // restart from the true residual
            }
            h->rr[k] = rt;
            h->rrmax[k] = rt;
            h->active[k] = 1;
        }
        for (int k = 0; k < q.n; ++k) h->sel[k] = 0;
    }
    return write_states(host);
}

int Engine::finish(CgState* host, hisq_info* infos, double seconds)
{
    int rc;
    for (size_t j = 0; j < P.size(); ++j) {
        Prob& q = P[j];
        for (int k = 0; k < q.n; ++k) {
            q.st_final[k] = host[j].status[k];
            q.rr_iter[k] = host[j].rr[k];
            host[j].sel[k] = 1;
        }
    }
    if ((rc = write_states(host))) return rc;
    for (Prob& q : P) {
        if (mixed) HIP_TRY(launch_accum_sel(q.x, q.w.x32, q.ncplx(), q.n, q.w.st, s));
        if ((rc = true_residual(q))) return rc;
        HIP_TRY(launch_layout(q.x, q.ux, q.lat.Vh, q.n, false, s));
    }
    if ((rc = read_states(host))) return rc;
    int worst = HISQ_OK;
    for (size_t j = 0; j < P.size(); ++j) {
        Prob& q = P[j];
        hisq_info* info = infos ? &infos[j] : nullptr;
        if (info) {
            std::memset(info, 0, sizeof(*info));
            const Tile& t = mixed ? q.t32 : q.t64;
            const Tile& te = mixed ? q.t32e : q.t64e;
            info->block_size = P.size() == 1 ? t.bs : batch_bs;
            info->rhs_per_thread = P.size() == 1 ? t.nr : q.bnr;
            info->tile_order = P.size() == 1 ? t.remap : 0;
            info->stage_rows = P.size() == 1 ? t.rows : 0;
            info->eo_block_size = P.size() == 1 ? te.bs : batch_bs;
            info->eo_rhs_per_thread = P.size() == 1 ? te.nr : q.bnr;
            info->eo_tile_order = P.size() == 1 ? te.remap : 0;
            info->eo_stage_rows = P.size() == 1 ? te.rows : 0;
        }
        int maxit = 0;
        for (int k = 0; k < q.n; ++k) {
            int stk = q.st_final[k];
            // |b| = 0 gives x = 0 exactly; a non-finite |b| can never converge
            const double rel = q.bb[k] > 0 ? std::sqrt(host[j].rr_true[k] / q.bb[k])
                                           : (q.bb[k] == 0.0 ? 0.0 : NAN);
            if (stk == HISQ_OK && !(rel <= prm.tol)) stk = HISQ_NOT_CONVERGED;
            worst = std::max(worst, stk);
            maxit = std::max(maxit, host[j].iters[k]);
            if (info) {
                info->iters[k] = host[j].iters[k];
                info->status[k] = stk;
                info->rel_true_res[k] = rel;
                info->rel_iter_res[k] =
                    q.bb[k] > 0 ? std::sqrt(std::max(0.0, q.rr_iter[k]) / q.bb[k]) : 0.0;
            }
        }
        if (info) {
            info->reliable_updates = updates;
            info->polls = polls;
            info->total_iters = maxit;
            info->seconds = seconds;
            for (int c = 0; c < HISQ_K_COUNT; ++c) {
                info->kernel_ms[c] = kms[c];
                info->kernel_launches[c] = klaunch[c];
            }
        }
    }
    return worst;
}

int Engine::run(hisq_info* infos)
{
    const auto t_start = std::chrono::steady_clock::now();
    int rc;
    CgState* host = host_buf;
    if (!host && (rc = host_state(&host))) return rc;

    // tiles (autotuned per problem on the reducing D_oe kernel; the state and
    // counters are armed for it here and reset again by setup())
    for (Prob& q : P) {
        HIP_TRY(launch_zero(q.w.cnt, q.w.cnt_bytes, s));
        HIP_TRY(launch_state_reset(q.w.st, q.n, 1, s));
        DslashArgs<double> probe = args64(q, 1);
        probe.in = q.x;
        probe.out = q.w.t64;
        if ((rc = get_tile(q.lat, q.n, HISQ_PREC_F64, HISQ_NAIK_FULL, probe, s, &q.t64, EPI_NORM))) return rc;
        if (mixed && P.size() == 1) {
            DslashArgs<float> p32{};
            p32.lat = q.lat;
            p32.parity = 1;
            p32.links = link_block<float>(q.links32, q.lat.Vh, nk, 1);
            p32.naik_scale = naik_scale_of(q.links32);
            p32.in = q.w.p32;
            p32.out = q.w.t32;
            p32.mass4 = q.m4;
            p32.state = q.w.st;
            p32.red = q.w.red;
            p32.cnt = q.w.cnt;
            if ((rc = get_tile(q.lat, q.n, HISQ_PREC_F32, nk, p32, s, &q.t32, EPI_NORM))) return rc;
        }
        // the D_eo kernel with the CG epilogue, timed on the iteration's own
        // buffers with the state re-armed (frozen, every rhs active, alpha = 0:
        // x and r keep their values, and setup() initialises them afterwards)
        q.t64e = q.t64;
        q.t32e = q.t32;
        if (P.size() == 1) {
            HIP_TRY(launch_zero(q.w.cnt, q.w.cnt_bytes, s));
            HIP_TRY(launch_state_reset(q.w.st, q.n, 1, s));
            if (mixed) {
                PupdateArgs<float> k1;
                DslashArgs<float> k2, k3;
                iter_args<float>(q, k1, k2, k3);
                if ((rc = get_tile(q.lat, q.n, HISQ_PREC_F32, nk, k3, s, &q.t32e, EPI_CG))) return rc;
            } else {
                PupdateArgs<double> k1;
                DslashArgs<double> k2, k3;
                iter_args<double>(q, k1, k2, k3);
                if ((rc = get_tile(q.lat, q.n, HISQ_PREC_F64, HISQ_NAIK_FULL, k3, s, &q.t64e, EPI_CG)))
                    return rc;
            }
        }
    }
    if (P.size() > 1) {
        static thread_local std::vector<char> tabbuf;
        tabbuf.resize(std::max(sizeof(BatchTable<double>), sizeof(BatchTable<float>)));
        rc = mixed ? tune_batched<float>(tabbuf.data()) : tune_batched<double>(tabbuf.data());
        if (rc) return rc;
        if ((rc = setup(host))) return rc;
        rc = mixed ? upload_table<float>(tabbuf.data(), {}, batch_bs)
                   : upload_table<double>(tabbuf.data(), {}, batch_bs);
        if (rc) return rc;
    } else if ((rc = setup(host))) {
        return rc;
    }

    const int kblk = poll_block_size();
    const bool profile = prm.profile != 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto release = on_scope_exit([&] {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        destroy_events(ev.data(), ev.size());
        ev.clear();
    });
    if (profile) {
        ev.assign(4 * kblk, nullptr);
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    }
    // Event timestamps are not available for events recorded inside a graph, so
    // a profiled solve launches its kernels directly on the stream.
    if (prm.use_graph && !profile) {
        hipStream_t cap;
        if ((rc = capture_stream(&cap))) return rc;
        HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
        rc = emit_block(cap, kblk, profile);
        const hipError_t ce = hipStreamEndCapture(cap, &graph);
        if (rc) return rc;
        HIP_TRY(ce);
        HIP_TRY(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    auto running = [&]() {
        for (const Prob& q : P)
            for (int k = 0; k < q.n; ++k)
                if (!q.fin[k]) return true;
        return false;
    };
    while (running()) {
        if (exec) {
            HIP_TRY(hipGraphLaunch(exec, s));
        } else if ((rc = emit_block(s, kblk, profile))) {
            return rc;
        }
        if ((rc = read_states(host))) return rc;
        ++polls;
        if (profile && (rc = collect_events(kblk))) return rc;
        if ((rc = poll_and_update(host))) return rc;
    }
    const double secs =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    return finish(host, infos, secs);
}

int check_params(const hisq_params* p, int n)
{
    if (!p) return fail(HISQ_EINVAL, "params is NULL");
    if (n < 1 || n > HISQ_MAX_RHS) return fail(HISQ_EINVAL, "nrhs = %d outside 1..8", n);
    if (p->mode != HISQ_MODE_FP64 && p->mode != HISQ_MODE_MIXED)
        return fail(HISQ_EINVAL, "unknown mode %d", p->mode);
    if (!valid_naik(p->naik))
        return fail(HISQ_EINVAL, "unknown naik storage %d", p->naik);
    if (!(p->tol > 0) || !std::isfinite(p->tol)) return fail(HISQ_EINVAL, "tol must be > 0");
    if (p->maxiter < 0) return fail(HISQ_EINVAL, "maxiter must be >= 0");
    if (p->mode == HISQ_MODE_MIXED && !(p->delta > 0 && p->delta < 1))
        return fail(HISQ_EINVAL, "delta must be in (0, 1)");
    if (p->poll_every < 0) return fail(HISQ_EINVAL, "poll_every must be >= 0");
    return HISQ_OK;
}

int solve_impl(double mass, int nrhs, const hisq_params* p, const void* links64,
               const void* links32, const double* b_e, double* x_e, const Ws& w, hisq_info* info,
               void* stream, const Lat& lat, CgState* host_buf = nullptr)
{
    Engine E;
    E.host_buf = host_buf;
    E.prm = *p;
    E.mixed = p->mode == HISQ_MODE_MIXED;
    E.nk = E.mixed ? p->naik : HISQ_NAIK_FULL;
    E.s = reinterpret_cast<hipStream_t>(stream);
    Prob q;
    q.lat = lat;
    q.n = nrhs;
    q.mass = mass;
    q.m4 = 4.0 * mass * mass;
    q.links64 = links64;
    q.links32 = links32;
    q.ub = reinterpret_cast<const d2*>(b_e);
    q.ux = reinterpret_cast<d2*>(x_e);
    q.b = w.bc;
    q.x = w.xc;
    q.w = w;
    E.states = w.st;
    E.P.push_back(q);
    return E.run(info);
}

// x = M^{-1} b on the full lattice, M = 2m + D, through the even-odd
// reduction: (4m^2 - D_eo D_oe) x_e = 2m b_e - D_eo b_o, then
// x_o = (b_o - D_oe x_e) / (2m).  Caller's site-major FP64 fields.
int full_impl(double mass, int n, const hisq_params* p, const void* links64, const void* links32,
              const d2* b_e, const d2* b_o, d2* x_e, d2* x_o, const Ws& w, hisq_info* info,
              hipStream_t s, const Lat& lat)
{
    const size_t nc = (size_t)lat.Vh * 3 * n;
    const Tile t = default_tile(n, HISQ_PREC_F64);
    DslashArgs<double> a{};
    a.lat = lat;
    a.parity = 0;
    a.links = link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, 0);
    a.in = b_o;
    a.out = w.fo;
    HIP_TRY(launch_ds(EPI_PLAIN, n, HISQ_NAIK_FULL, t, a, s, false));
    HIP_TRY(launch_axpby(b_e, w.fo, w.bp, nc, 2.0 * mass, -1.0, s));
    hisq_params q = *p;
    q.use_x0 = 0;
    const int st = solve_impl(mass, n, &q, links64, links32, reinterpret_cast<const double*>(w.bp),
                              reinterpret_cast<double*>(x_e), w, info, s, lat);
    if (st < 0) return st;
    a.parity = 1;
    a.links = link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, 1);
    a.in = x_e;
    a.out = w.fo;
    HIP_TRY(launch_ds(EPI_PLAIN, n, HISQ_NAIK_FULL, t, a, s, false));
    HIP_TRY(launch_axpby(b_o, w.fo, x_o, nc, 1.0 / (2.0 * mass), -1.0 / (2.0 * mass), s));
    return st;
}

// (y_e, y_o) = d^nder M / d mu^nder (x_e, x_o) at mu = 0; nder = 0 is M itself.
int apply_dM(double mass, int n, int nder, const void* links64, const d2* x_e, const d2* x_o,
             d2* y_e, d2* y_o, const Ws& w, hipStream_t s, const Lat& lat)
{
    const size_t nc = (size_t)lat.Vh * 3 * n;
    if (nder > 0) {
        HIP_TRY(launch_dslash_dmu(lat, 0, n, nder, link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, 0), x_o,
                                  y_e, s));
        HIP_TRY(launch_dslash_dmu(lat, 1, n, nder, link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, 1), x_e,
                                  y_o, s));
        return HISQ_OK;
    }
    const Tile t = default_tile(n, HISQ_PREC_F64);
    DslashArgs<double> a{};
    a.lat = lat;
    for (int par = 0; par < 2; ++par) {
        a.parity = par;
        a.links = link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, par);
        a.in = par == 0 ? x_o : x_e;
        a.out = w.fo;
        HIP_TRY(launch_ds(EPI_PLAIN, n, HISQ_NAIK_FULL, t, a, s, false));
        HIP_TRY(launch_axpby(par == 0 ? x_e : x_o, w.fo, par == 0 ? y_e : y_o, nc, 2.0 * mass, 1.0, s));
    }
    return HISQ_OK;
}

// Per-vector terms of the trace estimator of eq. (2): for orders (n_1..n_j),
// v = eta, then for i = j..1: v = M^-1 v, v = M^(n_i) v; est_k = eta_k^dag v_k.
int trace_impl(double mass, int n, const hisq_params* p, const void* links64, const void* links32,
               int nins, const int* orders, const d2* eta_e, const d2* eta_o, double* est,
               const Ws& w, hisq_info* info, hipStream_t s, const Lat& lat)
{
    const d2* ve = eta_e;
    const d2* vo = eta_o;
    int worst = HISQ_OK, total_iters = 0, updates = 0;
    double secs = 0.0;
    for (int j = nins - 1; j >= 0; --j) {
        const int st = full_impl(mass, n, p, links64, links32, ve, vo, w.xe, w.xo, w, info, s, lat);
        if (st < 0) return st;
        worst = std::max(worst, st);
        if (info) {
            total_iters += info->total_iters;
            updates += info->reliable_updates;
            secs += info->seconds;
        }
        int rc = apply_dM(mass, n, orders[j], links64, w.xe, w.xo, w.ve, w.vo, w, s, lat);
        if (rc) return rc;
        ve = w.ve;
        vo = w.vo;
    }
    HIP_TRY(launch_cdot(eta_e, w.ve, eta_o, w.vo, lat.Vh, n, w.dot, est, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (info) {
        info->total_iters = total_iters;
        info->reliable_updates = updates;
        info->seconds = secs;
    }
    return worst;
}

// Batched workspace: the states of all problems side by side, the batch
// table, then each problem's own regions.
size_t batched_layout(int nprob, const hisq_problem* probs, int mode, char* base,
                      std::vector<Ws>* ws, CgState** states, void** table)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        const size_t o = off;
        off = align256(off + bytes);
        return base ? base + o : nullptr;
    };
    *states = (CgState*)take(sizeof(CgState) * nprob);
    *table = take(std::max(sizeof(BatchTable<double>), sizeof(BatchTable<float>)));
    ws->assign(nprob, Ws());
    for (int j = 0; j < nprob; ++j) {
        const Lat lat = make_lat(probs[j].geom);
        Ws w;
        const size_t need = ws_layout(lat, probs[j].nrhs, mode, WS_SOLVE, nullptr, &w);
        char* region = take(need);
        ws_layout(lat, probs[j].nrhs, mode, WS_SOLVE, region, &w);
        w.st = base ? *states + j : nullptr;
        (*ws)[j] = w;
    }
    return off;
}

int check_problems(int nprob, const hisq_problem* probs, int mode)
{
    if (nprob < 1 || nprob > HISQ_MAX_PROBLEMS)
        return fail(HISQ_EINVAL, "nprob = %d outside 1..%d", nprob, HISQ_MAX_PROBLEMS);
    if (!probs) return fail(HISQ_EINVAL, "problems is NULL");
    for (int j = 0; j < nprob; ++j) {
        Lat lat;
        int rc = check_geom(&probs[j].geom, &lat);
        if (rc) return rc;
        if (probs[j].nrhs < 1 || probs[j].nrhs > HISQ_MAX_RHS)
            return fail(HISQ_EINVAL, "problem %d: nrhs = %d outside 1..8", j, probs[j].nrhs);
        if (!probs[j].links64 || !probs[j].b || !probs[j].x)
            return fail(HISQ_EINVAL, "problem %d: NULL pointer", j);
        if (misaligned({probs[j].links64, probs[j].links32, probs[j].b, probs[j].x}))
            return fail(HISQ_EINVAL, "problem %d: device buffers must be 16-byte aligned", j);
        if (mode == HISQ_MODE_MIXED && !probs[j].links32)
            return fail(HISQ_EINVAL, "problem %d: MIXED mode needs FP32 links", j);
        if (!std::isfinite(probs[j].mass)) return fail(HISQ_EINVAL, "problem %d: bad mass", j);
    }
    return HISQ_OK;
}

}  // namespace

// The body of hisq_cg_solve: argument and link checks, then the solve over the
// workspace `ws`; host_buf (nullable) receives the host copies of the CG state
// instead of the calling thread's pinned buffer.
int hisq::cg_solve_on(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                      const void* links64, const void* links32, const double* b_e, double* x_e,
                      void* ws, size_t ws_bytes, hisq_info* info, void* stream, CgState* host_buf)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_geom(g, &lat);
    if (rc) return rc;
    if ((rc = check_params(p, nrhs))) return rc;
    if (!links64 || !b_e || !x_e || !ws) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(links64, links32, b_e, x_e, ws);
    if (p->mode == HISQ_MODE_MIXED && !links32)
        return fail(HISQ_EINVAL, "MIXED mode needs FP32 links");
    if (!std::isfinite(mass)) return fail(HISQ_EINVAL, "mass must be finite");
    Ws w;
    const size_t need = ws_layout(lat, nrhs, p->mode, WS_SOLVE, nullptr, &w);
    if (ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if ((rc = check_solve_links(links64, links32, lat, p->mode, p->naik,
                                reinterpret_cast<hipStream_t>(stream))))
        return rc;
    ws_layout(lat, nrhs, p->mode, WS_SOLVE, reinterpret_cast<char*>(ws), &w);
    return solve_impl(mass, nrhs, p, links64, links32, b_e, x_e, w, info, stream, lat, host_buf);
}

int hisq::report_error(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

size_t hisq::cg_workspace_bytes(const Lat& lat, int nrhs, int mode)
{
    Ws w;
    return ws_layout(lat, nrhs, mode, WS_SOLVE, nullptr, &w);
}

// ===========================================================================
// C ABI
extern "C" {

void hisq_default_params(hisq_params* p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->mode = HISQ_MODE_FP64;
    p->naik = HISQ_NAIK_FULL;
    p->tol = 1e-10;
    p->maxiter = 20000;
    p->delta = 0.1;
    p->poll_every = 0;
    p->use_x0 = 0;
    p->use_graph = 1;
    p->profile = 0;
}

size_t hisq_links_bytes(const hisq_geom* g, int prec, int naik)
{
    Lat lat;
    if (check_geom(g, &lat)) return 0;
    if (prec != HISQ_PREC_F64 && prec != HISQ_PREC_F32) return 0;
    if (!valid_naik(naik)) return 0;
    if (naik != HISQ_NAIK_FULL && prec != HISQ_PREC_F32) return 0;
    const size_t elem = prec == HISQ_PREC_F64 ? sizeof(d2) : sizeof(f2);
    return kLinkHeaderBytes + 2 * link_block_reals(lat.Vh, naik) * (elem / 2);
}

size_t hisq_workspace_bytes(const hisq_geom* g, int nrhs, int mode)
{
    Lat lat;
    if (check_geom(g, &lat)) return 0;
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return 0;
    if (mode != HISQ_MODE_FP64 && mode != HISQ_MODE_MIXED) return 0;
    Ws w;
    return ws_layout(lat, nrhs, mode, WS_SOLVE, nullptr, &w);
}

size_t hisq_backward_workspace_bytes(const hisq_geom* g, int nrhs, int mode)
{
    Lat lat;
    if (check_geom(g, &lat)) return 0;
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return 0;
    if (mode != HISQ_MODE_FP64 && mode != HISQ_MODE_MIXED) return 0;
    Ws w;
    return ws_layout(lat, nrhs, mode, WS_BACKWARD, nullptr, &w);
}

size_t hisq_full_workspace_bytes(const hisq_geom* g, int nrhs, int mode)
{
    Lat lat;
    if (check_geom(g, &lat)) return 0;
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return 0;
    if (mode != HISQ_MODE_FP64 && mode != HISQ_MODE_MIXED) return 0;
    Ws w;
    return ws_layout(lat, nrhs, mode, WS_FULL, nullptr, &w);
}

size_t hisq_trace_workspace_bytes(const hisq_geom* g, int nrhs, int mode)
{
    Lat lat;
    if (check_geom(g, &lat)) return 0;
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return 0;
    if (mode != HISQ_MODE_FP64 && mode != HISQ_MODE_MIXED) return 0;
    Ws w;
    return ws_layout(lat, nrhs, mode, WS_TRACE, nullptr, &w);
}

int hisq_pack_links(const hisq_geom* g, const double* U, const double* N, int prec, int naik,
                    void* packed, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_geom(g, &lat);
    if (rc) return rc;
    if (!U || !N || !packed) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(U, N, packed);
    if (prec != HISQ_PREC_F64 && prec != HISQ_PREC_F32) return fail(HISQ_EINVAL, "bad prec %d", prec);
    if (!valid_naik(naik))
        return fail(HISQ_EINVAL, "bad naik %d", naik);
    if (naik != HISQ_NAIK_FULL && prec != HISQ_PREC_F32)
        return fail(HISQ_EINVAL, "compressed Naik storage is FP32 only");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    forget_links(packed);
    HIP_TRY(launch_pack(lat, reinterpret_cast<const d2*>(U), reinterpret_cast<const d2*>(N), prec,
                        naik, packed, s));
    if (naik != HISQ_NAIK_FULL) {
        // a buffer that fails its round-trip check is left without a valid
        // header, so that no later call accepts it
        auto reject = [&]() -> int {
            const uint32_t zero = 0;
            HIP_TRY(hipMemcpyAsync(packed, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
            return HISQ_OK;
        };
        LinkHeader h{};
        HIP_TRY(hipMemcpyAsync(&h, packed, sizeof(h), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        float err, smin, smax;
        std::memcpy(&err, &h.naik_err_bits, sizeof(err));
        std::memcpy(&smin, &h.scale_min_bits, sizeof(smin));
        std::memcpy(&smax, &h.scale_max_bits, sizeof(smax));
        const char* name = naik == HISQ_NAIK_R14 ? "r14" : naik == HISQ_NAIK_R13 ? "r13" : "r9";
        const float tol = naik == HISQ_NAIK_R9 ? kR9Tolerance : kNaikTolerance;
        if (!(err <= tol)) {
            if ((rc = reject())) return rc;
            return fail(HISQ_EPACK, "%s round-trip error %g: Naik links are not s * U(3)", name, err);
        }
        if (naik == HISQ_NAIK_R9) {
            if (!(smin > 0.0f) || !(smax - smin <= kR9ScaleSpread * smax)) {
                if ((rc = reject())) return rc;
                return fail(HISQ_EPACK, "r9 needs one Naik scale: |det N|^(1/3) spans %g .. %g", smin, smax);
            }
            const float scale = 0.5f * (smin + smax);
            LinkHeader* hd = reinterpret_cast<LinkHeader*>(packed);
            HIP_TRY(hipMemcpyAsync(&hd->naik_scale, &scale, sizeof(scale), hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
    }
    remember_links(packed, lat, prec, naik);
    return HISQ_OK;
}

int hisq_dslash(const hisq_geom* g, int out_parity, int nrhs, int prec, int naik, int layout,
                const void* packed, const void* in, void* out, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_geom(g, &lat);
    if (rc) return rc;
    if (!packed || !in || !out) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(packed, in, out);
    if (out_parity != 0 && out_parity != 1) return fail(HISQ_EINVAL, "out_parity must be 0 or 1");
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return fail(HISQ_EINVAL, "nrhs = %d outside 1..8", nrhs);
    if (prec != HISQ_PREC_F64 && prec != HISQ_PREC_F32) return fail(HISQ_EINVAL, "bad prec %d", prec);
    if (!valid_naik(naik))
        return fail(HISQ_EINVAL, "bad naik %d", naik);
    if (naik != HISQ_NAIK_FULL && prec != HISQ_PREC_F32)
        return fail(HISQ_EINVAL, "compressed Naik storage is FP32 only");
    if (layout != HISQ_LAYOUT_SITE && layout != HISQ_LAYOUT_COLOUR)
        return fail(HISQ_EINVAL, "bad layout %d", layout);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_links("packed", packed, lat, prec, naik, s, false))) return rc;
    const int nk = naik;
    const bool cm = layout == HISQ_LAYOUT_COLOUR;
    Tile t;
    if (prec == HISQ_PREC_F64) {
        DslashArgs<double> a{};
        a.lat = lat;
        a.parity = out_parity;
        a.links = link_block<double>(packed, lat.Vh, HISQ_NAIK_FULL, out_parity);
        a.in = reinterpret_cast<const d2*>(in);
        a.out = reinterpret_cast<d2*>(out);
        if ((rc = get_tile(lat, nrhs, prec, HISQ_NAIK_FULL, a, s, &t, EPI_PLAIN, cm))) return rc;
        HIP_TRY(launch_ds(EPI_PLAIN, nrhs, HISQ_NAIK_FULL, t, a, s, cm));
    } else {
        DslashArgs<float> a{};
        a.lat = lat;
        a.parity = out_parity;
        a.links = link_block<float>(packed, lat.Vh, nk, out_parity);
        a.naik_scale = naik_scale_of(packed);
        a.in = reinterpret_cast<const f2*>(in);
        a.out = reinterpret_cast<f2*>(out);
        if ((rc = get_tile(lat, nrhs, prec, nk, a, s, &t, EPI_PLAIN, cm))) return rc;
        HIP_TRY(launch_ds(EPI_PLAIN, nrhs, nk, t, a, s, cm));
    }
    return HISQ_OK;
}

int hisq_cg_solve(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                  const void* links64, const void* links32, const double* b_e, double* x_e,
                  void* ws, size_t ws_bytes, hisq_info* info, void* stream)
{
    return hisq::cg_solve_on(g, mass, nrhs, p, links64, links32, b_e, x_e, ws, ws_bytes, info,
                             stream, nullptr);
}

int hisq_cg_solve_backward(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                           const void* links64, const void* links32, const double* x_e,
                           const double* grad_x, double* grad_U, double* grad_N, double* grad_m,
                           double* grad_b, void* ws, size_t ws_bytes, hisq_info* info,
                           void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_geom(g, &lat);
    if (rc) return rc;
    if ((rc = check_params(p, nrhs))) return rc;
    if (!links64 || !x_e || !grad_x || !grad_U || !grad_N || !grad_m || !ws)
        return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(links64, links32, x_e, grad_x, grad_U, grad_N, grad_b, ws);
    if (p->mode == HISQ_MODE_MIXED && !links32)
        return fail(HISQ_EINVAL, "MIXED mode needs FP32 links");
    Ws w;
    const size_t need = ws_layout(lat, nrhs, p->mode, WS_BACKWARD, nullptr, &w);
    if (ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_solve_links(links64, links32, lat, p->mode, p->naik, s))) return rc;
    ws_layout(lat, nrhs, p->mode, WS_BACKWARD, reinterpret_cast<char*>(ws), &w);
    d2* y = grad_b ? reinterpret_cast<d2*>(grad_b) : w.y;
    // adjoint solve: A is Hermitian, so A y = grad_x uses the same operator
    hisq_params q = *p;
    q.use_x0 = 0;
    const int st = solve_impl(mass, nrhs, &q, links64, links32, grad_x, (double*)y, w, info,
                              stream, lat);
    if (st < 0) return st;
    // The force kernel reads colour-major fields: y is still in that order in
    // the solver's working copy (w.xc), x is converted into the free FP64
    // residual field (w.r64); then t = D_oe x and s = D_oe y (FP64, colour-major)
    const d2* yc = w.xc;
    d2* xc = w.r64;
    HIP_TRY(launch_layout(reinterpret_cast<const d2*>(x_e), xc, lat.Vh, nrhs, true, s));
    Tile t = default_tile(nrhs, HISQ_PREC_F64);
    DslashArgs<double> a{};
    a.lat = lat;
    a.parity = 1;
    a.links = link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, 1);
    a.in = xc;
    a.out = w.tx;
    HIP_TRY(launch_ds(EPI_PLAIN, nrhs, HISQ_NAIK_FULL, t, a, s, true));
    a.in = yc;
    a.out = w.sy;
    HIP_TRY(launch_ds(EPI_PLAIN, nrhs, HISQ_NAIK_FULL, t, a, s, true));
    hipEvent_t fe[2] = {nullptr, nullptr};
    auto release = on_scope_exit([&] { destroy_events(fe, 2); });
    if (p->profile) {
        HIP_TRY(hipEventCreate(&fe[0]));
        HIP_TRY(hipEventCreate(&fe[1]));
        HIP_TRY(hipEventRecord(fe[0], s));
    }
    HIP_TRY(launch_force(lat, nrhs, xc, yc, w.tx, w.sy, reinterpret_cast<d2*>(grad_U),
                         reinterpret_cast<d2*>(grad_N), s));
    if (p->profile) HIP_TRY(hipEventRecord(fe[1], s));
    HIP_TRY(launch_redot(y, reinterpret_cast<const d2*>(x_e), lat.Vh, nrhs, -8.0 * mass, grad_m,
                         w.red, w.cnt, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (p->profile) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, fe[0], fe[1]));
        if (info) {
            info->kernel_ms[HISQ_K_FORCE] = ms;
            info->kernel_launches[HISQ_K_FORCE] = 1;
        }
    }
    return st;
}

int hisq_dslash_dmu(const hisq_geom* g, int out_parity, int nrhs, int nder, const void* links64,
                    const double* in, double* out, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_geom(g, &lat);
    if (rc) return rc;
    if (!links64 || !in || !out) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(links64, in, out);
    if (out_parity != 0 && out_parity != 1) return fail(HISQ_EINVAL, "out_parity must be 0 or 1");
    if (nrhs < 1 || nrhs > HISQ_MAX_RHS) return fail(HISQ_EINVAL, "nrhs = %d outside 1..8", nrhs);
    if (nder < 0 || nder > HISQ_MAX_DERIVATIVE)
        return fail(HISQ_EINVAL, "nder = %d outside 0..%d", nder, HISQ_MAX_DERIVATIVE);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if ((rc = check_links("links64", links64, lat, HISQ_PREC_F64, HISQ_NAIK_FULL, s, false)))
        return rc;
    const d2* vin = reinterpret_cast<const d2*>(in);
    d2* vout = reinterpret_cast<d2*>(out);
    const d2* lk = link_block<double>(links64, lat.Vh, HISQ_NAIK_FULL, out_parity);
    if (nder > 0) {
        HIP_TRY(launch_dslash_dmu(lat, out_parity, nrhs, nder, lk, vin, vout, s));
        return HISQ_OK;
    }
    DslashArgs<double> a{};
    a.lat = lat;
    a.parity = out_parity;
    a.links = lk;
    a.in = vin;
    a.out = vout;
    HIP_TRY(launch_ds(EPI_PLAIN, nrhs, HISQ_NAIK_FULL, default_tile(nrhs, HISQ_PREC_F64), a, s, false));
    return HISQ_OK;
}

static int check_full_args(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                           const void* links64, const void* links32, Lat* lat)
{
    int rc = check_geom(g, lat);
    if (rc) return rc;
    if ((rc = check_params(p, nrhs))) return rc;
    if (!links64) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(links64, links32);
    if (p->mode == HISQ_MODE_MIXED && !links32)
        return fail(HISQ_EINVAL, "MIXED mode needs FP32 links");
    if (!std::isfinite(mass) || mass == 0.0)
        return fail(HISQ_EINVAL, "mass must be finite and nonzero (x_o = (b_o - D_oe x_e) / 2m)");
    return HISQ_OK;
}

int hisq_solve_full(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                    const void* links64, const void* links32, const double* b_e, const double* b_o,
                    double* x_e, double* x_o, void* ws, size_t ws_bytes, hisq_info* info,
                    void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_full_args(g, mass, nrhs, p, links64, links32, &lat);
    if (rc) return rc;
    if (!b_e || !b_o || !x_e || !x_o || !ws) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(b_e, b_o, x_e, x_o, ws);
    Ws w;
    const size_t need = ws_layout(lat, nrhs, p->mode, WS_FULL, nullptr, &w);
    if (ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if ((rc = check_solve_links(links64, links32, lat, p->mode, p->naik,
                                reinterpret_cast<hipStream_t>(stream))))
        return rc;
    ws_layout(lat, nrhs, p->mode, WS_FULL, reinterpret_cast<char*>(ws), &w);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = full_impl(mass, nrhs, p, links64, links32, reinterpret_cast<const d2*>(b_e),
                   reinterpret_cast<const d2*>(b_o), reinterpret_cast<d2*>(x_e),
                   reinterpret_cast<d2*>(x_o), w, info, s, lat);
    if (rc < 0) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return rc;
}

int hisq_trace_estimate(const hisq_geom* g, double mass, int nrhs, const hisq_params* p,
                        const void* links64, const void* links32, int ninsert, const int* orders,
                        const double* eta_e, const double* eta_o, double* est, void* ws,
                        size_t ws_bytes, hisq_info* info, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    Lat lat;
    int rc = check_full_args(g, mass, nrhs, p, links64, links32, &lat);
    if (rc) return rc;
    if (!eta_e || !eta_o || !est || !ws || !orders) return fail(HISQ_EINVAL, "NULL pointer");
    HISQ_CHECK_ALIGNED(eta_e, eta_o, ws);
    if ((reinterpret_cast<uintptr_t>(est) & 7u) != 0) return fail(HISQ_EINVAL, "est must be 8-byte aligned");
    if (ninsert < 1 || ninsert > HISQ_MAX_INSERTIONS)
        return fail(HISQ_EINVAL, "ninsert = %d outside 1..%d", ninsert, HISQ_MAX_INSERTIONS);
    for (int j = 0; j < ninsert; ++j)
        if (orders[j] < 0 || orders[j] > HISQ_MAX_DERIVATIVE)
            return fail(HISQ_EINVAL, "orders[%d] = %d outside 0..%d", j, orders[j], HISQ_MAX_DERIVATIVE);
    Ws w;
    const size_t need = ws_layout(lat, nrhs, p->mode, WS_TRACE, nullptr, &w);
    if (ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    if ((rc = check_solve_links(links64, links32, lat, p->mode, p->naik,
                                reinterpret_cast<hipStream_t>(stream))))
        return rc;
    ws_layout(lat, nrhs, p->mode, WS_TRACE, reinterpret_cast<char*>(ws), &w);
    return trace_impl(mass, nrhs, p, links64, links32, ninsert, orders,
                      reinterpret_cast<const d2*>(eta_e), reinterpret_cast<const d2*>(eta_o), est, w,
                      info, reinterpret_cast<hipStream_t>(stream), lat);
}

size_t hisq_batched_workspace_bytes(int nprob, const hisq_problem* probs, int mode)
{
    if (mode != HISQ_MODE_FP64 && mode != HISQ_MODE_MIXED) return 0;
    if (check_problems(nprob, probs, mode)) return 0;
    std::vector<Ws> ws;
    CgState* st;
    void* tab;
    return batched_layout(nprob, probs, mode, nullptr, &ws, &st, &tab);
}

int hisq_cg_solve_batched(int nprob, const hisq_problem* probs, const hisq_params* p, void* ws,
                          size_t ws_bytes, hisq_info* infos, void* stream)
{
    (void)hipGetLastError();  // drop a stale error left by an earlier failed call
    if (!p) return fail(HISQ_EINVAL, "params is NULL");
    int rc = check_params(p, 1);
    if (rc) return rc;
    if ((rc = check_problems(nprob, probs, p->mode))) return rc;
    if (!ws) return fail(HISQ_EINVAL, "workspace is NULL");
    HISQ_CHECK_ALIGNED(ws);
    std::vector<Ws> w;
    CgState* states;
    void* table;
    const size_t need = batched_layout(nprob, probs, p->mode, nullptr, &w, &states, &table);
    if (ws_bytes < need)
        return fail(HISQ_EWORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, need);
    for (int j = 0; j < nprob; ++j) {
        const Lat lat = make_lat(probs[j].geom);
        if ((rc = check_solve_links(probs[j].links64, probs[j].links32, lat, p->mode, p->naik,
                                    reinterpret_cast<hipStream_t>(stream))))
            return fail(rc, "problem %d: %s", j, std::string(g_err).c_str());
    }
    batched_layout(nprob, probs, p->mode, reinterpret_cast<char*>(ws), &w, &states, &table);
    Engine E;
    E.prm = *p;
    E.mixed = p->mode == HISQ_MODE_MIXED;
    E.nk = E.mixed ? p->naik : HISQ_NAIK_FULL;
    E.s = reinterpret_cast<hipStream_t>(stream);
    E.states = states;
    E.table = table;
    for (int j = 0; j < nprob; ++j) {
        Prob q;
        q.lat = make_lat(probs[j].geom);
        q.n = probs[j].nrhs;
        q.mass = probs[j].mass;
        q.m4 = 4.0 * q.mass * q.mass;
        q.links64 = probs[j].links64;
        q.links32 = probs[j].links32;
        q.ub = reinterpret_cast<const d2*>(probs[j].b);
        q.ux = reinterpret_cast<d2*>(probs[j].x);
        q.b = w[j].bc;
        q.x = w[j].xc;
        q.w = w[j];
        E.P.push_back(q);
    }
    return E.run(infos);
}

int hisq_set_tuning(int mode, int rhs_per_thread, int block_size, int tile_order, int stage_rows)
{
    if (mode < 0 || mode > 2) return fail(HISQ_EINVAL, "unknown tuning mode %d", mode);
    if (mode == 1) {
        if (rhs_per_thread < 1 || rhs_per_thread > HISQ_MAX_RHS)
            return fail(HISQ_EINVAL, "rhs_per_thread must be in 1..8");
        if (block_size != 64 && block_size != 128 && block_size != 256)
            return fail(HISQ_EINVAL, "block_size must be 64, 128 or 256");
        if (tile_order < 0 || tile_order > 3) return fail(HISQ_EINVAL, "tile_order must be 0..3");
        if (stage_rows < 0 || stage_rows > 64) return fail(HISQ_EINVAL, "stage_rows must be 0..64");
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_mode = mode;
    g_force_nr = rhs_per_thread;
    g_force_bs = block_size;
    g_force_order = mode == 1 ? tile_order : 1;
    g_force_rows = mode == 1 ? stage_rows : 0;
    g_force_eo_nr = 0;
    return HISQ_OK;
}

int hisq_set_tuning_eo(int rhs_per_thread, int block_size, int tile_order, int stage_rows)
{
    if (rhs_per_thread != 0) {
        if (rhs_per_thread < 1 || rhs_per_thread > HISQ_MAX_RHS)
            return fail(HISQ_EINVAL, "rhs_per_thread must be in 0..8");
        if (block_size != 64 && block_size != 128 && block_size != 256)
            return fail(HISQ_EINVAL, "block_size must be 64, 128 or 256");
        if (tile_order < 0 || tile_order > 3) return fail(HISQ_EINVAL, "tile_order must be 0..3");
        if (stage_rows < 0 || stage_rows > 64) return fail(HISQ_EINVAL, "stage_rows must be 0..64");
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_force_eo_nr = rhs_per_thread;
    g_force_eo_bs = block_size;
    g_force_eo_order = tile_order;
    g_force_eo_rows = stage_rows;
    return HISQ_OK;
}

const char* hisq_last_error(void) { return g_err; }

}  // extern "C"
