"""Benchmark: HISQ Dslash GB/s and CG time-to-solution on one MI355X.

Workload: 48^3 x 12 lattice, 8 bundled rhs, m = 0.01, links drawn with
smearing width 0.2 (synthetic stand-in for the finite-temperature gauge
ensembles the paper measures on), complex Gaussian sources.

One step = one mixed-precision (FP32 iteration, FP64 reliable updates) CG solve
of the 8-rhs bundle with r14 Naik links, from x = 0 to true residual 1e-10;
inputs and packed links are resident in HBM before the timed region.  Every
Dslash launch inside the timed steps is timed with HIP events on the stream it
runs on.

The JSON line reports
  value          algorithmic GB/s of the two half-Dslash kernels of the CG
                 (links + one read of the input + one write/update of outputs),
  roofline       the dominant kernel's achieved GB/s against 8 TB/s,
  cg             time-to-solution of the step against 8 sequential FP64 1-rhs
                 solves of the same sources (same GPU), iterations, residuals;
                 bundle_forms: the same 8-rhs solve in FP64 and in mixed
                 precision with full, r13 and r9 Naik links,
  accuracy       per-rhs true residual and the a-posteriori solution-error bound,
  dslash_sweep   standalone Dslash GB/s for n = 1, 2, 4, 8 (FP64, FP32, r14, r13, r9),
  full_and_trace the full-matrix solve and one bundle of eq. (2) trace terms,
  config2        32^3 x 8: Dslash sweep and CG time against bundle size,
  paper_lattice  64^3 x 16 (the paper's production size): r14 Dslash sweep and
                 one 8-rhs mixed solve,
  backward       24^3 x 6 gradient: adjoint solve and link-force kernel,
  batched        six solves in one launch per CG phase against six separate ones,
  cpu_baseline   the FP64 CPU oracle on the host cores: Dslash rates, full CGs,
                 and one headline rhs to 1e-13 (the headline's error against it).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Dslash GB/s (% HBM peak) at 1-8 rhs; CG solve time mixed vs FP64 @1e-10"
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lattice", type=str, default="48,48,48,12")
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--mass", type=float, default=0.01)
    ap.add_argument("--eps", type=float, default=0.2)
    ap.add_argument("--naik", choices=["r14", "r13", "r9", "full"], default="r14")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-paper-lattice", action="store_true",
                    help="skip the 64^3 x 16 Dslash sweep and solve")
    ap.add_argument("--no-trace", action="store_true")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the 32^3 x 8 Dslash sweep and CG bundle gains (and the "
                         "64^3 x 16 block)")
    ap.add_argument("--no-backward", action="store_true",
                    help="skip the 24^3 x 6 gradient (adjoint solve + link force) timing")
    ap.add_argument("--no-oracle-cg", action="store_true",
                    help="skip the oracle's FP64 CG runs in the CPU baseline (the longest part)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--tile", default=DEFAULT_TILE,
                    help="tile of the solve's D_oe Dslash (and p-update): "
                         "'rhs_per_thread,tile_order,stage_rows' (the autotuner's pick for this "
                         "workload, pinned so that every run and every counter profile times the "
                         "same kernels) or 'auto' (autotune both Dslash kernels)")
    ap.add_argument("--tile-eo", default=DEFAULT_TILE_EO,
                    help="tile of the D_eo Dslash with the CG epilogue: "
                         "'rhs_per_thread,block_size,tile_order,stage_rows' (the autotuner's pick), "
                         "used unless --tile is 'auto'")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three 1 GiB device-to-device copies (the reference kernel "
                         "that scales hardware byte counters)")
    return ap.parse_args()


# Files whose contents decide the Dslash kernels' code: a counter summary taken
# from other contents no longer describes the kernel.
# The autotuner's picks for the solve's two Dslash kernels at 48^3 x 12, n = 8,
# mixed r14 (D_oe: rhs per thread, tile order, staged rows; D_eo with the CG
# epilogue: rhs per thread, block size, tile order, staged rows), pinned so
# that every run and every counter profile times the same kernels.
DEFAULT_TILE = "4,3,4"
DEFAULT_TILE_EO = "2,256,3,0"

KERNEL_SOURCES = ("paper_1411_4439_amd/csrc/dslash.hip", "paper_1411_4439_amd/csrc/stencil.h",
                  "paper_1411_4439_amd/csrc/naik.h", "paper_1411_4439_amd/csrc/hisq_device.h",
                  "paper_1411_4439_amd/csrc/hisq_internal.h", "paper_1411_4439_amd/build.py")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, tile):
    """HBM bytes per launch of `kernel` from a committed hardware-counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy), or None when no summary
    matches this kernel's current source, workload and tile."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if (kv.get("kernel") == kernel and kv.get("workload") == workload
                and kv.get("source_sha256") == kernel_source_sha() and kv.get("tile") == tile
                and "traffic_bytes_per_launch" in kv):
            return float(kv["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    return None, None


_LINKS = {}


def links_of(W, L, eps, seed):
    """Seeded canonical links, generated once per (lattice, eps, seed) in this run."""
    key = (tuple(L), eps, seed)
    if key not in _LINKS:
        _LINKS[key] = W.make_links(L, eps, seed)
    return _LINKS[key]


def median_event_ms(fn, stream, reps, warm=5):
    """Median duration of `reps` launches of fn, each between its own pair of
    HIP events on `stream`, after `warm` untimed launches."""
    import torch
    for _ in range(warm):
        fn()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    evs[0].record(stream)
    for r in range(reps):
        fn()
        evs[r + 1].record(stream)
    evs[-1].synchronize()
    return float(np.median([evs[r].elapsed_time(evs[r + 1]) for r in range(reps)]))


def config2_block(H, R, W, dev, stream):
    """32^3 x 8, m = 0.02: standalone Dslash at n = 1, 2, 4, 8 (FP64, FP32, FP32
    with r14 Naik links), and CG time-to-solution at n = 1, 2, 4, 8, mixed r14 and
    FP64, with the bundle gain n * t(1) / t(n) (the paper's 4-rhs over 1-rhs gain
    is about 2.05, against the 2.16 of its Dslash intensity, Sec. 3)."""
    import torch
    L, m = (32, 32, 32, 8), 0.02
    Vh = W.half_volume(L)
    U, N = links_of(W, L, 0.3, W.links_seed(2))
    links = H.Links(L, dev(U), dev(N))
    b8 = W.make_sources(L, 8, W.sources_seed(2))
    H.hisq_set_tuning(0)
    sweep = {}
    for prec, nk, tag in ((H.PREC_F64, H.NAIK_FULL, "f64"), (H.PREC_F32, H.NAIK_FULL, "f32"),
                          (H.PREC_F32, H.NAIK_R14, "f32_r14")):
        dt = torch.complex128 if prec == H.PREC_F64 else torch.complex64
        for nn in (1, 2, 4, 8):
            vin = dev(b8[:, :, :nn]).to(dt).permute(1, 0, 2).contiguous()
            vout = torch.empty_like(vin)
            packed = links.packed(prec, nk)
            ms = median_event_ms(lambda: H.hisq_dslash(L, 1, nn, prec, nk, H.LAYOUT_COLOUR, packed,
                                                       vin, vout), stream, 100, warm=10)
            scale = 2 if prec == H.PREC_F64 else 1
            byt = Vh * scale * (R.LINK_BYTES_F32["r14" if nk == H.NAIK_R14 else "full"]
                                + 2 * R.VEC_BYTES_F32 * nn)
            sweep["%s_n%d" % (tag, nn)] = {"ms": round(ms, 4), "GBps": round(byt / ms / 1e6, 1),
                                           "pct_hbm_peak": round(byt / ms / 1e6 / HBM_PEAK_GBPS * 100, 1)}
    cg = {}
    for mode, nk, tag in ((H.MODE_MIXED, H.NAIK_R14, "mixed_r14"), (H.MODE_FP64, H.NAIK_FULL, "fp64")):
        per = {}
        for nn in (1, 2, 4, 8):
            bd = dev(b8[:, :, :nn])
            ws = H.empty_bytes(H.hisq_workspace_bytes(L, nn, mode))
            H.solve(links, m, bd, mode=mode, naik=nk, ws=ws)  # tune + warm
            torch.cuda.synchronize()
            best = 1e30
            for _ in range(2):
                t0 = time.perf_counter()
                _, st, info = H.solve(links, m, bd, mode=mode, naik=nk, ws=ws)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            if st != H.HISQ_OK:
                raise SystemExit("config2 solve failed: %s" % info)
            per[nn] = {"seconds": round(best, 4), "seconds_per_rhs": round(best / nn, 4),
                       "iters_max": max(info["iters"]),
                       "rel_true_res_max": max(info["rel_true_res"])}
        for nn in (2, 4, 8):
            per[nn]["gain_vs_1rhs"] = round(nn * per[1]["seconds"] / per[nn]["seconds"], 2)
        cg[tag] = {"n%d" % k: v for k, v in per.items()}
    cg["paper_4rhs_gain"] = "about 2.05 (95% of the 2.16 Dslash intensity gain), Sec. 3, single precision"
    return {"workload": "32x32x32x8, m=0.02, eps=0.3, colour-major fields, autotuned tiles",
            "dslash_sweep": sweep, "cg": cg}


def paper_lattice_block(H, R, W, dev, stream):
    """64^3 x 16, the size of the paper's production lattices (Sec. 3): the
    standalone FP32 r14 half-Dslash at n = 1, 2, 4, 8 (colour-major, autotuned)
    and one mixed-precision r14 CG solve of an 8-rhs bundle (m = 0.01, eps =
    0.2, true residual 1e-10), to show how the kernels scale past the headline
    lattice."""
    import torch
    L, m, n = (64, 64, 64, 16), 0.01, 8
    Vh = W.half_volume(L)
    t0 = time.time()
    U, N = W.make_links(L, 0.2, W.links_seed(6))  # not cached: 4.8 GB on the host
    b = W.make_sources(L, n, W.sources_seed(6))
    log("64^3 x 16 inputs in %.1f s" % (time.time() - t0))
    links = H.Links(L, dev(U), dev(N), f32=False, r14=True)
    del U, N
    H.hisq_set_tuning(0)
    bd = dev(b)
    sweep = {}
    packed = links.packed(H.PREC_F32, H.NAIK_R14)
    for nn in (1, 2, 4, 8):
        vin = bd[:, :, :nn].to(torch.complex64).permute(1, 0, 2).contiguous()
        vout = torch.empty_like(vin)
        ms = median_event_ms(lambda: H.hisq_dslash(L, 1, nn, H.PREC_F32, H.NAIK_R14, H.LAYOUT_COLOUR,
                                                   packed, vin, vout), stream, 100, warm=10)
        byt = Vh * (R.LINK_BYTES_F32["r14"] + 2 * R.VEC_BYTES_F32 * nn)
        sweep["f32_r14_n%d" % nn] = {"ms": round(ms, 4), "GBps": round(byt / ms / 1e6, 1),
                                     "pct_hbm_peak": round(byt / ms / 1e6 / HBM_PEAK_GBPS * 100, 1)}
        del vin, vout
    ws = H.empty_bytes(H.hisq_workspace_bytes(L, n, H.MODE_MIXED))
    H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14, ws=ws)  # tune + warm
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, st, info = H.solve(links, m, bd, mode=H.MODE_MIXED, naik=H.NAIK_R14, ws=ws)
    torch.cuda.synchronize()
    cg = {"seconds": round(time.perf_counter() - t1, 4), "status": st, "iters_max": max(info["iters"]),
          "reliable_updates": info["reliable_updates"],
          "rel_true_res_max": float("%.3e" % max(info["rel_true_res"]))}
    return {"workload": "64x64x64x16, m=0.01, eps=0.2, 8 rhs, colour-major fields, autotuned tiles",
            "dslash_sweep": sweep, "cg_mixed_r14_n8": cg}


def backward_block(H, W, dev):
    """24^3 x 6, n = 4, m = 0.05: the forward solve, then the backward (adjoint
    solve on the same operator, two FP64 half-Dslash, the link-force kernel and
    dL/dm), in FP64 and in mixed precision with r14 Naik links; the link-force
    kernel's algorithmic GB/s: it reads x, y (even) and D_oe x, D_oe y (odd), each
    once, and writes dL/dU and dL/dN, V (1152 + 96 n) bytes."""
    import torch
    L, m, n = (24, 24, 24, 6), 0.05, 4
    V = W.volume(L)
    U, N = W.make_links(L, 0.3, W.links_seed(5))
    links = H.Links(L, dev(U), dev(N))
    eta = dev(W.make_sources(L, n, W.sources_seed(5)))
    phi = dev(W.make_sources(L, n, W.sources_seed(5, 1)))
    H.hisq_set_tuning(0)
    out = {"workload": "24x24x24x6, n=4, m=0.05, eps=0.3; L = sum_k Re(phi_k^dag x_k)"}
    force_bytes = V * (1152 + 96 * n)
    for mode, nk, tag in ((H.MODE_FP64, H.NAIK_FULL, "fp64"), (H.MODE_MIXED, H.NAIK_R14, "mixed_r14")):
        gU = torch.empty((4, V, 3, 3), dtype=torch.complex128, device="cuda")
        gN = torch.empty_like(gU)
        gm = torch.zeros((), dtype=torch.float64, device="cuda")
        gb = torch.empty_like(eta)
        wsb = H.empty_bytes(H.hisq_backward_workspace_bytes(L, n, mode))
        l32 = links.packed(H.PREC_F32, nk) if mode == H.MODE_MIXED else None
        x, st, info = H.solve(links, m, eta, mode=mode, naik=nk)  # tune + warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, info = H.solve(links, m, eta, mode=mode, naik=nk)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0

        def bwd(profile=0):
            p = H.hisq_default_params(mode=mode, naik=nk, profile=profile)
            return H.hisq_cg_solve_backward(L, m, n, p, links.f64, l32, x, phi, gU, gN, gm, gb, wsb)
        bwd()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stb, infb = bwd()
        torch.cuda.synchronize()
        t_bwd = time.perf_counter() - t0
        fms = []
        for _ in range(5):
            _, infp = bwd(profile=1)
            fms.append(infp.kernel_ms[H.K_FORCE])
        f_ms = float(np.median(fms))
        out[tag] = {"forward_seconds": round(t_fwd, 4), "forward_iters_max": max(info["iters"]),
                    "backward_seconds": round(t_bwd, 4), "adjoint_iters_max": infb.total_iters,
                    "adjoint_solve_seconds": round(infb.seconds, 4), "status": stb,
                    "force_kernel_ms": round(f_ms, 4),
                    "force_kernel_GBps": round(force_bytes / f_ms / 1e6, 1),
                    "force_kernel_frac": round(force_bytes / f_ms / 1e6 / 8000.0, 3),
                    "force_algorithmic_bytes": force_bytes}
    return out


def cpu_baseline(args, W, R, L, U, N, b, n, m, Vh, iters, ms_per_step, x_head0):
    """The FP64 CPU oracle, as it stands, on the host cores: half-Dslash rates on
    the 48^3 x 12 workload (all threads and one), on 8^4 and 32^3 x 8 at n = 1, 2,
    4, 8; full oracle CGs on 8^4 (n = 1) and 32^3 x 8 (n = 1 and 8) to relative
    residual 1e-10; and one rhs of the 48^3 x 12 headline to 1e-13, whose
    solution gives the headline's error against the oracle."""
    import oracle
    import platform

    def timed(fn, seconds, cap=1000):
        t0c = time.perf_counter()
        k = 0
        while True:
            fn()
            k += 1
            if time.perf_counter() - t0c > seconds or k >= cap:
                return k, (time.perf_counter() - t0c) / k

    vh = b[:, :, :n]
    threads = oracle.num_threads()
    reps, cpu_s = timed(lambda: oracle.dslash_eo(L, U, N, vh, 1), args.cpu_seconds * 0.3)
    oracle.set_num_threads(1)
    reps_1, cpu_1 = timed(lambda: oracle.dslash_eo(L, U, N, vh, 1), args.cpu_seconds * 0.1)
    oracle.set_num_threads(threads)
    cpu_bytes = Vh * 2 * (R.LINK_BYTES_F32["full"] + 2 * R.VEC_BYTES_F32 * n)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    res = {"value": round(cpu_bytes / cpu_s / 1e9, 3), "unit": "GB/s", "cores": threads,
           "kind": "oracle",
           "sample": "%d FP64 half-Dslash applications, %s, %d rhs (%.3f s each)"
                     % (reps, "x".join(map(str, L)), n, cpu_s),
           "cpu_model": model or platform.processor(), "nproc": os.cpu_count(),
           "one_thread_GBps": round(cpu_bytes / cpu_1 / 1e9, 3)}
    # Dslash on 8^4 and 32^3 x 8, all threads and one thread
    table = {}
    for Lc, seed in (((8, 8, 8, 8), W.links_seed(1)), ((32, 32, 32, 8), W.links_seed(2))):
        Uc, Nc = links_of(W, Lc, 0.3, seed)
        bc = W.make_sources(Lc, 8, seed + 500)
        vhc = W.half_volume(Lc)
        for nn in (1, 2, 4, 8):
            v = np.ascontiguousarray(bc[:, :, :nn])
            byt = vhc * 2 * (R.LINK_BYTES_F32["full"] + 2 * R.VEC_BYTES_F32 * nn)
            row = {}
            for th in (threads, 1):
                oracle.set_num_threads(th)
                k, sec = timed(lambda: oracle.dslash_eo(Lc, Uc, Nc, v, 1), 0.25, cap=200)
                row["GBps_%dthreads" % th] = round(byt / sec / 1e9, 3)
            oracle.set_num_threads(threads)
            table["%s_n%d" % ("x".join(map(str, Lc)), nn)] = row
    res["dslash_GBps"] = table
    if not args.no_oracle_cg:
        cgs = {}
        for Lc, mc, nn, cfg in (((8, 8, 8, 8), 0.1, 1, 1), ((32, 32, 32, 8), 0.02, 1, 2),
                                ((32, 32, 32, 8), 0.02, 8, 2)):
            Uc, Nc = links_of(W, Lc, 0.3, W.links_seed(cfg))
            bc = np.ascontiguousarray(W.make_sources(Lc, 8, W.sources_seed(cfg))[:, :, :nn])
            t0c = time.perf_counter()
            _, inf = oracle.cg(Lc, Uc, Nc, mc, bc, tol=1e-10)
            cgs["%s_n%d" % ("x".join(map(str, Lc)), nn)] = {
                "seconds": round(time.perf_counter() - t0c, 3), "iters_max": int(max(inf["iters"])),
                "true_res_max": float(max(inf["true_res"]))}
        # one rhs of the headline, to 1e-13: measured CG time and the GPU's error
        t0c = time.perf_counter()
        xo, inf = oracle.cg(L, U, N, m, np.ascontiguousarray(b[:, :, :1]), tol=1e-13)
        t_o = time.perf_counter() - t0c
        err = float(np.linalg.norm(x_head0 - xo[:, :, 0]) / np.linalg.norm(xo[:, :, 0]))
        cgs["%s_n1_tol1e-13" % "x".join(map(str, L))] = {
            "seconds": round(t_o, 2), "iters": int(inf["iters"][0]),
            "true_res": float(inf["true_res"][0])}
        res["cg"] = cgs
        res["headline_rhs0_error_vs_oracle"] = float("%.3e" % err)
        res["gpu_seconds_per_rhs"] = round(ms_per_step / 1e3 / n, 4)
    return res



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the solver shards by rhs bundle with no "
              "communication, so --gpus %d is not run (use --gpus 1)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1411_4439_amd import hisq as H
    from paper_1411_4439_amd import roofline as R
    from paper_1411_4439_amd import workload as W

    L = tuple(int(v) for v in args.lattice.split(","))
    n, m = args.nrhs, args.mass
    naik = {"r14": H.NAIK_R14, "r13": H.NAIK_R13, "r9": H.NAIK_R9}.get(args.naik, H.NAIK_FULL)
    Vh = W.half_volume(L)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    t0 = time.time()
    U, N = W.make_links(L, args.eps, W.links_seed(3))
    b = W.make_sources(L, n, W.sources_seed(3))
    log("generated links and sources in %.1f s" % (time.time() - t0))
    Ud, Nd, bd = dev(U), dev(N), dev(b)
    links = H.Links(L, Ud, Nd, r13=not args.no_sweep or args.naik == "r13",
                    r9=not args.no_sweep or args.naik == "r9")
    torch.cuda.synchronize()
    nr = order = rows = 0
    if args.tile != "auto":
        nr, order, rows = (int(v) for v in args.tile.split(","))
        eo_tile = tuple(int(v) for v in args.tile_eo.split(","))
        H.hisq_set_tuning(1, nr, 64, order, rows)
        H.hisq_set_tuning_eo(*eo_tile)
    ws = H.empty_bytes(H.hisq_workspace_bytes(L, n, H.MODE_MIXED))
    x = torch.empty_like(bd)
    stream = torch.cuda.current_stream()

    def step(profile=1):
        p = H.hisq_default_params(mode=H.MODE_MIXED, naik=naik, tol=1e-10, profile=profile)
        st, info = H.hisq_cg_solve(L, m, n, p, links.f64, links.packed(H.PREC_F32, naik), bd, x, ws)
        return st, info

    for w in range(args.warmup):
        st, info = step()
        log("warmup %d: status %d iters %s" % (w, st, list(info.iters[:n])))
    torch.cuda.synchronize()
    infos = []
    t_start = time.perf_counter()
    for k in range(args.steps):
        st, info = step()
        infos.append(info.to_dict(n))
        log("step %d: status %d, %.3f s, iters %s, updates %d" % (
            k, st, info.seconds, list(info.iters[:n]), info.reliable_updates))
        if st != H.HISQ_OK:
            raise SystemExit("solve failed: %s" % infos[-1])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps

    # the same solve without per-kernel events, each poll block one hipGraph
    graph_s = []
    for _ in range(2):
        torch.cuda.synchronize()
        tg = time.perf_counter()
        st, _ = step(profile=0)
        torch.cuda.synchronize()
        graph_s.append(time.perf_counter() - tg)

    # kernel-level figures from the HIP events recorded inside the timed steps
    nk = args.naik
    link_b = R.LINK_BYTES_F32[nk]
    vec_b = R.VEC_BYTES_F32
    bytes_oe = Vh * (link_b + 2 * vec_b * n)          # links, read p, write t
    bytes_eo = Vh * (link_b + 6 * vec_b * n)          # links, read t, p, x, r; write x, r
    bytes_pu = Vh * 3 * vec_b * n                     # read r, p; write p
    tot_ms = [sum(i["kernel_ms"][c] for i in infos) for c in range(4)]
    tot_n = [sum(i["kernel_launches"][c] for i in infos) for c in range(4)]
    # per-iteration kernels: average over the launches that did work, i.e. one
    # per iteration of the bundle (the last poll block may hold a few launches
    # after every rhs converged, which exit at once; their few microseconds stay
    # in the numerator, so the figure errs low)
    work = sum(i["total_iters"] for i in infos)
    avg_ms = [tot_ms[c] / max(work if c < 3 else tot_n[c], 1) for c in range(4)]
    gbps_oe = bytes_oe / (avg_ms[H.K_DSLASH_OE] * 1e-3) / 1e9
    gbps_eo = bytes_eo / (avg_ms[H.K_DSLASH_EO] * 1e-3) / 1e9
    gbps_pu = bytes_pu / (avg_ms[H.K_PUPDATE] * 1e-3) / 1e9
    dslash_gbps = (bytes_oe + bytes_eo) / ((avg_ms[1] + avg_ms[2]) * 1e-3) / 1e9
    dslash_gflops = 2 * Vh * R.FLOPS_PER_SITE_RHS * n / ((avg_ms[1] + avg_ms[2]) * 1e-3) / 1e9
    if tot_ms[H.K_DSLASH_EO] >= tot_ms[H.K_DSLASH_OE]:
        dom = ("dslash_eo_cg_epilogue", gbps_eo, bytes_eo, avg_ms[2])
    else:
        dom = ("dslash_oe_norm", gbps_oe, bytes_oe, avg_ms[1])
    iters = infos[-1]["iters"]
    pre = "eo_" if dom[0] == "dslash_eo_cg_epilogue" else ""
    tile = "nr=%d bs=%d order=%d rows=%d" % tuple(
        infos[-1][pre + f] for f in ("rhs_per_thread", "block_size", "tile_order", "stage_rows"))
    workload = ("HISQ even-odd CG, mixed FP32/FP64, %s Naik, %dx%dx%dx%d, %d rhs, m=%g"
                % (nk, L[0], L[1], L[2], L[3], n, m))
    traffic, traffic_src = measured_traffic(dom[0], workload, tile)
    result = {
        "metric": METRIC,
        "value": round(dslash_gbps, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded links eta*exp(i*%.1f*H), N=-(1/24)UUU, Gaussian sources)" % args.eps,
        "config": {"workload": workload,
                   "lattice": list(L), "nrhs": n, "mass": m, "tol": 1e-10, "naik": nk,
                   "parallelism": "single GPU (rhs bundles shard with no communication)"},
        "pct_hbm_peak": round(100 * dslash_gbps / HBM_PEAK_GBPS, 1),
        "dslash_gflops": round(dslash_gflops, 1),
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[1], 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(dom[1] / HBM_PEAK_GBPS, 4),
                     "traffic": None if traffic is None else round(traffic),
                     "traffic_source": traffic_src,
                     "algorithmic_bytes_per_launch": dom[2], "avg_launch_ms": round(dom[3], 5),
                     "tile": tile, "kernel_source_sha256": kernel_source_sha()},
        "kernels": {"dslash_oe_norm": {"avg_ms": round(avg_ms[1], 5), "GBps": round(gbps_oe, 1),
                                       "launches": tot_n[1], "launches_with_work": work},
                    "dslash_eo_cg_epilogue": {"avg_ms": round(avg_ms[2], 5), "GBps": round(gbps_eo, 1),
                                              "launches": tot_n[2], "launches_with_work": work},
                    "pupdate": {"avg_ms": round(avg_ms[0], 5), "GBps": round(gbps_pu, 1),
                                "launches": tot_n[0], "launches_with_work": work},
                    "reliable_update": {"avg_ms": round(avg_ms[3], 4), "count": tot_n[3]}},
        "cg": {"mixed_seconds": round(ms_per_step / 1e3, 4),
               "mixed_seconds_graph": round(min(graph_s), 4), "iters": iters,
               "reliable_updates": infos[-1]["reliable_updates"],
               "rel_true_res_max": max(infos[-1]["rel_true_res"]),
               "tile_oe": {"rhs_per_thread": infos[-1]["rhs_per_thread"],
                           "block": infos[-1]["block_size"], "order": infos[-1]["tile_order"],
                           "stage_rows": infos[-1]["stage_rows"]},
               "tile_eo": {"rhs_per_thread": infos[-1]["eo_rhs_per_thread"],
                           "block": infos[-1]["eo_block_size"], "order": infos[-1]["eo_tile_order"],
                           "stage_rows": infos[-1]["eo_stage_rows"]}},
    }
    # accuracy of the headline solution: the a-posteriori bound
    # ||x - x*|| / ||x|| <= ||b - A x|| / (4 m^2 ||x||), since lambda_min(A) >= 4 m^2
    # (the oracle's own solution error for one rhs is added by the CPU-baseline leg)
    xnorm = torch.linalg.vector_norm(x, dim=(0, 1)).cpu().numpy()
    bnorm = torch.linalg.vector_norm(bd, dim=(0, 1)).cpu().numpy()
    rel_true = np.array(infos[-1]["rel_true_res"])
    result["accuracy"] = {
        "rel_true_res": [float("%.3e" % v) for v in rel_true],
        "error_bound": [float("%.3e" % v) for v in rel_true * bnorm / (4 * m * m * xnorm)],
        "bound_note": "||x - x*|| / ||x|| <= ||b - A x|| / (4 m^2 ||x||) per rhs"}
    x_head0 = x[:, :, 0].cpu().numpy()

    # the comparison solver and the standalone sweep use the autotuner's tiles
    H.hisq_set_tuning(0)

    if not args.no_fp64_compare:
        # the plain FP64 1-rhs solver, 8 times in sequence, same sources and GPU
        ws1 = H.empty_bytes(H.hisq_workspace_bytes(L, 1, H.MODE_FP64))
        p = H.hisq_default_params(mode=H.MODE_FP64, tol=1e-10)
        cols = [bd[:, :, k:k + 1].contiguous() for k in range(n)]
        x1 = torch.empty_like(cols[0])
        H.hisq_cg_solve(L, m, 1, p, links.f64, None, cols[0], x1, ws1)  # tune + warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        it64 = []
        for k in range(n):
            st, info = H.hisq_cg_solve(L, m, 1, p, links.f64, None, cols[k], x1, ws1)
            it64.append(info.iters[0])
        torch.cuda.synchronize()
        fp64_s = time.perf_counter() - t1
        result["cg"]["fp64_1rhs_x%d_seconds" % n] = round(fp64_s, 4)
        result["cg"]["fp64_iters"] = it64
        result["cg"]["speedup_vs_fp64_1rhs"] = round(fp64_s / (ms_per_step / 1e3), 2)
        log("FP64 %d x 1-rhs: %.3f s (iters %s)" % (n, fp64_s, it64))

        # the same bundle in the other precision forms: FP64 throughout, and
        # mixed with the Naik links stored in full (18 reals), r13 and r9
        # (autotuned tiles, poll blocks as hipGraphs; one tuning + warm-up solve,
        # then one timed)
        forms = {}
        wsf = H.empty_bytes(H.hisq_workspace_bytes(L, n, H.MODE_FP64))
        for tag, mode, nk2 in (("fp64", H.MODE_FP64, H.NAIK_FULL), ("mixed_full", H.MODE_MIXED, H.NAIK_FULL),
                               ("mixed_r13", H.MODE_MIXED, H.NAIK_R13), ("mixed_r9", H.MODE_MIXED, H.NAIK_R9)):
            l32 = links.packed(H.PREC_F32, nk2) if mode == H.MODE_MIXED else None
            if mode == H.MODE_MIXED and l32 is None:
                continue
            wsb = wsf if mode == H.MODE_FP64 else ws
            p = H.hisq_default_params(mode=mode, naik=nk2, tol=1e-10)
            H.hisq_cg_solve(L, m, n, p, links.f64, l32, bd, x, wsb)
            torch.cuda.synchronize()
            tf = time.perf_counter()
            st, info = H.hisq_cg_solve(L, m, n, p, links.f64, l32, bd, x, wsb)
            torch.cuda.synchronize()
            forms[tag] = {"seconds": round(time.perf_counter() - tf, 4), "status": st,
                          "iters_max": max(info.iters[:n]), "reliable_updates": info.reliable_updates,
                          "rel_true_res_max": float("%.3e" % max(info.rel_true_res[:n]))}
        result["cg"]["bundle_forms"] = forms
        log("bundle forms", json.dumps(forms))

    if not args.no_sweep:
        sweep = {}
        # the solver's colour-major field order, plus the caller's site-major
        # order at the largest bundle for comparison
        cases = [(prec, nk2, tag, nn, H.LAYOUT_COLOUR)
                 for prec, nk2, tag in ((H.PREC_F64, H.NAIK_FULL, "f64"),
                                        (H.PREC_F32, H.NAIK_FULL, "f32"),
                                        (H.PREC_F32, H.NAIK_R14, "f32_r14"),
                                        (H.PREC_F32, H.NAIK_R13, "f32_r13"),
                                        (H.PREC_F32, H.NAIK_R9, "f32_r9"))
                 for nn in (1, 2, 4, 8)]
        cases.append((H.PREC_F32, H.NAIK_R14, "f32_r14_sitemajor", n, H.LAYOUT_SITE))
        for prec, nk2, tag, nn, lay in cases:
            dt = torch.complex128 if prec == H.PREC_F64 else torch.complex64
            vin = bd[:, :, :nn].to(dt)
            if lay == H.LAYOUT_COLOUR:
                vin = vin.permute(1, 0, 2)
            vin = vin.contiguous()
            vout = torch.empty_like(vin)
            packed = links.packed(prec, nk2)
            for _ in range(10):
                H.hisq_dslash(L, 1, nn, prec, nk2, lay, packed, vin, vout)
            # 100 timed launches, each between its own pair of events; median
            evs = [torch.cuda.Event(enable_timing=True) for _ in range(101)]
            evs[0].record(stream)
            for r in range(100):
                H.hisq_dslash(L, 1, nn, prec, nk2, lay, packed, vin, vout)
                evs[r + 1].record(stream)
            evs[-1].synchronize()
            ms = float(np.median([evs[r].elapsed_time(evs[r + 1]) for r in range(100)]))
            scale = 2 if prec == H.PREC_F64 else 1
            kname = {H.NAIK_R14: "r14", H.NAIK_R13: "r13", H.NAIK_R9: "r9"}.get(nk2, "full")
            byt = Vh * scale * (R.LINK_BYTES_F32[kname] + 2 * vec_b * nn)
            sweep["%s_n%d" % (tag, nn)] = {"ms": round(ms, 4), "GBps": round(byt / ms / 1e6, 1),
                                           "GFlops": round(Vh * R.FLOPS_PER_SITE_RHS * nn / ms / 1e6, 1)}
        result["dslash_sweep"] = sweep
        log("sweep", json.dumps(sweep))

        # the attainable-bandwidth reference (the paper's STREAM analogue): a
        # 1 GiB device-to-device copy, read + write bytes over time, median of 20
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(21)]
        evs[0].record(stream)
        for r in range(20):
            dst.copy_(src)
            evs[r + 1].record(stream)
        evs[-1].synchronize()
        cms = float(np.median([evs[r].elapsed_time(evs[r + 1]) for r in range(20)]))
        copy_gbps = 2 * (1 << 30) / cms / 1e6
        del src, dst
        result["hbm_copy_GBps"] = round(copy_gbps, 1)
        result["pct_of_copy"] = round(100 * dslash_gbps / copy_gbps, 1)
        log("copy %.1f GB/s" % copy_gbps)

    if not args.no_trace:
        # the full-matrix solve (even-odd reduction around the same CG) and one
        # bundle of 8 Z2 noise vectors through the eq. (2) estimator term
        # eta^dag M' M^-1 eta, at the headline shape
        eta_e, eta_o = W.make_noise(L, n, W.sources_seed(3, 1), "z2")
        ee, eo = dev(eta_e), dev(eta_o)
        if args.tile != "auto":
            H.hisq_set_tuning(1, nr, 64, order, rows)
            H.hisq_set_tuning_eo(*eo_tile)
        wsf = H.empty_bytes(H.hisq_trace_workspace_bytes(L, n, H.MODE_MIXED))
        H.solve_full(links, m, ee, eo, mode=H.MODE_MIXED, naik=naik, ws=wsf)  # warm
        torch.cuda.synchronize()
        tf = time.perf_counter()
        _, _, stf, inff = H.solve_full(links, m, ee, eo, mode=H.MODE_MIXED, naik=naik, ws=wsf)
        torch.cuda.synchronize()
        t_full = time.perf_counter() - tf
        tt = time.perf_counter()
        est, stt, inft = H.trace_estimate(links, m, (1,), ee, eo, mode=H.MODE_MIXED, naik=naik, ws=wsf)
        torch.cuda.synchronize()
        t_trace = time.perf_counter() - tt
        # the mu-derivative Dslash alone (FP64 links, temporal slots only):
        # 4 links of 144 B, each input once and each output once per site
        vo = torch.empty_like(ee)
        for _ in range(10):
            H.hisq_dslash_dmu(L, 1, n, 1, links.f64, ee, vo)
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(51)]
        evs[0].record(stream)
        for r in range(50):
            H.hisq_dslash_dmu(L, 1, n, 1, links.f64, ee, vo)
            evs[r + 1].record(stream)
        evs[-1].synchronize()
        dms = float(np.median([evs[r].elapsed_time(evs[r + 1]) for r in range(50)]))
        dmu_bytes = Vh * (4 * 144 + 2 * 48 * n)
        H.hisq_set_tuning(0)
        result["full_and_trace"] = {
            "full_solve_seconds": round(t_full, 4), "full_solve_status": stf,
            "full_solve_iters": inff["iters"],
            "trace_bundle_seconds": round(t_trace, 4), "trace_status": stt,
            "trace_terms_per_second": round(n / t_trace, 1),
            "trace_term_mean": [float(np.mean(est.real)), float(np.mean(est.imag))],
            "dslash_dmu1_f64_ms": round(dms, 4),
            "dslash_dmu1_f64_GBps": round(dmu_bytes / dms / 1e6, 1)}
        log("full/trace", json.dumps(result["full_and_trace"]))
        del wsf, ee, eo, vo

    if not args.no_config2:
        result["config2"] = config2_block(H, R, W, dev, stream)
    if not args.no_config2 and not args.no_paper_lattice:
        result["paper_lattice"] = paper_lattice_block(H, R, W, dev, stream)
        log("paper lattice", json.dumps(result["paper_lattice"]))
        log("config2", json.dumps(result["config2"]))

    if not args.no_backward:
        result["backward"] = backward_block(H, W, dev)
        log("backward", json.dumps(result["backward"]))

    if not args.no_batched:
        # config 4: six solves (three lattices x two masses, bundles of 3, 5, 8)
        # in one batched launch per CG phase, against the same six solved one by one
        probs, keep = [], []
        j = 0
        for Lb, nb in W.BATCHED_PROBLEMS:
            for mb in W.BATCHED_MASSES:
                Ub, Nb = W.make_links(Lb, 0.3, W.links_seed(4, j))
                lb = H.Links(Lb, dev(Ub), dev(Nb), f32=False, r14=True)
                bb = dev(W.make_sources(Lb, nb, W.sources_seed(4, j)))
                xb = torch.empty_like(bb)
                keep.append((Lb, nb, mb, lb, bb, xb))
                probs.append(H.Problem(H.geom(Lb), mb, nb, lb.f64.data_ptr(),
                                       lb.f32r14.data_ptr(), bb.data_ptr(), xb.data_ptr()))
                j += 1
        pb = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14)
        wsb = H.empty_bytes(H.hisq_batched_workspace_bytes(probs, H.MODE_MIXED))
        H.hisq_cg_solve_batched(probs, pb, wsb)  # tune + warm
        for Lb, nb, mb, lb, bb, xb in keep:
            H.solve(lb, mb, bb, mode=H.MODE_MIXED, naik=H.NAIK_R14)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        stb, infb = H.hisq_cg_solve_batched(probs, pb, wsb)
        torch.cuda.synchronize()
        t_batched = time.perf_counter() - tb
        pprof = H.hisq_default_params(mode=H.MODE_MIXED, naik=H.NAIK_R14, profile=1)
        _, infp = H.hisq_cg_solve_batched(probs, pprof, wsb)
        it_b = max(i.total_iters for i in infp)
        phase_ms = {name: round(infp[0].kernel_ms[c] / max(it_b, 1), 5)
                    for name, c in (("pupdate", H.K_PUPDATE), ("dslash_oe_norm", H.K_DSLASH_OE),
                                    ("dslash_eo_cg_epilogue", H.K_DSLASH_EO))}
        ts = time.perf_counter()
        sep_iters = []
        for Lb, nb, mb, lb, bb, xb in keep:
            _, st1, inf1 = H.solve(lb, mb, bb, mode=H.MODE_MIXED, naik=H.NAIK_R14)
            sep_iters.append(inf1["total_iters"])
        torch.cuda.synchronize()
        t_sep = time.perf_counter() - ts
        result["batched"] = {"workload": "6 solves: %s x m in %s, mixed r14, tol 1e-10"
                                         % (["%s n=%d" % ("x".join(map(str, Lb)), nb)
                                             for Lb, nb in W.BATCHED_PROBLEMS], list(W.BATCHED_MASSES)),
                             "status": stb, "batched_seconds": round(t_batched, 4),
                             "separate_seconds": round(t_sep, 4),
                             "speedup": round(t_sep / t_batched, 2),
                             "iters": [i.total_iters for i in infb], "separate_iters": sep_iters,
                             "per_iteration_kernel_ms": phase_ms,
                             "block_size": infb[0].block_size,
                             "rhs_per_thread": [i.rhs_per_thread for i in infb]}
        log("batched", json.dumps(result["batched"]))
        del keep, probs, wsb

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, W, R, L, U, N, b, n, m, Vh, iters, ms_per_step,
                                              x_head0)
    print(json.dumps(result), flush=True)

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB device-to-device copies done")


if __name__ == "__main__":
    main()
