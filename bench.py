"""Benchmark: cell updates/s of the SRHD patch step on one MI355X.

Workload: the off-centre ellipsoidal blast wave on a 256^3 periodic grid stored as 32,768 patches
of 8^3 cells with 3 ghost cells (ambient rho = 1, Theta = 1e-6; source rho = 1e-2, p = 1e4).  One
step is the whole hot path: the CFL time step (Eqs. 26-28, a device reduction), the ghost fill and
the fused MUSCL-Hancock patch step (inversions, PLM, half step, HLLC, update, limiter retries).
The timed run is K steps from the initial state (10 by default, as the workload specifies) with the
inputs resident in HBM.  The headline value is the mixed-precision step (FP32 reconstruction /
flux / update increment, FP64 inversion); the plain FP64 step is measured beside it on the same
inputs, with the per-field difference after one step.

Printed: one JSON line (metric, value, ...) with a `roofline` object for the dominant kernel (the
patch step) and a `cpu_baseline` object (the CPU oracle on a bounded sample of the same workload).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "cell updates/s on 1 MI355X: plain FP64 vs FP32+learned guess at stated rel err"
PEAK_ALU = 78.6e12       # FP64 vector FLOP/s (also the unpacked-FP32 rate; packed FP32 is off)
PEAK_HBM = 8.0e12        # bytes/s

# Algorithmic floating-point operations of the step (each +, -, *, /, sqrt counts 1, an FMA 2),
# counted from the formulas the kernel evaluates; per item:
FLOP_NEWTON_ITER = 48    # one Newton iteration (Eqs. 15, 16, A1, A2)
FLOP_INVERSION = 192     # exact L (error-free products + K=3 compensated sum), guess, recovery
FLOP_HALF_CELL = 570     # 15 slopes, 6 face states -> prim2cons + flux, half-step correction
FLOP_FACE = 105          # slope + face state + prim2cons + correction (inversion counted apart)
FLOP_RIEMANN = 260       # HLLC: 2 prim2cons, 2 fluxes, 4 signal speeds, HLL averages, star state
FLOP_UPDATE = 180        # flux differences, update, exact-L admissibility check of the output
HALF_CELLS, INTERFACES, OUT_CELLS = 896, 1728, 512
IO_BYTES_PER_PATCH = {                         # what one patch's step consumes and produces
    "padded": (1376 + 512) * 5 * 8,            # FP64 tile cells + FP64 output
    "grid": 1376 * 5 * 4 + 512 * 5 * (8 + 8 + 4),   # FP32 tile prims, cons in/out, prims out
}

# HBM bytes per launch of the mixed step kernel on this workload, from the rocprofv3
# FETCH_SIZE / WRITE_SIZE runs summarised in profiles/step_blast256_mixed.md; valid only for the
# kernel sources they were taken on (hash of the step kernel and its device header).
PROFILED_TRAFFIC = {"sources_sha256_16": "13c733f46a8f4176", "read": 3769.6e6, "write": 673.2e6,
                    "summary": "profiles/step_blast256_mixed.md"}


def step_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("srhd_step.hip", "srhd_device.hpp"):
        with open(os.path.join(ROOT, "paper_2012_11130_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_flops(n_patch, stats):
    """Algorithmic FLOPs of one step launch from its device counters."""
    attempts = n_patch + stats["n_retry"]
    return (attempts * (HALF_CELLS * FLOP_HALF_CELL + 2 * INTERFACES * FLOP_FACE
                        + INTERFACES * FLOP_RIEMANN + OUT_CELLS * FLOP_UPDATE)
            + stats["n_inversions"] * FLOP_INVERSION + stats["newton_iters"] * FLOP_NEWTON_ITER)


def summarize_profile(d, calib_mib):
    """Per-kernel table from rocprofv3 databases of three runs of this script under `d`:
    prof_trace (--kernel-trace --stats), prof_fetch (--pmc FETCH_SIZE), prof_write
    (--pmc WRITE_SIZE).  Byte counters are rescaled by what they read for the calibration copy
    (--calib-copy MiB read once and written once)."""
    import collections
    import glob
    import re
    import sqlite3

    def short(kn):
        m = re.search(r"srhd::\(anonymous namespace\)::(k_\w+(<\w+>)?)", kn)
        if m:
            return m.group(1)
        if "MulFunctor" in kn:
            return "calibration_copy"
        return kn.split("(")[0][-40:]

    def rows(sub, query):
        out = collections.defaultdict(list)
        for path in glob.glob(os.path.join(d, sub, "*results.db")):
            for kn, v in sqlite3.connect(path).execute(query):
                out[short(kn)].append(v)
        return out

    dur = rows("prof_trace", "select name, duration from kernels")
    fet = rows("prof_fetch", "select kernel_name, value from counters_collection")
    wri = rows("prof_write", "select kernel_name, value from counters_collection")
    avg = lambda v: sum(v) / len(v) if v else float("nan")
    kib = calib_mib * 1024.0
    ff = kib / avg(fet["calibration_copy"]) if fet.get("calibration_copy") else float("nan")
    fw = kib / avg(wri["calibration_copy"]) if wri.get("calibration_copy") else float("nan")
    print("calibration: FETCH_SIZE x %.3f, WRITE_SIZE x %.3f (copy of %d MiB)" % (ff, fw, calib_mib))
    print("| kernel | calls | avg us | HBM read MB/launch | HBM write MB/launch |")
    print("|---|---|---|---|---|")
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        print("| %s | %d | %.1f | %.1f | %.1f |" % (k, len(dur[k]), avg(dur[k]) / 1e3,
                                                  avg(fet.get(k, [])) * ff * 1.024e-3,
                                                  avg(wri.get(k, [])) * fw * 1.024e-3))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="print the per-kernel table of rocprofv3 runs under DIR and exit")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cells", type=int, default=256, help="cells per side of the blast grid")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--conversion", type=int, default=100_000_000,
                    help="states of the standalone conversion batch (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--path", choices=("grid", "padded"), default="grid",
                    help="grid: gather-mode step chain (default); padded: CFL + fill + step")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="MiB of a plain elementwise copy run once before the steps, as the "
                         "calibration kernel for hardware byte counters (0 = none)")
    return ap.parse_args()


def main():
    args = parse()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.calib_copy or 512)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2012_11130_amd import srhd as S

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------------- inputs (resident in HBM)
    t0 = time.time()
    g = W.blast(args.cells, seed=1003, order="morton")
    P = g.n_patch
    n_cells = P * 512
    prim = torch.from_numpy(g.prim).to(dev)                            # [P][5][8][8][8]
    prim_soa = prim.reshape(P, 5, 512).permute(1, 0, 2).contiguous().reshape(5, -1)
    cons_soa = S.srhd_prim2cons(prim_soa)
    cons0 = cons_soa.reshape(5, P, 512).permute(1, 0, 2).contiguous().reshape(P, 5, 8, 8, 8)
    nb = torch.from_numpy(g.neighbor).to(dev)
    dh = g.dh_lev
    N = 14
    pad = torch.empty((P, 5, N, N, N), dtype=torch.float64, device=dev)
    bufs = [torch.empty_like(cons0), torch.empty_like(cons0)]
    dt = torch.empty(1, dtype=torch.float64, device=dev)
    stats = S.new_stats(dev)
    torch.cuda.synchronize()
    print("# inputs ready in %.1f s (%d patches, %d cells)" % (time.time() - t0, P, n_cells),
          file=sys.stderr, flush=True)
    if args.calib_copy:
        src = torch.ones(args.calib_copy << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)          # reads and writes calib_copy MiB once each
        torch.cuda.synchronize()
        del src, dst

    def run_padded(prec, n_steps, time_kernel=False):
        """n_steps from the initial state with CFL kernel + ghost fill + padded step."""
        bufs[0].copy_(cons0)
        cur = 0
        S.srhd_stats_reset(stats)
        evs = []
        e_start = torch.cuda.Event(enable_timing=True)
        e_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e_start.record(stream)
        for _ in range(n_steps):
            S.srhd_cfl_dt(bufs[cur], dh, 0.5, dt_lev=dt)
            S.srhd_fill_ghosts(bufs[cur], nb, 3, padded=pad)
            if time_kernel:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            S.srhd_fluid_step(pad, dt, dh, out=bufs[1 - cur], prec=prec, stats=stats)
            if time_kernel:
                b.record(stream)
                evs.append((a, b))
            cur = 1 - cur
        e_end.record(stream)
        torch.cuda.synchronize()
        ms = e_start.elapsed_time(e_end)
        kms = [a.elapsed_time(b) for a, b in evs]
        return ms, kms, S.stats_dict(stats), bufs[cur]

    pbufs = {}

    def run_grid(prec, n_steps, time_kernel=False):
        """n_steps from the initial state with the gather-mode step: each step is one kernel
        that reads ghosts from neighbour interiors and returns the next S_max; the entry
        inversion of the initial state is inside the timed region."""
        pdt = S.prims_dtype(prec)
        key = str(pdt)
        if key not in pbufs:
            pbufs[key] = [torch.empty(cons0.shape, dtype=pdt, device=dev) for _ in range(2)]
        pb = pbufs[key]
        sb = [torch.empty(1, dtype=torch.int64, device=dev) for _ in range(2)]
        bufs[0].copy_(cons0)
        cur = 0
        S.srhd_stats_reset(stats)
        evs = []
        e_start = torch.cuda.Event(enable_timing=True)
        e_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e_start.record(stream)
        S.srhd_grid_prims(bufs[0], prec=prec, prims=pb[0], smax_bits=sb[0])
        for _ in range(n_steps):
            if time_kernel:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            S.srhd_fluid_step_grid(bufs[cur], pb[cur], nb, dh, smax_in=sb[cur], c_cfl=0.5,
                                   cons_out=bufs[1 - cur], prims_out=pb[1 - cur],
                                   smax_out=sb[1 - cur], prec=prec, stats=stats)
            if time_kernel:
                b.record(stream)
                evs.append((a, b))
            cur = 1 - cur
        e_end.record(stream)
        torch.cuda.synchronize()
        ms = e_start.elapsed_time(e_end)
        kms = [a.elapsed_time(b) for a, b in evs]
        return ms, kms, S.stats_dict(stats), bufs[cur]

    run = run_grid if args.path == "grid" else run_padded

    def measure(prec):
        if args.warmup:
            run(prec, args.warmup)
        ms, kms, st, final = run(prec, args.steps, time_kernel=True)
        return ms, kms, st, final.clone()

    ms_mx, kms_mx, st_mx, fin_mx = measure(S.PREC_MIXED)
    print("# mixed: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
          % (ms_mx, args.steps, float(np.mean(kms_mx)), st_mx), file=sys.stderr, flush=True)
    value = n_cells * args.steps / (ms_mx * 1e-3)

    # per-field difference of one mixed step against one FP64 step from the same state
    res = {}
    if not args.no_fp64:
        ms_64, kms_64, st_64, fin_64 = measure(S.PREC_FP64)
        print("# fp64: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
              % (ms_64, args.steps, float(np.mean(kms_64)), st_64), file=sys.stderr, flush=True)
        S.srhd_cfl_dt(cons0, dh, 0.5, dt_lev=dt)
        S.srhd_fill_ghosts(cons0, nb, 3, padded=pad)
        o64 = S.srhd_fluid_step(pad, dt, dh, prec=S.PREC_FP64).cpu().numpy()
        omx = S.srhd_fluid_step(pad, dt, dh, prec=S.PREC_MIXED).cpu().numpy()
        mscale = max(float(np.max(np.sqrt((o64[:, 1:4] ** 2).sum(axis=1)))), 1e-300)
        err1 = {"D": float(np.max(np.abs(omx[:, 0] / o64[:, 0] - 1))),
                "Et": float(np.max(np.abs(omx[:, 4] / o64[:, 4] - 1))),
                "M": float(np.max(np.abs(omx[:, 1:4] - o64[:, 1:4]))) / mscale}
        a, b = fin_mx.cpu().numpy(), fin_64.cpu().numpy()
        ms2 = max(float(np.max(np.sqrt((b[:, 1:4] ** 2).sum(axis=1)))), 1e-300)
        errK = {"D": float(np.max(np.abs(a[:, 0] / b[:, 0] - 1))),
                "Et": float(np.max(np.abs(a[:, 4] / b[:, 4] - 1))),
                "M": float(np.max(np.abs(a[:, 1:4] - b[:, 1:4]))) / ms2}
        res["fp64"] = {"value": n_cells * args.steps / (ms_64 * 1e-3), "ms_per_step": ms_64 / args.steps,
                       "step_kernel_ms": float(np.mean(kms_64)), "stats": st_64}
        res["mixed_vs_fp64_rel_err"] = {"one_step": err1, "after_%d_steps" % args.steps: errK}

    # ---------------------------------------------------------------- roofline of the step kernel
    kavg = float(np.mean(kms_mx)) * 1e-3
    flops = step_flops(P, {k: v / args.steps for k, v in st_mx.items()})
    traffic = None
    if (step_sources_hash() == PROFILED_TRAFFIC["sources_sha256_16"] and args.cells == 256
            and args.path == PROFILED_TRAFFIC.get("path", "padded")):
        traffic = PROFILED_TRAFFIC["read"] + PROFILED_TRAFFIC["write"]
    roofline = {"bound": "alu", "achieved": flops / kavg / 1e12, "peak": PEAK_ALU / 1e12,
                "unit": "TFLOP/s", "frac": flops / kavg / PEAK_ALU, "traffic": traffic,
                "kernel": "k_step<float,%s> (mixed)" % ("gather" if args.path == "grid" else "padded"),
                "launch_ms": kavg * 1e3,
                "hbm_GBps_algorithmic": IO_BYTES_PER_PATCH[args.path] * P / kavg / 1e9,
                "flops_per_launch": flops}

    # ---------------------------------------------------------------- standalone conversions
    if args.conversion:
        n = args.conversion
        gen = torch.Generator(device=dev)
        gen.manual_seed(1002)
        lr = torch.empty(n, dtype=torch.float64, device=dev)

        def logu(lo, hi):
            return torch.exp(lr.uniform_(math.log(lo), math.log(hi), generator=gen))
        cp = torch.empty((5, n), dtype=torch.float64, device=dev)
        cp[0] = logu(1e-6, 1e6)
        th = logu(1e-8, 1e4)
        gam = logu(1.0, 1e6)
        dirn = torch.randn((3, n), dtype=torch.float64, device=dev, generator=gen)
        dirn /= torch.sqrt((dirn * dirn).sum(dim=0))
        cp[1:4] = torch.sqrt((gam - 1) * (gam + 1)) * dirn
        cp[4] = cp[0] * th
        del th, gam, dirn, lr
        cc = S.srhd_prim2cons(cp)
        out = torch.empty_like(cc)
        stt = torch.empty(n, dtype=torch.int8, device=dev)
        conv = {}
        for name, src in (("fp64", cc), ("fp32", cc.float())):
            o = out if name == "fp64" else torch.empty_like(src)
            S.srhd_cons2prim(src, prim=o, status=stt)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record(stream)
            for _ in range(reps):
                S.srhd_cons2prim(src, prim=o, status=stt)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps * 1e-3
            bpe = 2 * 5 * src.element_size() + 1
            conv[name] = {"states_per_s": n / t, "ms": t * 1e3,
                          "hbm_frac": n * bpe / t / PEAK_HBM,
                          "unphysical_frac": float((stt == 1).float().mean().item())}
        res["conversion_batch_1e8"] = conv
        del cp, cc, out, stt

    # ---------------------------------------------------------------- CPU baseline (the oracle)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        cons_h = cons0.cpu().numpy()
        threads = O.num_threads()
        # calibrate on 64 patches, then a sample sized for about cpu_seconds of wall time
        rng = np.random.default_rng(0)

        def oracle_pass(idx):
            t = time.perf_counter()
            dt_o, _, _ = O.cfl_dt(cons_h[idx], None, dh, 0.5)
            pad_o = O.fill_ghosts(cons_h, g.neighbor[idx], 3)
            O.fluid_step(pad_o, dt_o, dh)
            return time.perf_counter() - t
        probe = rng.choice(P, 64, replace=False)
        tp = oracle_pass(probe)
        m = int(min(P, max(64, args.cpu_seconds / max(tp, 1e-6) * 64)))
        idx = np.sort(rng.choice(P, m, replace=False))
        tc = oracle_pass(idx)
        cpu = {"value": m * 512 / tc, "unit": "cell updates/s", "cores": threads,
               "kind": "oracle",
               "sample": "%d random patches (%d cells) of the 256^3 blast, one FP64 step from "
                         "the initial state: CFL + ghost fill + MUSCL-Hancock step, %.1f s" % (m, m * 512, tc)}

    line = {
        "metric": METRIC, "value": value, "unit": "cell updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_mx / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "blast_%d^3_periodic_%dpatches_mixed_precision" % (args.cells, P),
                   "path": args.path, "patch_order": "morton",
                   "cells": n_cells, "patches": P, "ghost": 3, "riemann": "HLLC",
                   "limiter_theta": 1.5, "guess": "analytic", "steps_per_run": args.steps},
        "roofline": roofline, "cpu_baseline": cpu, "mixed_stats": st_mx,
    }
    line.update(res)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
