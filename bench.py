"""Benchmark: cell updates/s of the SRHD patch step on one MI355X.

Workload: the off-centre ellipsoidal blast wave on a 256^3 periodic grid stored as 32,768 patches
of 8^3 cells with 3 ghost cells (ambient rho = 1, Theta = 1e-6; source rho = 1e-2, p = 1e4).  One
step is the whole hot path: the CFL time step (Eqs. 26-28, a device reduction), the ghost fill and
the fused MUSCL-Hancock patch step (inversions, PLM, half step, HLLC, update, limiter retries).
The timed run is K steps from the initial state (10 by default, as the workload specifies) with the
inputs resident in HBM.  The headline value is the mixed-precision step (FP32 reconstruction /
flux / update increment, FP64 inversion); the plain FP64 step is measured beside it on the same
inputs, with the per-field difference after one step.  With trained weights present
(paper_2012_11130_amd/mlp_guess.npz) the headline step uses the learned Newton guess and the
mixed step with the analytic guess is measured beside it; Newton iterations per inversion and the
fallback rate of each are reported.

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
FLOP_INV_REST = 58       # an inversion besides L and its iterations: guess, recovery
FLOP_L_EXACT = 134       # L from error-free products and the K=3 compensated sum (FP64 bulk)
FLOP_L_PLAIN = 14        # L from the plain sum of the exact products: the branch the FP32-bulk
                         # kernels take where every lane of a wavefront has cond <= 1024
FLOP_HALF_CELL = 570     # 15 slopes, 6 face states -> prim2cons + flux, half-step correction
FLOP_FACE = 105          # slope + face state + prim2cons + correction (inversion counted apart)
FLOP_RIEMANN = 260       # HLLC: 2 prim2cons, 2 fluxes, 4 signal speeds, HLL averages, star state
FLOP_UPDATE = 46         # flux differences and update of an output cell (its L counted apart)
FLOP_MLP_VALU = 1088     # learned guess, VALU part: features and standardisation (~20), layer 1
                         # (64 x 3 FMA = 384), 128 SiLU (exp, add, reciprocal, multiply = 512),
                         # layer 3 (64 FMA = 128), partner-lane sum and exponential (~44)
MFMA_FLOP_MLP = 2 * 64 * 64   # layer 2 on the matrix cores per evaluation
HALF_CELLS, INTERFACES, OUT_CELLS = 896, 1728, 512
IO_BYTES_PER_PATCH = {                         # what one patch's step consumes and produces
    "padded": (1376 + 512) * 5 * 8,            # FP64 tile cells + FP64 output
    "grid": 1376 * 5 * 4 + 512 * 5 * (8 + 8 + 4),   # FP32 tile prims, cons in/out, prims out
}

# Hardware counters of the step kernels on this workload (rocprofv3 FETCH_SIZE / WRITE_SIZE,
# rescaled by a plain copy's reading, and the VALU instruction counters: FP64 + FP32 flops with an
# FMA as 2), summarised in the profile named below; valid only for the kernel sources they were
# taken on (hash of the files that make up the step kernels).  headline: one step of the
# mixed-precision chain with the learned guess, gather layout, two-workgroup register variant --
# the kernel without the network (2,307.8 us), the learned pass beside it on the second stream
# (232.3 us, overlapped), the list (9.9 us), the counter prologue (4.2 us) and the guard's empty
# FP64 pass (6.4 us); ms is their sum without the overlapped pass, valu_issue that of the first
# kernel.  fp64: the FP64 step kernel (with its prologue).
PROFILED = {"sources_sha256_16": "f0fd3add91e52df2", "path": "grid",
            "summary": "profiles/step_blast256_counters.md",
            "headline": {"ms": 2.3283, "read": 1314.5e6, "write": 1020.5e6,
                         "flops": 1.711e10 + 4.524e10 + 4.165e7 + 1.929e8, "valu_issue": 0.878},
            "fp64": {"ms": 5.4791, "read": 1903.0e6, "write": 1345.4e6, "flops": 1.185e11,
                     "valu_issue": 0.626}}
STEP_SOURCES = ("srhd_step_impl.hpp", "srhd_step_mixed.hip", "srhd_step_fp64.hip", "srhd_step.hip",
                "srhd_device.hpp", "srhd_mlp.hpp")


def _finite(v):
    """The JSON line with every non-finite float replaced by null (strict JSON has no NaN)."""
    if isinstance(v, dict):
        return {k: _finite(x) for k, x in v.items()}
    if isinstance(v, (list, tuple)):
        return [_finite(x) for x in v]
    if isinstance(v, float) and not math.isfinite(v):
        return None
    return v


def step_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2012_11130_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def step_flops(n_patch, stats, fp32_bulk, gather):
    """Algorithmic VALU FLOPs of one step launch from its device counters, with L at the cost
    of the branch the kernel takes: the plain sum of the exact products in the FP32-bulk kernels
    (their rare compensated sums, in wavefronts holding a lane with cond > 1024, are not
    counted), the compensated sum in FP64.  A gather-layout output inversion reuses the L of its
    cell's check.  The learned guess's VALU work counts per network evaluation (n_mlp), its
    matrix-core work apart."""
    L = FLOP_L_PLAIN if fp32_bulk else FLOP_L_EXACT
    attempts = n_patch + stats["n_retry"]
    out_inv = OUT_CELLS * n_patch if gather else 0
    return (attempts * (HALF_CELLS * FLOP_HALF_CELL + 2 * INTERFACES * FLOP_FACE
                        + INTERFACES * FLOP_RIEMANN + OUT_CELLS * (FLOP_UPDATE + L))
            + stats["n_inversions"] * FLOP_INV_REST + (stats["n_inversions"] - out_inv) * L
            + stats.get("n_mlp", 0) * FLOP_MLP_VALU + stats["newton_iters"] * FLOP_NEWTON_ITER)


def summarize_profile(d, calib_mib):
    """Per-kernel tables from rocprofv3 databases of runs of this script under `d`: prof_trace
    (--kernel-trace --stats) and any number of counter runs prof_<name> (--pmc ...).  Byte
    counters are rescaled by what they read for the calibration copy (--calib-copy MiB read once
    and written once); instruction counters are per launch, summed over the whole device."""
    import collections
    import glob
    import re
    import sqlite3

    def short(kn):
        m = re.search(r"srhd::\(anonymous namespace\)::(k_\w+(<[^>]*>)?)", kn)
        if m:
            return m.group(1).replace(" ", "")
        if "neg_kernel" in kn:
            return "calibration_copy"
        return kn.split("(")[0][-40:]

    dur = collections.defaultdict(list)
    info = {}
    for path in glob.glob(os.path.join(d, "prof_trace", "*results.db")):
        db = sqlite3.connect(path)
        for kn, v in db.execute("select name, duration from kernels"):
            dur[short(kn)].append(v)
    cnt = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in glob.glob(os.path.join(d, "prof_*", "*results.db")):
        if os.sep + "prof_trace" + os.sep in path:
            continue
        db = sqlite3.connect(path)
        q = ("select kernel_name, counter_name, value, vgpr_count, accum_vgpr_count, sgpr_count, "
             "lds_block_size, scratch_size from counters_collection")
        for kn, cn, v, vg, ag, sg, lds, scr in db.execute(q):
            k = short(kn)
            cnt[k][cn].append(v)
            info[k] = (vg, ag, sg, lds, scr)
    avg = lambda v: sum(v) / len(v) if v else float("nan")
    kib = calib_mib * 1024.0
    cal = cnt.get("calibration_copy", {})
    ff = kib / avg(cal["FETCH_SIZE"]) if cal.get("FETCH_SIZE") else float("nan")
    fw = kib / avg(cal["WRITE_SIZE"]) if cal.get("WRITE_SIZE") else float("nan")
    print("calibration: FETCH_SIZE x %.3f, WRITE_SIZE x %.3f (copy of %d MiB)" % (ff, fw, calib_mib))
    print("| kernel | calls | avg us | HBM read MB/launch | HBM write MB/launch | arch VGPR | acc VGPR | SGPR | LDS B | scratch B |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for k in sorted(dur, key=lambda k: -sum(dur[k])):
        c = cnt.get(k, {})
        vg, ag, sg, lds, scr = info.get(k, ("", "", "", "", ""))
        print("| %s | %d | %.1f | %.1f | %.1f | %s | %s | %s | %s | %s |"
              % (k, len(dur[k]), avg(dur[k]) / 1e3, avg(c.get("FETCH_SIZE", [])) * ff * 1.024e-3,
                 avg(c.get("WRITE_SIZE", [])) * fw * 1.024e-3, vg, ag, sg, lds, scr))
    # VALU work from the instruction counters (64 lanes per instruction, FMA = 2 flops)
    f64 = ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64")
    f32 = ("SQ_INSTS_VALU_FMA_F32", "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_TRANS_F32")
    rows = [k for k in sorted(dur, key=lambda k: -sum(dur[k])) if "SQ_INSTS_VALU" in cnt.get(k, {})
            or "SQ_INSTS_VALU_FMA_F64" in cnt.get(k, {})]
    if rows:
        issue_peak = 256 * 4 * 2.4e9 / 4      # wave64 VALU instructions/s (4 SIMDs x 16 lanes per CU)
        print()
        print("| kernel | FP64 flops/launch | FP32 flops/launch | VALU TFLOP/s (FP64+FP32) | of 78.6 | VALU instr/launch | VALU issue of peak | LDS instr/launch | LDS bank-conflict cycles / LDS active cycles |")
        print("|---|---|---|---|---|---|---|---|---|")
        for k in rows:
            c = cnt[k]
            t = avg(dur[k]) * 1e-9
            def fl(names):
                if not all(n in c for n in names):
                    return float("nan")
                return 64 * (2 * avg(c[names[0]]) + avg(c[names[1]]) + avg(c[names[2]]) + avg(c[names[3]]))
            a64, a32 = fl(f64), fl(f32)
            vi = avg(c.get("SQ_INSTS_VALU", []))
            act = avg(c.get("SQ_LDS_IDX_ACTIVE", []))
            bc = avg(c.get("SQ_LDS_BANK_CONFLICT", [])) / act if act > 0 else float("nan")
            print("| %s | %.3e | %.3e | %.2f | %.1f %% | %.3e | %.1f %% | %.3e | %.3f |"
                  % (k, a64, a32, (a64 + a32) / t / 1e12, 100 * (a64 + a32) / t / PEAK_ALU, vi,
                     100 * vi / t / issue_peak, avg(c.get("SQ_INSTS_LDS", [])), bc))
    # where the wavefronts spend their time: fractions of SQ_WAVE_CYCLES (summed over waves)
    wn = ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS", "SQ_ACTIVE_INST_ANY",
          "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_VMEM")
    rows = [k for k in sorted(dur, key=lambda k: -sum(dur[k]))
            if all(n in cnt.get(k, {}) for n in ("SQ_WAVE_CYCLES",) + wn)]
    if rows:
        print()
        print("| kernel | waiting (any) | waiting on an instruction | waiting on LDS | issuing (any) | VALU | LDS | VMEM |")
        print("|---|---|---|---|---|---|---|---|")
        for k in rows:
            c = cnt[k]
            wc = avg(c["SQ_WAVE_CYCLES"])
            print("| %s | %s |" % (k, " | ".join("%.1f %%" % (100 * avg(c[n]) / wc) for n in wn)))


def run_jet(args, S, W, dev, stream, guess, guess_name):
    """The multi-level jet list: padded patches whose ghosts hold the analytic initial state,
    one step = the CFL reduction + one launch of the step over every patch, under the schedule
    the autotuner picks.  Every timed step starts from the same initial state."""
    import torch
    pl = W.jet_patch_list(n_patch=args.jet)
    P = pl["corner"].shape[0]
    dh = pl["dh_lev"]
    states = S.srhd_prim2cons(torch.from_numpy(W.jet_states().T.copy()).to(dev)).T.cpu().numpy()
    lab = W.jet_labels_torch(pl, dev)
    pad = W.assemble_labeled(lab, states)
    del lab
    level = torch.from_numpy(pl["level"]).to(dev)
    interior = pad[:, :, 3:11, 3:11, 3:11].contiguous()
    dt = torch.empty(len(dh), dtype=torch.float64, device=dev)
    out = torch.empty((P, 5, 8, 8, 8), dtype=torch.float64, device=dev)
    stats = S.new_stats(dev)
    S.srhd_cfl_dt(interior, dh, 0.5, dt_lev=dt)
    res = {"patches": P, "cells": P * 512, "levels": [int((pl["level"] == l).sum()) for l in range(len(dh))]}
    for name, prec, g in (("mixed", S.PREC_MIXED, guess), ("fp64", S.PREC_FP64, None)):
        if args.sched != "auto":
            gr, ch, oc = (int(v) for v in args.sched.split(","))
            sch, table = S.Sched(gr, ch, dev, occupancy=0 if prec == S.PREC_FP64 else oc), []
        else:
            sch, table = S.srhd_autotune_step(pad, dt, dh, level=level, out=out, prec=prec, guess=g,
                                              reps=2)
        for _ in range(args.warmup):
            S.srhd_cfl_dt(interior, dh, 0.5, dt_lev=dt)
            S.srhd_fluid_step(pad, dt, dh, level=level, out=out, prec=prec, guess=g, sched=sch)
        S.srhd_stats_reset(stats)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ks = []
        e0.record(stream)
        for _ in range(args.steps):
            S.srhd_cfl_dt(interior, dh, 0.5, dt_lev=dt)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            S.srhd_fluid_step(pad, dt, dh, level=level, out=out, prec=prec, guess=g, sched=sch,
                              stats=stats)
            b.record(stream)
            ks.append((a, b))
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        st = S.stats_dict(stats)
        inv = max(st["n_inversions"], 1)
        res[name] = {"value": P * 512 / (ms * 1e-3), "unit": "cell updates/s", "ms_per_step": ms,
                     "step_kernel_ms": float(np.mean([x.elapsed_time(y) for x, y in ks])),
                     "guess": guess_name if g is not None else "analytic",
                     "schedule": {"groups": sch.groups, "chunk": sch.chunk, "occupancy": sch.occupancy},
                     "autotune_ms": [[t[0], t[1], t[2], round(t[3], 3)] for t in table],
                     "iters_per_inversion": st["newton_iters"] / inv,
                     "fallback_rate": st["n_fallback"] / inv,
                     "retries_per_step": st["n_retry"] / args.steps,
                     "fp64_patches_per_step": st["n_fp64_patch"] / args.steps}
        print("# jet %s: %.2f ms per step, schedule %s" % (name, ms, sch), file=sys.stderr, flush=True)
    # per-field difference of one step from the initial state against the FP64 step, with the
    # precision guard (the default) and without it (kappa_max = 0: the FP32 bulk everywhere)
    S.srhd_cfl_dt(interior, dh, 0.5, dt_lev=dt)
    o64 = S.srhd_fluid_step(pad, dt, dh, level=level, prec=S.PREC_FP64)
    omx = S.srhd_fluid_step(pad, dt, dh, level=level, prec=S.PREC_MIXED, guess=guess)
    res["mixed_vs_fp64_rel_err_one_step"] = field_err_torch(omx, o64)
    del omx
    ooff = S.srhd_fluid_step(pad, dt, dh, level=level, prec=S.PREC_MIXED, guess=guess, kappa_max=0.0)
    res["mixed_unguarded_vs_fp64_rel_err_one_step"] = field_err_torch(ooff, o64)
    print("# jet one step vs FP64: guarded %s, unguarded %s"
          % (res["mixed_vs_fp64_rel_err_one_step"], res["mixed_unguarded_vs_fp64_rel_err_one_step"]),
          file=sys.stderr, flush=True)
    del ooff, o64, pad, interior, out
    torch.cuda.empty_cache()
    return res


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_conversion_parity(O, samples, threads):
    """Oracle inversion of the sampled conserved states of each variant ({name: (cons [5][m],
    GPU prims [5][m] as FP64, GPU status [m])}): oracle states/s, identical UNPHYSICAL flags and
    the GPU's per-field error (rho, p pointwise relative, U normwise per state) over the states
    both accept."""
    out = {}
    for name, (cons, gp, gst) in samples.items():
        c = np.ascontiguousarray(cons.astype(np.float64))
        t = time.perf_counter()
        ref, ost, _ = O.cons2prim(c)
        dt_ = time.perf_counter() - t
        ok = (ost != 1) & (gst != 1)
        g, r = gp[:, ok], ref[:, ok]
        un = np.maximum(np.sqrt((r[1:4] ** 2).sum(axis=0)), 1e-300)
        out[name] = {"states": int(c.shape[1]), "oracle_states_per_s": c.shape[1] / dt_,
                     "cores": threads,
                     "unphysical_flags_equal": bool(np.array_equal(ost == 1, gst == 1)),
                     "rho": float(np.max(np.abs(g[0] / r[0] - 1))),
                     "p": float(np.max(np.abs(g[4] / r[4] - 1))),
                     "U": float(np.max(np.max(np.abs(g[1:4] - r[1:4]), axis=0) / un))}
    return out


def roundtrip_by_cond(prim, gen, status, cond, u):
    """Round-trip error of an inversion (prim [5][n], any float type) against the generating
    primitives gen [5][n] (FP64), per decade of Eq. 20's condition number: rho and p pointwise
    relative, U normwise per state; over the states not flagged unphysical.  Each bin reports
    the count, the median and largest error per field and the largest error / (cond u)."""
    import torch
    ok = status != 1
    w = prim.double()
    er = (w[0] / gen[0] - 1).abs()
    ep = (w[4] / gen[4] - 1).abs()
    un = torch.sqrt((gen[1:4] ** 2).sum(dim=0)).clamp_min(1e-300)
    eu = (w[1:4] - gen[1:4]).abs().amax(dim=0) / un
    lg = torch.floor(torch.log10(cond.clamp(1.0, 1e30)))
    bins = []
    for b in range(0, 31):
        m = ok & (lg == b)
        c = int(m.sum().item())
        if c == 0:
            continue
        row = {"cond_decade": "1e%d" % b, "states": c}
        worst = 0.0
        for name, e in (("rho", er), ("p", ep), ("U", eu)):
            v = e[m]
            row[name + "_median"] = float(v.median().item())
            row[name + "_max"] = float(v.max().item())
            worst = max(worst, float((v / (cond[m] * u)).max().item()))
        row["max_err_over_cond_u"] = worst
        bins.append(row)
    del er, ep, eu, lg
    return bins


def field_err_torch(x, ref):
    """Per-field difference of two step outputs [P][5][8][8][8] on the device: D and Et pointwise
    relative, the momentum against the largest |M| of ref (the parity tests' metric)."""
    import torch
    e = {}
    for f, name in ((0, "D"), (4, "Et")):
        e[name] = float((x[:, f] / ref[:, f] - 1).abs().max().item())
    ms = float(torch.sqrt((ref[:, 1:4] ** 2).sum(dim=1)).max().item())
    e["M"] = float((x[:, 1:4] - ref[:, 1:4]).abs().max().item()) / max(ms, 1e-300)
    e["non_finite_cells"] = int((~torch.isfinite(x)).any(dim=1).sum().item())
    return e


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
    ap.add_argument("--jet", type=int, default=400_000,
                    help="patches of the multi-level jet list measured beside the headline (0 = skip)")
    ap.add_argument("--path", choices=("grid", "padded"), default="grid",
                    help="grid: gather-mode step chain (default); padded: CFL + fill + step")
    ap.add_argument("--guess", choices=("learned", "analytic"), default="learned",
                    help="Newton guess of the headline mixed step (learned needs the weights file)")
    ap.add_argument("--weights", default=None, help="weights of the learned guess (.npz)")
    ap.add_argument("--sched", default="auto",
                    help="launch schedule of the step: auto (the autotuner's choice per "
                         "configuration) or groups,chunk,occupancy")
    ap.add_argument("--no-vl", dest="vl", action="store_false",
                    help="skip the VL integrator's runs")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the original-scheme and polytropic-EoS runs")
    ap.add_argument("--no-amr", dest="amr", action="store_false",
                    help="skip the two-level AMR cycle")
    ap.add_argument("--only-headline", action="store_true",
                    help="measure the headline configuration only (no analytic-guess, "
                         "configured-input or FP32-inversion comparisons)")
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
        print("bench.py measures one GPU only: the step has no multi-GPU path (each GPU would "
              "own a contiguous range of the Morton-ordered patch list); run with --gpus 1",
              file=sys.stderr)
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
        torch.neg(src, out=dst)               # reads and writes calib_copy MiB once each (the only
                                              # negation kernel of the run)
        torch.cuda.synchronize()
        del src, dst

    def run_padded(prec, n_steps, time_kernel=False, guess=None, sched=None, integrator=0):
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
            S.srhd_fluid_step(pad, dt, dh, out=bufs[1 - cur], prec=prec, stats=stats, guess=guess,
                              sched=sched, integrator=integrator)
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

    def run_grid(prec, n_steps, time_kernel=False, guess=None, sched=None, integrator=S.MHM):
        """n_steps from the initial state with the gather-mode step: each step is one kernel
        that reads ghosts from neighbour interiors and returns the next S_max; the entry
        inversion of the initial state is inside the timed region."""
        pdt = S.prims_dtype(prec)
        key = str(pdt)
        if key not in pbufs:
            pbufs[key] = [torch.empty(cons0.shape, dtype=pdt, device=dev) for _ in range(2)]
        pb = pbufs[key]
        sb = [torch.empty(1, dtype=torch.int64, device=dev) for _ in range(2)]
        # the learned guess's network masks travel with the state (the split's list before each
        # step, and its learned kernel beside the other on a second stream)
        learned = guess is not None and guess.kind == S.GUESS_MLP
        nmask = [S.new_net_mask(cons0.shape[0], dev) if learned else None for _ in range(2)]
        bufs[0].copy_(cons0)
        cur = 0
        S.srhd_stats_reset(stats)
        evs = []
        e_start = torch.cuda.Event(enable_timing=True)
        e_end = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e_start.record(stream)
        S.srhd_grid_prims(bufs[0], prec=prec, prims=pb[0], smax_bits=sb[0], guess=guess,
                          net_mask=nmask[0])
        for _ in range(n_steps):
            if time_kernel:
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
            S.srhd_fluid_step_grid(bufs[cur], pb[cur], nb, dh, smax_in=sb[cur], c_cfl=0.5,
                                   cons_out=bufs[1 - cur], prims_out=pb[1 - cur],
                                   smax_out=sb[1 - cur], prec=prec, stats=stats, guess=guess,
                                   sched=sched, net_in=nmask[cur], net_out=nmask[1 - cur],
                                   integrator=integrator)
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

    def tune(prec, guess):
        """The autotuner's schedule for this configuration, on the initial state."""
        if args.sched != "auto":
            gr, ch, oc = (int(v) for v in args.sched.split(","))
            if prec == S.PREC_FP64:
                oc = 0
            return S.Sched(gr, ch, dev, occupancy=oc), []
        if args.path == "grid":
            mask = S.new_net_mask(cons0.shape[0], dev)
            prims, smax = S.srhd_grid_prims(cons0, prec=prec, guess=guess, net_mask=mask)
            sch, table = S.srhd_autotune_step_grid(cons0, prims, nb, dh, smax_in=smax, prec=prec,
                                                   guess=guess, reps=2, net_in=mask)
        else:
            S.srhd_cfl_dt(cons0, dh, 0.5, dt_lev=dt)
            S.srhd_fill_ghosts(cons0, nb, 3, padded=pad)
            sch, table = S.srhd_autotune_step(pad, dt, dh, prec=prec, guess=guess, reps=2)
        return sch, [[t[0], t[1], t[2], round(t[3], 4)] for t in table]

    schedules = {}

    def measure(prec, guess=None, name=""):
        sch, table = tune(prec, guess)
        schedules[name] = {"groups": sch.groups, "chunk": sch.chunk, "occupancy": sch.occupancy,
                           "autotune_ms": table}
        if args.warmup:
            run(prec, args.warmup, guess=guess, sched=sch)
        ms, kms, st, final = run(prec, args.steps, time_kernel=True, guess=guess, sched=sch)
        return ms, kms, st, final.clone()

    def newton_summary(st):
        inv = max(st["n_inversions"], 1)
        return {"iters_per_inversion": st["newton_iters"] / inv,
                "fallback_rate": st["n_fallback"] / inv, "noconv": st["n_noconv"]}

    mlp = None
    if args.guess == "learned":
        from paper_2012_11130_amd import mlp_train
        mlp = mlp_train.load(args.weights or mlp_train.DEFAULT_WEIGHTS, device="cuda:0")
        if mlp is None:
            print("# no weights of the learned guess: headline uses the analytic guess",
                  file=sys.stderr, flush=True)
    guess = mlp.guess() if mlp is not None else None
    guess_name = ("learned (BF16 MLP on log L, log m, log x; consulted where L > %g)" % mlp.gate
                  if mlp is not None else "analytic")

    # achievable HBM bandwidth: a plain device-to-device copy of 2 GiB, read once and written once
    src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    tcopy = c0.elapsed_time(c1) / 10 * 1e-3
    stream_copy = {"bytes_per_copy": 2 * src.numel() * 8, "GBps": 2 * src.numel() * 8 / tcopy / 1e9,
                   "frac_of_8TBps": 2 * src.numel() * 8 / tcopy / PEAK_HBM}
    del src, dst
    print("# stream copy: %.0f GB/s" % stream_copy["GBps"], file=sys.stderr, flush=True)

    ms_mx, kms_mx, st_mx, fin_mx = measure(S.PREC_MIXED, guess, "headline")
    print("# mixed, %s guess: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
          % (guess_name, ms_mx, args.steps, float(np.mean(kms_mx)), st_mx), file=sys.stderr, flush=True)
    value = n_cells * args.steps / (ms_mx * 1e-3)
    res = {"newton": {"headline": newton_summary(st_mx)}, "stream_copy": stream_copy}
    if mlp is not None and not args.only_headline:
        ms_an, kms_an, st_an, fin_an = measure(S.PREC_MIXED, None, "mixed_analytic")
        print("# mixed, analytic guess: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
              % (ms_an, args.steps, float(np.mean(kms_an)), st_an), file=sys.stderr, flush=True)
        a, b = fin_mx.cpu().numpy(), fin_an.cpu().numpy()
        res["mixed_analytic"] = {"value": n_cells * args.steps / (ms_an * 1e-3),
                                 "ms_per_step": ms_an / args.steps,
                                 "step_kernel_ms": float(np.mean(kms_an)), "stats": st_an,
                                 "max_abs_diff_vs_headline": float(np.max(np.abs(a - b)))}
        res["newton"]["mixed_analytic"] = newton_summary(st_an)
        mlp_c = mlp_train.load(mlp_train.CONS_WEIGHTS, device="cuda:0")
        if mlp_c is not None:
            ms_c, kms_c, st_c, _ = measure(S.PREC_MIXED, mlp_c.guess(), "mixed_learned_cons_inputs")
            print("# mixed, learned guess on (log D, log m, log x), every state: %.2f ms for %d steps"
                  % (ms_c, args.steps), file=sys.stderr, flush=True)
            res["mixed_learned_cons_inputs"] = {"value": n_cells * args.steps / (ms_c * 1e-3),
                                                "ms_per_step": ms_c / args.steps,
                                                "step_kernel_ms": float(np.mean(kms_c)),
                                                "stats": st_c}
            res["newton"]["mixed_learned_cons_inputs"] = newton_summary(st_c)

    # the FP32-inversion mode (FP32 Newton after the exact FP64 L) with the headline's guess
    if not args.only_headline:
        ms_32, kms_32, st_32, fin_32 = measure(S.PREC_FP32, guess, "fp32_inversion")
        print("# fp32 inversion, %s guess: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
              % (guess_name, ms_32, args.steps, float(np.mean(kms_32)), st_32), file=sys.stderr, flush=True)
        res["fp32_inversion"] = {"value": n_cells * args.steps / (ms_32 * 1e-3), "ms_per_step": ms_32 / args.steps,
                                 "step_kernel_ms": float(np.mean(kms_32)), "stats": st_32,
                                 "guess": guess_name}
        res["newton"]["fp32_inversion"] = newton_summary(st_32)

    def field_err(x, ref):
        # over the cells finite on both sides (a non-finite cell is counted, not compared)
        fin = np.isfinite(x).all(axis=1) & np.isfinite(ref).all(axis=1)
        x, ref = x.transpose(1, 0, 2, 3, 4)[:, fin], ref.transpose(1, 0, 2, 3, 4)[:, fin]
        if x.shape[1] == 0:
            return {"non_finite_cells": int((~fin).sum())}
        ms = max(float(np.max(np.sqrt((ref[1:4] ** 2).sum(axis=0)))), 1e-300)
        return {"D": float(np.max(np.abs(x[0] / ref[0] - 1))),
                "Et": float(np.max(np.abs(x[4] / ref[4] - 1))),
                "M": float(np.max(np.abs(x[1:4] - ref[1:4]))) / ms,
                "non_finite_cells": int((~fin).sum())}

    # per-field difference of one FP32-bulk step against one FP64 step from the same state, and
    # after the timed run (each from its own state)
    if not args.no_fp64:
        ms_64, kms_64, st_64, fin_64 = measure(S.PREC_FP64, None, "fp64")
        print("# fp64: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
              % (ms_64, args.steps, float(np.mean(kms_64)), st_64), file=sys.stderr, flush=True)
        S.srhd_cfl_dt(cons0, dh, 0.5, dt_lev=dt)
        S.srhd_fill_ghosts(cons0, nb, 3, padded=pad)
        o64 = S.srhd_fluid_step(pad, dt, dh, prec=S.PREC_FP64).cpu().numpy()
        omx = S.srhd_fluid_step(pad, dt, dh, prec=S.PREC_MIXED, guess=guess).cpu().numpy()

        b = fin_64.cpu().numpy()
        res["fp64"] = {"value": n_cells * args.steps / (ms_64 * 1e-3), "ms_per_step": ms_64 / args.steps,
                       "step_kernel_ms": float(np.mean(kms_64)), "stats": st_64}
        res["newton"]["fp64"] = newton_summary(st_64)
        res["mixed_vs_fp64_rel_err"] = {"one_step": field_err(omx, o64),
                                        "after_%d_steps" % args.steps: field_err(fin_mx.cpu().numpy(), b)}
        if "fp32_inversion" in res:
            o32 = S.srhd_fluid_step(pad, dt, dh, prec=S.PREC_FP32, guess=guess).cpu().numpy()
            res["fp32_inversion"]["vs_fp64_rel_err"] = {
                "one_step": field_err(o32, o64),
                "after_%d_steps" % args.steps: field_err(fin_32.cpu().numpy(), b)}

    # the VL integrator, analytic guess: the gather layout (one kernel per step, the next step's
    # S_max fused) and the padded layout (CFL kernel + ghost fill + VL step per step)
    if args.vl and not args.only_headline:
        res["vl"] = {}
        finals = {}
        for layout in ("grid", "padded"):
            for prec, name in ((S.PREC_MIXED, "mixed"), (S.PREC_FP64, "fp64")):
                runner = run_grid if layout == "grid" else run_padded
                if args.sched != "auto":
                    gr, ch, oc = (int(v) for v in args.sched.split(","))
                    sch, table = S.Sched(gr, ch, dev, occupancy=0 if prec == S.PREC_FP64 else oc), []
                elif layout == "grid":
                    prims, smax = S.srhd_grid_prims(cons0, prec=prec)
                    sch, table = S.srhd_autotune_step_grid(cons0, prims, nb, dh, smax_in=smax,
                                                           prec=prec, reps=2, integrator=S.VL)
                    del prims
                else:
                    S.srhd_cfl_dt(cons0, dh, 0.5, dt_lev=dt)
                    S.srhd_fill_ghosts(cons0, nb, 3, padded=pad)
                    sch, table = S.srhd_autotune_step(pad, dt, dh, prec=prec, reps=2,
                                                      integrator=S.VL)
                key = name if layout == "grid" else "padded_" + name
                schedules["vl_" + key] = {"groups": sch.groups, "chunk": sch.chunk,
                                          "occupancy": sch.occupancy,
                                          "autotune_ms": [[t[0], t[1], t[2], round(t[3], 4)] for t in table]}
                if args.warmup:
                    runner(prec, args.warmup, sched=sch, integrator=S.VL)
                ms_v, kms_v, st_v, fin_v = runner(prec, args.steps, time_kernel=True, sched=sch,
                                                  integrator=S.VL)
                finals[key] = fin_v.cpu().numpy()
                print("# VL %s %s: %.2f ms for %d steps (step kernel %.3f ms avg); stats %s"
                      % (layout, name, ms_v, args.steps, float(np.mean(kms_v)), st_v),
                      file=sys.stderr, flush=True)
                res["vl"][key] = {"value": n_cells * args.steps / (ms_v * 1e-3),
                                  "ms_per_step": ms_v / args.steps,
                                  "step_kernel_ms": float(np.mean(kms_v)), "stats": st_v,
                                  "newton": newton_summary(st_v)}
        res["vl"]["mixed_vs_fp64_rel_err_after_%d_steps" % args.steps] = field_err(finals["mixed"],
                                                                                 finals["fp64"])
        # the padded chain takes dt from the CFL kernel, the gather chain from the fused S_max: in
        # FP64 the two are the same bits, so the two layouts end in the same state
        res["vl"]["fp64_layouts_equal"] = bool(np.array_equal(finals["fp64"], finals["padded_fp64"]))

    # the widened rows on the same blast (padded layout, analytic guess): the original
    # total-energy scheme and the polytropic EoS, one-workgroup-per-patch launch
    if args.variants and not args.only_headline:
        def time_padded(n_steps, **kw):
            """n_steps from the initial state: ghost fill + one step per step.  Reduced-energy
            runs take the CFL time step of the current state every step (the CFL kernel is
            inside the timed region); the original scheme's total-energy state has no CFL
            entry, so its runs keep 0.8 x the initial state's CFL step throughout (the blast's
            S_max grows by less than 10 % over these steps)."""
            gamma = kw.get("gamma")
            cur = cons0.clone()
            if gamma:
                cur = S.srhd_prim2cons(prim_soa, gamma=gamma).reshape(5, P, 512).permute(
                    1, 0, 2).contiguous().reshape(P, 5, 8, 8, 8)
            total = kw.get("energy") == S.ENERGY_TOTAL
            if total:
                S.srhd_cfl_dt(cur, dh, 0.5 * 0.8, dt_lev=dt)
                cur[:, 4] += cur[:, 0]                 # E = Et + D: the original scheme's state
            start = cur.clone()
            nxt = torch.empty_like(cur)
            st = S.new_stats(dev)

            def one(stats):
                nonlocal cur, nxt
                if not total:
                    S.srhd_cfl_dt(cur, dh, 0.5, dt_lev=dt, gamma=gamma)
                S.srhd_fill_ghosts(cur, nb, 3, padded=pad)
                S.srhd_fluid_step(pad, dt, dh, out=nxt, stats=stats, **kw)
                cur, nxt = nxt, cur
            for _ in range(args.warmup):
                one(None)
            cur.copy_(start)
            a0 = torch.cuda.Event(enable_timing=True)
            a1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a0.record(stream)
            for _ in range(n_steps):
                one(st)
            a1.record(stream)
            torch.cuda.synchronize()
            ms = a0.elapsed_time(a1)
            return {"value": n_cells * n_steps / (ms * 1e-3), "ms_per_step": ms / n_steps,
                    "stats": S.stats_dict(st),
                    "non_finite_cells": int((~torch.isfinite(cur)).any(dim=1).sum().item())}
        res["original_scheme"] = {
            "fp64": time_padded(args.steps, prec=S.PREC_FP64, energy=S.ENERGY_TOTAL),
            "fp32": time_padded(args.steps, prec=S.PREC_FP32, energy=S.ENERGY_TOTAL)}
        # Gamma = 4/3, the hot limit of TM: the blast's source gas has Theta = 1e6
        res["polytropic_4_3"] = {
            "fp64": time_padded(args.steps, prec=S.PREC_FP64, gamma=4.0 / 3.0),
            "mixed": time_padded(args.steps, prec=S.PREC_MIXED, gamma=4.0 / 3.0)}
        for k in ("original_scheme", "polytropic_4_3"):
            print("# %s: %s" % (k, {m: "%.3g cell updates/s, %d unphysical" % (v["value"], v["stats"]["n_unphysical"])
                                     for m, v in res[k].items()}), file=sys.stderr, flush=True)

    # two AMR levels: 16^3 coarse patches with the central 8^3 refined (4,096 fine patches);
    # one cycle = CFL, coarse step, two fine sub-steps with coarse-to-fine ghosts, restriction,
    # coarse-fine flux correction, all on the GPU (FP64, MUSCL-Hancock)
    if args.amr and not args.only_headline:
        t2 = W.two_level(16, 4, 12)
        def amr_cons(xyz):
            x, y, z = xyz
            s_ = np.sin(2 * np.pi * (x + 0.5 * y))
            w = np.stack([1.0 + 0.2 * s_, 0.3 + 0.1 * np.cos(2 * np.pi * z) + 0 * x, 0.1 * s_, 0 * x,
                          1.0 + 0.3 * np.cos(2 * np.pi * y) + 0 * x], axis=1)
            Pn = w.shape[0]
            ws = torch.from_numpy(np.ascontiguousarray(w.reshape(Pn, 5, 512).transpose(1, 0, 2).reshape(5, -1))).to(dev)
            return S.srhd_prim2cons(ws).reshape(5, Pn, 512).permute(1, 0, 2).contiguous().reshape(Pn, 5, 8, 8, 8)
        ac, af = amr_cons(t2["coarse_xyz"]), amr_cons(t2["fine_xyz"])
        g2 = {k: torch.from_numpy(np.ascontiguousarray(t2[k])).to(dev)
              for k in ("coarse_neighbor", "fine_neighbor", "parent", "octant", "parent_of", "child", "faces")}
        S.srhd_restrict(ac, g2["parent_of"], g2["child"], af)
        dh2 = [t2["dh_c"], t2["dh_f"]]
        Pc, Pf = ac.shape[0], af.shape[0]
        fc = torch.empty((Pc, 6, 5, 64), dtype=torch.float64, device=dev)
        fcw, ffl = torch.empty_like(fc), torch.empty((Pf, 6, 5, 64), dtype=torch.float64, device=dev)
        ffs = torch.zeros_like(ffl)
        both = torch.empty((Pc + Pf, 5, 8, 8, 8), dtype=torch.float64, device=dev)
        dt2 = torch.empty(2, dtype=torch.float64, device=dev)
        skipped = torch.zeros(1, dtype=torch.int64, device=dev)

        def amr_cycle(c, f):
            both[:Pc].copy_(c)
            both[Pc:].copy_(f)
            S.srhd_cfl_dt(both, dh2, 0.5, dt_lev=dt2)
            dtv = dt2.cpu().numpy()
            pc = S.srhd_fill_ghosts(c, g2["coarse_neighbor"], 3)
            cn = S.srhd_fluid_step(pc, dt2[0:1], [dh2[0]], flux_out=fc)
            pcn = S.srhd_fill_ghosts(cn, g2["coarse_neighbor"], 3)
            for sub in range(2):
                pf = S.srhd_fill_ghosts(f, g2["fine_neighbor"], 3)
                S.srhd_fill_ghosts_coarse(pf, g2["fine_neighbor"], g2["parent"], g2["octant"], pc,
                                          pcn if sub else None, 0.5 * sub)
                f = S.srhd_fluid_step(pf, dt2[1:2], [dh2[1]], flux_out=ffl)
                S.srhd_flux_accumulate(ffs, ffl, float(sub), float(dtv[1]))
            S.srhd_restrict(cn, g2["parent_of"], g2["child"], f)
            S.srhd_flux_accumulate(fcw, fc, 0.0, float(dtv[0]))
            S.srhd_flux_correct(cn, g2["faces"], fcw, ffs, dh2[0], skipped=skipped)
            return cn, f
        c, f = ac, af
        for _ in range(args.warmup):
            c, f = amr_cycle(c, f)
        torch.cuda.synchronize()
        t0 = time.time()
        n_cyc = args.steps
        for _ in range(n_cyc):
            c, f = amr_cycle(c, f)
        torch.cuda.synchronize()
        ms = (time.time() - t0) * 1e3
        upd = (Pc + 2 * Pf) * 512
        res["amr_two_level"] = {"coarse_patches": Pc, "fine_patches": Pf, "cycles": n_cyc,
                                "ms_per_cycle": ms / n_cyc,
                                "value": upd * n_cyc / (ms * 1e-3), "unit": "cell updates/s",
                                "note": "wall clock per cycle incl. one host read of dt",
                                "flux_correction_skipped": int(skipped.item())}
        print("# AMR two levels: %.2f ms per cycle (%.3g cell updates/s)"
              % (ms / n_cyc, upd * n_cyc / (ms * 1e-3)), file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- roofline of the step kernel
    kavg = float(np.mean(kms_mx)) * 1e-3
    per_launch = {k: v / args.steps for k, v in st_mx.items()}
    flops = step_flops(P, per_launch, True, args.path == "grid")
    prof = None
    if (step_sources_hash() == PROFILED["sources_sha256_16"] and args.cells == 256
            and args.path == PROFILED["path"] and mlp is not None
            and schedules.get("headline", {}).get("occupancy") == 2):
        prof = PROFILED["headline"]
    io = IO_BYTES_PER_PATCH[args.path] * P
    roofline = {"bound": "alu", "achieved": flops / kavg / 1e12, "peak": PEAK_ALU / 1e12,
                "unit": "TFLOP/s", "frac": flops / kavg / PEAK_ALU,
                "traffic": (prof["read"] + prof["write"]) if prof else None,
                "kernel": "k_step<float,%s,%s> (mixed)" % ("gather" if args.path == "grid" else "padded",
                                                           "mlp" if mlp is not None else "analytic"),
                "launch_ms": kavg * 1e3, "flops_per_launch": flops,
                "flops_note": "L charged at the plain-sum cost the FP32-bulk kernel takes where a "
                              "wavefront is well conditioned (compensated fallbacks not counted)",
                "hbm_GBps_algorithmic": io / kavg / 1e9, "hbm_frac_algorithmic": io / kavg / PEAK_HBM,
                "hbm_frac_of_stream_copy": io / kavg / (stream_copy["GBps"] * 1e9)}
    if prof:
        roofline["counters"] = {"summary": PROFILED["summary"], "profiled_ms": prof["ms"],
                                "flops_per_launch": prof["flops"],
                                "frac": prof["flops"] / (prof["ms"] * 1e-3) / PEAK_ALU,
                                "hbm_frac": (prof["read"] + prof["write"]) / (prof["ms"] * 1e-3) / PEAK_HBM,
                                "valu_issue_frac": prof["valu_issue"]}
    if mlp is not None:
        mf = per_launch["n_mlp"] * MFMA_FLOP_MLP
        roofline["mfma_bf16"] = {"flops_per_launch": mf, "achieved_TFLOPs": mf / kavg / 1e12,
                                 "frac_of_2500": mf / kavg / 2.5e15}
    if "fp64" in res and args.path == "grid":
        k64 = res["fp64"]["step_kernel_ms"] * 1e-3
        pl64 = {k: v / args.steps for k, v in res["fp64"]["stats"].items()}
        f64 = step_flops(P, pl64, False, True)
        io64 = (1376 * 5 * 8 + 512 * 5 * (8 + 8 + 8)) * P
        res["fp64"]["roofline"] = {"bound": "alu", "achieved": f64 / k64 / 1e12, "unit": "TFLOP/s",
                                   "peak": PEAK_ALU / 1e12, "frac": f64 / k64 / PEAK_ALU,
                                   "flops_per_launch": f64, "launch_ms": k64 * 1e3,
                                   "hbm_frac_algorithmic": io64 / k64 / PEAK_HBM}
        p64 = PROFILED.get("fp64") if prof else None
        if p64:
            res["fp64"]["roofline"]["counters"] = {
                "profiled_ms": p64["ms"], "flops_per_launch": p64["flops"],
                "frac": p64["flops"] / (p64["ms"] * 1e-3) / PEAK_ALU,
                "hbm_frac": (p64["read"] + p64["write"]) / (p64["ms"] * 1e-3) / PEAK_HBM,
                "valu_issue_frac": p64["valu_issue"]}

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
        its = torch.empty(n, dtype=torch.uint8, device=dev)
        conv = {}
        variants = [("fp64", cc, None), ("fp32", cc.float(), None)]
        if mlp is not None:
            variants += [("fp64_learned_guess", cc, guess), ("fp32_learned_guess", variants[1][1], guess)]
        # Eq. 20's condition number of each stored state: L's subtraction a - b with
        # a = x^2 + 2x, b = m^2 (x = Et/D, m = |M|/D), cond = (a + b) / |a - b| (from the FP64
        # conserved variables; about 1 + M^2)
        xx = cc[4] / cc[0]
        mm = (cc[1] ** 2 + cc[2] ** 2 + cc[3] ** 2) / (cc[0] ** 2)
        aa = xx * (xx + 2.0)
        cond = (aa + mm) / (aa - mm).abs()
        del xx, mm, aa
        conv_sample = {}
        n_sample = min(n, 1_000_000)
        for name, src, gs in variants:
            o = out if src.dtype == torch.float64 else torch.empty_like(src)
            S.srhd_cons2prim(src, prim=o, status=stt, iters=its, guess=gs)
            torch.cuda.synchronize()
            mean_it = float(its.double().mean().item())
            if gs is None:
                conv_sample[name] = (src[:, :n_sample].cpu().numpy(), o[:, :n_sample].double().cpu().numpy(),
                                     stt[:n_sample].cpu().numpy())
                rt = roundtrip_by_cond(o, cp, stt, cond, 2.0 ** -53 if name == "fp64" else 2.0 ** -24)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            reps = 5
            e0.record(stream)
            for _ in range(reps):
                S.srhd_cons2prim(src, prim=o, status=stt, guess=gs)
            e1.record(stream)
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) / reps * 1e-3
            bpe = 2 * 5 * src.element_size() + 1
            conv[name] = {"states_per_s": n / t, "ms": t * 1e3,
                          "hbm_frac": n * bpe / t / PEAK_HBM, "newton_iters_mean": mean_it,
                          "unphysical_frac": float((stt == 1).float().mean().item()),
                          "fallback_frac": float((stt == 2).float().mean().item())}
            if gs is None:
                conv[name]["roundtrip_err_by_cond"] = rt
        res["conversion_batch_1e8"] = conv
        del cp, cc, out, stt, its, variants, cond

    # ---------------------------------------------------------------- jet patch list
    if args.jet:
        res["jet_patch_list"] = run_jet(args, S, W, dev, stream, guess, guess_name)

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
        # the same on one core, on a sample sized for about a third of that time
        O.set_num_threads(1)
        try:
            m1 = int(max(8, min(m, (args.cpu_seconds / 3.0) / max(tc / m * threads, 1e-9))))
            idx1 = np.sort(rng.choice(P, m1, replace=False))
            tc1 = oracle_pass(idx1)
        finally:
            O.set_num_threads(threads)
        cpu = {"value": m * 512 / tc, "unit": "cell updates/s", "cores": threads,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": "%d random patches (%d cells) of the 256^3 blast, one FP64 step from "
                         "the initial state: CFL + ghost fill + MUSCL-Hancock step, %.1f s" % (m, m * 512, tc),
               "one_core": {"value": m1 * 512 / tc1, "unit": "cell updates/s", "cores": 1,
                            "sample": "%d random patches of the same, %.1f s" % (m1, tc1)}}
        # the conversion batch: the oracle inverts the first states of each FP64 / FP32 variant
        # (the FP32 one from its FP32 conserved variables, widened exactly), timed, and the
        # GPU's results are compared with it state by state (outside the GPU's timed region)
        if args.conversion and conv_sample:
            res["conversion_batch_1e8"]["oracle_sample"] = oracle_conversion_parity(O, conv_sample, threads)

    line = {
        "metric": METRIC, "value": value, "unit": "cell updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_mx / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "blast_%d^3_periodic_%dpatches_mixed_precision" % (args.cells, P),
                   "path": args.path, "patch_order": "morton",
                   "cells": n_cells, "patches": P, "ghost": 3, "riemann": "HLLC",
                   "limiter_theta": 1.5, "guess": guess_name, "steps_per_run": args.steps},
        "roofline": roofline, "cpu_baseline": cpu, "mixed_stats": st_mx,
    }
    line["schedules"] = schedules
    line.update(res)
    print(json.dumps(_finite(line)), flush=True)


if __name__ == "__main__":
    main()
