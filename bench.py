"""Benchmark: IFGF matvecs per second on one MI355X.

Headline workload: unit sphere, N = 6,291,456 points (6 x 1024 x 1024
cube-sphere), kappa = 128 pi (diameter 128 wavelengths), 4 complex Gaussian
density vectors per apply, (P_s, P_ang) = (3, 5) Chebyshev nodes, 1 x 2 x 4
leaf cones, H_D about a quarter wavelength, FP64 arithmetic throughout (the
precision the oracle and the paper's accuracy figures refer to).  One timed
step is one IFGF apply of the 4 right-hand sides with inputs resident in
device memory; value = 4 / (seconds per step) matvecs per second.  Plan
construction is excluded from the timed region and reported separately (as
the paper reports T_pre apart from T_acc).

Extras in the same JSON line: the mixed path (FP32 arithmetic, FP64
geometry) on the same workload, FP64 at 1 right-hand side, and the figures
of the N = 393,216, kappa = 32 pi sphere (mixed 1 and 16 right-hand sides,
FP64, adjoint, graph replay, target gradient).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
       [--no-extras] [--workload 5|2] [--precision fp64|mixed]
Prints one JSON line.

Profiling: `python bench.py --profile-commands DIR` prints the four
rocprofv3 commands (kernel trace with stats; FETCH_SIZE; WRITE_SIZE; SQ
instruction counters) whose outputs `python bench.py --summarize DIR` turns
into the summaries under profiles/.  The counter runs also time a plain copy
kernel of known size (--copy-calibration), whose counter readings give the
bytes-per-KiB scale applied to the IFGF kernels' readings.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for roofline fractions.
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "ifgf_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2010_02857_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


# the profiled configuration: the headline (workload 5, FP64, its 4 RHS)
PROFILE_WORKLOAD = 5
PROFILE_PRECISION = "fp64"
TRACE_ARGS = "--steps 2 --warmup 1 --no-extras --no-cpu-baseline --no-eps"
PMC_ARGS = "--steps 1 --warmup 1 --no-extras --no-cpu-baseline --no-eps --copy-calibration"
SQ_ARGS = "--steps 1 --warmup 1 --no-extras --no-cpu-baseline --no-eps"
# the profiled configuration: the headline by default; the profiling and
# summary commands take --workload / --precision / --nrhs too
PROFILE = {"workload": PROFILE_WORKLOAD, "precision": PROFILE_PRECISION, "nrhs": 0, "autotune": False}


def workload_tag(workload: int, precision: str, nrhs: int) -> str:
    n = {2: 393216, 5: 6291456}[workload]
    if nrhs <= 0:
        nrhs = {2: 1, 5: 4}[workload]
    return f"sphere{n}_{precision}_{nrhs}rhs"


def config_args() -> str:
    a = f" --workload {PROFILE['workload']} --precision {PROFILE['precision']}"
    a += f" --nrhs {PROFILE['nrhs']}" if PROFILE["nrhs"] > 0 else ""
    return a + (" --autotune" if PROFILE["autotune"] else "")
SQ_COUNTERS = ("SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VALU_MFMA_F32 SQ_INSTS_VALU_MFMA_F64 "
               "SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_LDS")
SIMDS = 1024                   # 256 CUs x 4 SIMDs
CLOCK_HZ = 2.4e9
COPY_NUMEL = 64 << 20          # float32 elements read and written by the calibration copy
# child-to-parent variants that run on the matrix cores
MFMA_VARIANTS = ("mfma", "mfma_geometry", "boxes", "box_acc", "box_acc_half")


def profile_commands(d: str) -> list[str]:
    c = config_args()
    return [
        f"rocprofv3 --kernel-trace --stats --output-format csv -d {d}/trace -o run -- python3 bench.py {TRACE_ARGS}{c} "
        f"--stats-out {d}/plan_stats.json",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fetch -o run -- python3 bench.py {PMC_ARGS}{c}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/write -o run -- python3 bench.py {PMC_ARGS}{c}",
        f"rocprofv3 --pmc {SQ_COUNTERS} --output-format csv -d {d}/sq -o run -- python3 bench.py {SQ_ARGS}{c}",
    ]


def _short(name: str) -> str:
    name = name.replace("void ifgf::(anonymous namespace)::", "")
    return name.split("(")[0] if name.startswith("k_") else name[:60]


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _steps(args: str) -> int:
    a = args.split()
    return int(a[a.index("--steps") + 1])


def _timed(rows: list, steps: int) -> list:
    """The rows of the timed region: every dispatch from the start of the
    last `steps` applies on (each apply launches k_leaf_nodes once; the
    autotuning and warm-up launches come before)."""
    rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
    leaf = sorted({int(r["Dispatch_Id"]) for r in rows if "k_leaf_nodes" in r["Kernel_Name"]})
    if len(leaf) < steps:
        raise RuntimeError("fewer applies in the profile than timed steps")
    first = leaf[-steps]
    # the apply starts with its permutation, launched before the leaf values
    perm = [int(r["Dispatch_Id"]) for r in rows if "k_permute_in" in r["Kernel_Name"]
            and int(r["Dispatch_Id"]) < first]
    if perm:
        first = max(perm)
    return [r for r in rows if int(r["Dispatch_Id"]) >= first]


def summarize(d: str) -> int:
    WORKLOAD_TAG = workload_tag(PROFILE["workload"], PROFILE["precision"], PROFILE["nrhs"])
    """Writes profiles/<stage>_<workload>_kernel_trace.md and, from the two
    counter runs, profiles/traffic_<stage>_<workload>.{json,md}; only the
    launches of the timed matvecs are counted."""
    import collections
    import csv
    cmds = profile_commands(d)
    out_dir = os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    stage = "child_to_parent"
    # kernel trace of the timed region
    steps = _steps(TRACE_ARGS)
    rows = _timed(list(csv.DictReader(open(_find(os.path.join(d, "trace"), "kernel_trace.csv")))), steps)
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        a = agg[r["Kernel_Name"]]
        a[0] += 1
        a[1] += int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    total = sum(v[1] for v in agg.values())
    lines = [f"# Kernel trace, {WORKLOAD_TAG}: {TRACE_ARGS}{config_args()}", "",
             "Command (repository root):", "", "    " + cmds[0], "",
             f"Launches of the {steps} timed matvecs (autotuning and warm-up launches excluded).", "",
             "| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
    for name, (c, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| `{_short(name)}` | {c} | {ns / 1e6:.3f} | {ns / c / 1e6:.4f} | {100.0 * ns / total:.2f} |")
    st_calls = sum(c for name, (c, ns) in agg.items() if "k_child_to_parent" in name)
    st_ns = sum(ns for name, (c, ns) in agg.items() if "k_child_to_parent" in name)
    lines += ["", f"Stage `{stage}` (all k_child_to_parent* kernels): {st_calls} launches, "
              f"average {st_ns / max(st_calls, 1) / 1e6:.4f} ms per launch; "
              f"{total / steps / 1e6:.3f} ms of kernel time per matvec (summed over both streams, whose "
              f"kernels overlap).", ""]
    with open(os.path.join(out_dir, f"{stage}_{WORKLOAD_TAG}_kernel_trace.md"), "w") as fh:
        fh.write("\n".join(lines))
    # HBM traffic from FETCH_SIZE / WRITE_SIZE (KiB per dispatch)
    rec = {"kernel_source_hash": kernel_source_hash(), "stage": stage, "workload": WORKLOAD_TAG,
           "commands": cmds[1:]}
    md = [f"# HBM traffic of `{stage}`, {WORKLOAD_TAG}", "", "Commands (repository root):", ""]
    md += ["    " + c for c in cmds[1:]] + [""]
    psteps = _steps(PMC_ARGS)
    for ctr, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        allrows = list(csv.DictReader(open(_find(os.path.join(d, sub), "counter_collection.csv"))))
        copy = [float(r["Counter_Value"]) for r in allrows if "neg" in r["Kernel_Name"] and r["Counter_Name"] == ctr]
        crow = _timed(allrows, psteps)
        kib = [float(r["Counter_Value"]) for r in crow
               if "k_child_to_parent" in r["Kernel_Name"] and r["Counter_Name"] == ctr]
        if not copy or not kib:
            raise RuntimeError(f"{ctr}: copy or {stage} dispatches missing")
        scale = COPY_NUMEL * 4 / (sum(copy) / len(copy) * 1024.0)      # bytes per counter KiB
        per_launch = sum(kib) / len(kib) * 1024.0 * scale
        rec[f"{sub}_bytes_per_launch"] = per_launch
        rec[f"{sub}_copy_scale"] = scale
        rec[f"{sub}_dispatches"] = len(kib)
        md.append(f"* {ctr}: copy kernel ({COPY_NUMEL * 4} B read and written) counts "
                  f"{sum(copy) / len(copy):.1f} KiB per dispatch, scale {scale:.4f} B per counted byte; "
                  f"`{stage}`: {len(kib)} dispatches of the {psteps} timed matvecs, "
                  f"{per_launch / 1e6:.2f} MB per launch after scaling.")
    rec["hbm_bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    md += ["", f"HBM bytes per launch (fetch + write): {rec['hbm_bytes_per_launch'] / 1e6:.2f} MB. "
           f"Kernel source hash {rec['kernel_source_hash']}.", ""]
    # every kernel of the matvec: scaled HBM bytes per matvec over its time per
    # matvec in the kernel trace (kernels on the two streams overlap, so each
    # runs beside others)
    per_k = collections.defaultdict(lambda: [0.0, 0.0])
    for ctr, sub, k in (("FETCH_SIZE", "fetch", 0), ("WRITE_SIZE", "write", 1)):
        allrows = list(csv.DictReader(open(_find(os.path.join(d, sub), "counter_collection.csv"))))
        for r in _timed(allrows, psteps):
            if r["Counter_Name"] == ctr and r["Kernel_Name"].startswith("void ifgf"):
                per_k[_short(r["Kernel_Name"])][k] += float(r["Counter_Value"]) * 1024.0 * rec[f"{sub}_copy_scale"] / psteps
    dur = collections.defaultdict(float)
    for r in rows:
        dur[_short(r["Kernel_Name"])] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9 / steps
    md += ["Every kernel of one matvec (HBM bytes from the counter runs, time from the kernel trace):", "",
           "| kernel | ms | fetch MB | write MB | HBM GB/s | of 8000 |", "|---|---|---|---|---|---|"]
    for name, (fb, wb) in sorted(per_k.items(), key=lambda kv: -dur.get(kv[0], 0.0)):
        t = dur.get(name, 0.0)
        if t <= 0.0:
            continue
        gbs = (fb + wb) / t / 1e9
        md.append(f"| `{name}` | {t * 1e3:.3f} | {fb / 1e6:.1f} | {wb / 1e6:.1f} | {gbs:.0f} | {gbs / 8000.0:.3f} |")
    md.append("")
    with open(os.path.join(out_dir, f"traffic_{stage}_{WORKLOAD_TAG}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(os.path.join(out_dir, f"traffic_{stage}_{WORKLOAD_TAG}.md"), "w") as fh:
        fh.write("\n".join(md))
    print(json.dumps(rec))
    summarize_sq(d, cmds[3], rows)
    return 0


def summarize_sq(d: str, cmd: str, trace_rows: list) -> None:
    WORKLOAD_TAG = workload_tag(PROFILE["workload"], PROFILE["precision"], PROFILE["nrhs"])
    """profiles/sq_child_to_parent_<workload>.md: instruction counts of each
    child-to-parent launch of one timed matvec (SQ counters, summed over the
    chip), per evaluation and as a fraction of the chip's issue capacity over
    the launch's duration in the kernel trace (a wave64 VALU instruction
    occupies a SIMD for 4 cycles, a 16x16x4 FP32 MFMA for 32)."""
    import collections
    import csv
    st = json.load(open(os.path.join(d, "plan_stats.json")))
    evals = st["n_parent_evals"]
    D = st["D"]
    rows = _timed(list(csv.DictReader(open(_find(os.path.join(d, "sq"), "counter_collection.csv")))),
                  _steps(SQ_ARGS))
    per = collections.OrderedDict()
    for r in rows:
        if "k_child_to_parent" not in r["Kernel_Name"]:
            continue
        e = per.setdefault(int(r["Dispatch_Id"]), {"name": _short(r["Kernel_Name"])})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    # durations of the same launches in the trace run (its first timed matvec)
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
           for r in sorted(trace_rows, key=lambda r: int(r["Dispatch_Id"])) if "k_child_to_parent" in r["Kernel_Name"]]
    lines = [f"# Instruction mix of `child_to_parent`, {WORKLOAD_TAG}", "",
             "Command (repository root):", "", "    " + cmd, "",
             "One timed matvec; launches in order of the child level.  Per evaluation: lane instructions "
             "(wave instructions x 64) per (parent interpolation point, child) evaluation (MFMA F64: wave "
             "instructions per evaluation).  Issue fractions: "
             f"VALU = 4 x wave VALU instructions, MFMA = busy cycles, over {SIMDS} SIMDs x "
             f"{CLOCK_HZ / 1e9:.1f} GHz x the launch's duration in the kernel trace.", "",
             "| child level | kernel | ms | VALU / eval | LDS / eval | MFMA F64 / eval | VALU issue | MFMA busy |",
             "|---|---|---|---|---|---|---|---|"]
    for i, (k, e) in enumerate(per.items()):
        lvl = D - i
        t = dur[i] if i < len(dur) else float("nan")
        cap = SIMDS * CLOCK_HZ * t
        ev = max(evals[lvl], 1)
        lines.append(f"| {lvl} | `{e['name']}` | {t * 1e3:.3f} | {e.get('SQ_INSTS_VALU', 0) * 64 / ev:.0f} | "
                     f"{e.get('SQ_INSTS_LDS', 0) * 64 / ev:.0f} | {e.get('SQ_INSTS_VALU_MFMA_F64', 0) / ev:.2f} | "
                     f"{4 * e.get('SQ_INSTS_VALU', 0) / cap:.2f} | {e.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) / cap:.2f} |")
    lines.append("")
    # the other stages, per kernel over the matvec: VALU issue (transcendentals
    # included) and MFMA busy against the same capacity
    agg = collections.OrderedDict()
    for r in rows:
        if "k_child_to_parent" in r["Kernel_Name"] or not r["Kernel_Name"].startswith("void ifgf"):
            continue
        e = agg.setdefault(_short(r["Kernel_Name"]), {})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    tdur = collections.defaultdict(float)
    nsteps = _steps(TRACE_ARGS)
    for r in trace_rows:
        tdur[_short(r["Kernel_Name"])] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9 / nsteps
    lines += ["The other stages (all launches of one matvec):", "",
              "| kernel | ms | VALU issue | MFMA busy |", "|---|---|---|---|"]
    for name, e in agg.items():
        t = tdur.get(name, 0.0)
        if t <= 0.0:
            continue
        cap = SIMDS * CLOCK_HZ * t
        lines.append(f"| `{name}` | {t * 1e3:.3f} | {4 * e.get('SQ_INSTS_VALU', 0) / cap:.2f} | "
                     f"{e.get('SQ_VALU_MFMA_BUSY_CYCLES', 0) / cap:.2f} |")
    lines.append("")
    with open(os.path.join(ROOT, "profiles", f"sq_child_to_parent_{WORKLOAD_TAG}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def stage_work(stats: dict, stage: str, nrhs: int, P: int, elem_bytes: int) -> tuple[float, float]:
    """Algorithmic (flops, bytes) of one apply's launches of a stage.

    child_to_parent / cousin_eval: per interpolation, P complex-by-real
    multiply-adds per right-hand side (4 P flops) plus the complex product with
    the centred-factor ratio (8 flops); bytes: the cone values read once and
    the parent values written once (child_to_parent), or the cone values read
    once plus the output read and written (cousin_eval).
    leaf_nodes / nearfield: one complex multiply-add (8 flops) per source pair
    and right-hand side; bytes: densities read and values written once."""
    D = stats["D"]
    cones = stats["n_cones"]
    n = stats["n_points"]
    if stage == "child_to_parent":
        ev = sum(stats["n_parent_evals"][3:D + 1])
        flops = ev * nrhs * (4 * P + 8)
        read = sum(cones[d] for d in range(4, D + 1))        # child cone values, once
        write = sum(cones[d] for d in range(3, D))          # parent cone values, once
        return flops, (read + write) * P * nrhs * elem_bytes
    if stage == "cousin_eval":
        ev = sum(stats["n_cousin_evals"][3:D + 1])
        flops = ev * nrhs * (4 * P + 8)
        byts = sum(cones[d] for d in range(3, D + 1)) * P * nrhs * elem_bytes + (D - 2) * 2 * n * nrhs * elem_bytes
        return flops, byts
    if stage == "leaf_nodes":
        return stats["n_leaf_pairs"] * nrhs * 8.0, cones[D] * P * nrhs * elem_bytes + n * nrhs * elem_bytes
    if stage == "nearfield":
        return stats["n_near_pairs"] * nrhs * 8.0, 2 * n * nrhs * elem_bytes
    return 0.0, 2 * n * nrhs * elem_bytes


def roofline_of(stats: dict, stages: dict, levels: dict, choice: dict, nrhs: int, steps: int, P: int,
                elem_bytes: int, fp64: bool, traffic) -> dict:
    """Roofline of the child-to-parent stage (the dominant one): algorithmic
    flops of one launch (the plan's (parent point, child) evaluations x
    (4 P + 8) flops x right-hand sides) over its average launch duration,
    measured with HIP events on its stream over the timed region; per level
    too, with the variant that ran there."""
    ms, launches = stages["child_to_parent"]
    flops, byts = stage_work(stats, "child_to_parent", nrhs, P, elem_bytes)
    per_launch_s = ms / 1e3 / launches
    lpa = launches / steps
    achieved = flops / lpa / per_launch_s / 1e12
    mfma = all(choice.get(d) in MFMA_VARIANTS for d in levels)
    peak = PEAK_FP64_TFLOPS if fp64 else PEAK_FP32_TFLOPS
    per_level = {}
    for d, (lms, lcnt) in sorted(levels.items()):
        ev = stats["n_parent_evals"][d] * nrhs * (4 * P + 8)
        t = lms / 1e3 / lcnt
        per_level[str(d)] = {"variant": choice.get(d), "avg_ms": round(t * 1e3, 3),
                             "TFLOPs": round(ev / t / 1e12, 3), "frac": round(ev / t / 1e12 / peak, 4)}
    return {"bound": "mfma" if mfma else "alu", "kernel": "child_to_parent", "achieved": round(achieved, 3),
            "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 5), "traffic": traffic,
            "avg_launch_ms": round(per_launch_s * 1e3, 4), "launches_per_step": lpa,
            "algorithmic_flops_per_launch": flops / lpa, "algorithmic_bytes_per_launch": byts / lpa,
            "achieved_algorithmic_GBps": round(byts / lpa / per_launch_s / 1e9, 1), "hbm_peak_GBps": PEAK_HBM_GBS,
            "peak_note": ("FP64: 78.6 TFLOP/s for both the vector units and the matrix cores" if fp64 else
                          "FP32: 157.3 TFLOP/s (matrix cores; packed vector FP32, not used here)"),
            "per_level": per_level}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=PROFILE_WORKLOAD, choices=(2, 5))
    ap.add_argument("--precision", default=PROFILE_PRECISION, choices=("fp64", "mixed"))
    ap.add_argument("--nrhs", type=int, default=0, help="right-hand sides (0: the workload's own)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the other precisions and workloads")
    ap.add_argument("--no-eps", action="store_true", help="skip the direct-sum accuracy check (profiling runs)")
    ap.add_argument("--autotune", action="store_true", help="autotune the headline plan (default: the default rule)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain copy of known size (for scaling HBM byte counters)")
    ap.add_argument("--stats-out", metavar="FILE", help="write the headline plan's statistics as JSON")
    ap.add_argument("--profile-commands", metavar="DIR", help="print the profiling commands and exit")
    ap.add_argument("--summarize", metavar="DIR", help="write profiles/ summaries from profiling outputs and exit")
    args = ap.parse_args()
    PROFILE.update(workload=args.workload, precision=args.precision, nrhs=args.nrhs, autotune=args.autotune)
    if args.profile_commands:
        print("\n".join(profile_commands(args.profile_commands)))
        return 0
    if args.summarize:
        return summarize(args.summarize)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        return 2

    import torch

    import oracle
    from paper_2010_02857_amd import ifgf, inputs

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.copy_calibration:
        src = torch.ones(COPY_NUMEL, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    w = inputs.WORKLOADS[args.workload]
    p = w.points()
    n = p.shape[0]
    nrhs = args.nrhs if args.nrhs > 0 else w.nrhs
    prec = args.precision
    fp64 = prec == "fp64"
    cdt = torch.complex128 if fp64 else torch.complex64
    a = w.densities(nrhs)
    P = 75

    def time_fn(fn, reps):
        fn()
        torch.cuda.synchronize()
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record()
        for _ in range(reps):
            fn()
        s1.record()
        torch.cuda.synchronize()
        return s0.elapsed_time(s1) / reps

    # ---- plan (excluded from the timed region)
    t0 = time.time()
    plan = ifgf.Plan(p, w.kappa, precision=prec, max_nrhs=nrhs, store_levels=0)
    t_plan = time.time() - t0
    st = plan.stats()
    log(f"plan: {w.name} N={n} D={st['D']} {prec} cones/level={st['n_cones'][3:]} {t_plan:.1f}s "
        f"device {st['device_bytes'] / 1e9:.2f} GB")
    if args.stats_out:
        os.makedirs(os.path.dirname(os.path.abspath(args.stats_out)), exist_ok=True)
        with open(args.stats_out, "w") as fh:
            json.dump(st, fh)
    t_tune = 0.0
    if args.autotune:
        t0 = time.time()
        plan.autotune(nrhs)
        t_tune = time.time() - t0
    choice = plan.kernel_choice(nrhs)
    log(f"child-to-parent kernels ({'autotuned' if args.autotune else 'default rule'}): {choice}")
    x = torch.from_numpy(a).to(cdt).cuda()

    for _ in range(args.warmup):
        plan.apply(x)
    torch.cuda.synchronize()

    # ---- timed region: K applies, per-stage HIP events on the launch streams
    plan.profile(True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        out = plan.apply(x)
    e1.record()
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    stages = plan.stage_times()
    c2p_levels = plan.level_times("child_to_parent")
    cousin_levels = plan.level_times("cousin_eval")
    plan.profile(False)
    ms_step = ms_total / args.steps
    value = nrhs * 1000.0 / ms_step
    log(f"{prec} {nrhs} RHS: {ms_step:.3f} ms/apply; stages {stages}")
    assert plan.misses() == 0
    ws_bytes = plan.stats()["device_bytes"]

    # ---- accuracy against the direct sum on 1000 random targets (every RHS);
    # the same direct sum, timed, is the CPU baseline (extrapolated)
    M = 1000
    idx = inputs.error_subset(args.workload, n, M)
    outh = out.cpu().numpy()
    eps, t_direct, d = None, None, None
    if not args.no_eps:
        t0 = time.time()
        d = oracle.direct(p, a, w.kappa, targets=p[idx], skip=idx)
        t_direct = time.time() - t0
        eps = float(np.linalg.norm(outh[:, idx] - d) / np.linalg.norm(d))
        log(f"eps_M vs direct (M={M}, {nrhs} RHS) = {eps:.3e}; direct sum {t_direct:.1f} s")

    # ---- roofline of the dominant kernel stage (child-to-parent)
    traffic = None
    tf = os.path.join(ROOT, "profiles", f"traffic_child_to_parent_{workload_tag(args.workload, prec, nrhs)}.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if rec.get("kernel_source_hash") == kernel_source_hash():
            traffic = rec.get("hbm_bytes_per_launch")
    roofline = roofline_of(st, stages, c2p_levels, choice, nrhs, args.steps, P, 16 if fp64 else 8, fp64, traffic)

    result = {
        "metric": "IFGF matvecs/s at rel err <=1e-3 (FP64 vs mixed, 1 vs batched RHS); N^2/s",
        "value": round(value, 4),
        "unit": "matvecs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": n, "kappa": w.kappa, "nrhs": nrhs,
                   "precision": "fp64" if fp64 else "mixed (f32 arithmetic, f64 geometry)", "degrees": [3, 5],
                   "leaf_cones": [1, 2, 4], "levels": st["D"]},
        "eps_vs_direct": eps,
        "eps_targets": M,
        "n2_per_s": float(n) * n * value,
        "t_plan_s": round(t_plan, 2),
        "t_autotune_s": round(t_tune, 2),
        "plan_device_bytes": int(st["device_bytes"]),
        "device_bytes_with_workspaces": int(ws_bytes),
        "torch_max_allocated_bytes": int(torch.cuda.max_memory_allocated()),
        "child_to_parent_kernels": {str(k): v for k, v in choice.items()},
        "stage_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in stages.items() if v[1]},
        "cousin_eval_ms_per_level": {str(k): round(v[0] / args.steps, 3) for k, v in cousin_levels.items()},
        "roofline": roofline,
        "paper_context": "Table timings1, N = 6291456 sphere row: one matvec on one CPU core of another machine "
                         "(context only, not a target)",
    }

    if not args.no_extras and args.workload == 5:
        # FP64 at 1 RHS on the same plan (the plain single-RHS FP64 IFGF)
        if fp64:
            x1 = x[:1].contiguous()
            ms1 = time_fn(lambda: plan.apply(x1), 2)
            result["fp64_1rhs_matvecs_per_s"] = round(1000.0 / ms1, 4)
            log(f"fp64 1 RHS: {ms1:.1f} ms")
        del plan, x
        torch.cuda.empty_cache()
        # the mixed path on the same workload and right-hand sides
        t0 = time.time()
        pm = ifgf.Plan(p, w.kappa, precision="mixed", max_nrhs=nrhs, store_levels=0)
        t_pm = time.time() - t0
        xm = torch.from_numpy(a).to(torch.complex64).cuda()
        pm.profile(True)
        msm = time_fn(lambda: pm.apply(xm), 5)
        stm = pm.stage_times()
        pm.profile(False)
        outm = pm.apply(xm).cpu().numpy()
        epsm = float(np.linalg.norm(outm[:, idx] - d) / np.linalg.norm(d)) if d is not None else None
        result.update({
            "mixed_matvecs_per_s": round(nrhs * 1000.0 / msm, 4),
            "mixed_ms_per_step": round(msm, 3),
            "mixed_eps_vs_direct": epsm,
            "mixed_vs_fp64_rel": float(np.linalg.norm(outm - outh) / np.linalg.norm(outh)) if fp64 else None,
            "mixed_t_plan_s": round(t_pm, 2),
            "mixed_child_to_parent_kernels": {str(k): v for k, v in pm.kernel_choice(nrhs).items()},
            "mixed_stage_ms_per_step": {k: round(v[0] / 6, 3) for k, v in stm.items() if v[1]},
        })
        if fp64:
            result["speedup_mixed_vs_fp64"] = round(ms_step / msm, 3)
            if "fp64_1rhs_matvecs_per_s" in result:
                result["speedup_mixed_batched_vs_fp64_1rhs"] = round(
                    result["mixed_matvecs_per_s"] / result["fp64_1rhs_matvecs_per_s"], 3)
        log(f"mixed {nrhs} RHS: {msm:.1f} ms, eps {epsm}")
        del pm, xm
        torch.cuda.empty_cache()
        # the same mixed matvec captured as one hipGraph and replayed
        pg = ifgf.Plan(p, w.kappa, precision="mixed", max_nrhs=nrhs, store_levels=0, use_graph=True)
        xg = torch.from_numpy(a).to(torch.complex64).cuda()
        og = torch.empty_like(xg)
        pg.apply(xg, out=og)
        msg = time_fn(lambda: pg.apply(xg, out=og), 5)
        outg = og.cpu().numpy()
        result["mixed_graph_matvecs_per_s"] = round(nrhs * 1000.0 / msg, 4)
        result["mixed_graph_equals_eager"] = bool(np.array_equal(outg, outm))
        log(f"mixed {nrhs} RHS graph replay: {msg:.1f} ms, equal to eager: {result['mixed_graph_equals_eager']}")
        del pg, xg, og
        torch.cuda.empty_cache()
        result["sphere393216"] = sphere393216_extras(torch, ifgf, inputs, oracle, time_fn, log)
        result["graded_adaptive"] = graded_adaptive_extras(torch, ifgf, inputs, oracle, time_fn, log)
        result["laplace393216"] = laplace_extras(torch, ifgf, inputs, oracle, time_fn, log)

    # ---- the oracle on the host cores: the O1 direct sum above, on M of the
    # N targets, extrapolated to one full matvec of all right-hand sides
    if not args.no_cpu_baseline and t_direct is not None:
        cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        full_s = t_direct * n / M
        result["cpu_baseline"] = {"value": round(nrhs / full_s, 7), "unit": "matvecs/s", "cores": cores,
                                  "kind": "oracle",
                                  "sample": f"FP64 direct sum (the oracle's O(N^2) definition) on {M} random "
                                            f"targets x {n} sources x {nrhs} RHS: {t_direct:.1f} s; extrapolated "
                                            f"x{n // M} to one full matvec ({full_s:.0f} s)",
                                  "extrapolated": True}

    print(json.dumps(result), flush=True)
    return 0


def sphere393216_extras(torch, ifgf, inputs, oracle, time_fn, log) -> dict:
    """The N = 393216, kappa = 32 pi sphere: mixed 1 and 16 RHS (with the
    child-to-parent roofline of each), FP64 1 RHS, adjoint, graph replay,
    target gradient."""
    w = inputs.WORKLOADS[2]
    p = w.points()
    n = p.shape[0]
    a = w.densities()
    res = {"workload": w.name}
    t0 = time.time()
    plan = ifgf.Plan(p, w.kappa, precision="mixed", max_nrhs=16, store_levels=0)
    res["t_plan_s"] = round(time.time() - t0, 2)
    st = plan.stats()
    plan.autotune(1)
    plan.autotune(16)
    x = torch.from_numpy(a).to(torch.complex64).cuda()
    plan.profile(True)
    ms1 = time_fn(lambda: plan.apply(x), 10)
    s1 = plan.stage_times()
    l1 = plan.level_times("child_to_parent")
    plan.profile(False)
    ch1 = plan.kernel_choice(1)
    res["mixed_1rhs_matvecs_per_s"] = round(1000.0 / ms1, 3)
    res["roofline_1rhs"] = roofline_of(st, s1, l1, ch1, 1, 11, 75, 8, False, None)
    res["stage_ms_1rhs"] = {k: round(v[0] / 11, 3) for k, v in s1.items() if v[1]}
    out = plan.apply(x).cpu().numpy()
    idx = inputs.error_subset(2, n, 1000)
    d = oracle.direct(p, a, w.kappa, targets=p[idx], skip=idx)
    res["mixed_eps_vs_direct"] = float(np.linalg.norm(out[:, idx] - d) / np.linalg.norm(d))
    res["adjoint_matvecs_per_s"] = round(1000.0 / time_fn(lambda: plan.adjoint(x), 5), 3)
    g = torch.from_numpy(inputs.densities(402, 1, n)).to(torch.complex64).cuda()
    res["grad_targets_per_s"] = round(1000.0 / time_fn(lambda: plan.grad_targets(x, g), 3), 3)
    x16 = torch.from_numpy(inputs.densities(2, 16, n)).to(torch.complex64).cuda()
    plan.profile(True)
    ms16 = time_fn(lambda: plan.apply(x16), 3)
    s16 = plan.stage_times()
    l16 = plan.level_times("child_to_parent")
    plan.profile(False)
    res["mixed_16rhs_matvecs_per_s"] = round(16 * 1000.0 / ms16, 3)
    res["roofline_16rhs"] = roofline_of(st, s16, l16, plan.kernel_choice(16), 16, 4, 75, 8, False, None)
    res["stage_ms_16rhs"] = {k: round(v[0] / 4, 3) for k, v in s16.items() if v[1]}
    # the same stages with every kernel on one stream: the times above overlap
    # (the cousin stage shares the GPU with the child-to-parent chain)
    os.environ["IFGF_SIDE_STREAM"] = "0"
    plan.profile(True)
    ms16s = time_fn(lambda: plan.apply(x16), 3)
    s16s = plan.stage_times()
    plan.profile(False)
    del os.environ["IFGF_SIDE_STREAM"]
    res["mixed_16rhs_one_stream_matvecs_per_s"] = round(16 * 1000.0 / ms16s, 3)
    res["stage_ms_16rhs_one_stream"] = {k: round(v[0] / 4, 3) for k, v in s16s.items() if v[1]}
    del plan
    torch.cuda.empty_cache()
    gplan = ifgf.Plan(p, w.kappa, precision="mixed", max_nrhs=1, store_levels=0, use_graph=True)
    gplan.autotune(1)
    gout = torch.empty_like(x)
    res["graph_replay_1rhs_matvecs_per_s"] = round(1000.0 / time_fn(lambda: gplan.apply(x, out=gout), 10), 3)
    res["graph_replay_equals_eager"] = bool(np.array_equal(gout.cpu().numpy(), out)) \
        if gplan.kernel_choice(1) == ch1 else None
    del gplan
    torch.cuda.empty_cache()
    p64 = ifgf.Plan(p, w.kappa, precision="fp64", max_nrhs=1, store_levels=0)
    x64 = torch.from_numpy(a).cuda()
    ms64 = time_fn(lambda: p64.apply(x64), 5)
    res["fp64_1rhs_matvecs_per_s"] = round(1000.0 / ms64, 3)
    res["speedup_mixed_vs_fp64_1rhs"] = round(ms64 / ms1, 3)
    res["speedup_mixed16_vs_fp64_1rhs"] = round(16 * ms64 / ms16, 3)
    del p64
    torch.cuda.empty_cache()
    log(f"sphere393216: {res}")
    return res


def laplace_extras(torch, ifgf, inputs, oracle, time_fn, log) -> dict:
    """The Laplace kernel (k = 0) on the N = 393216 sphere, the third row of
    the paper's Table timingsLaplace: constant cone counts per box (reading
    R5 with a_d = 1), levels chosen for at most 8 points per leaf box; node
    counts and leaf cones (3,5) 1x2x4 (the Helmholtz default), (4,6) 2x4x8
    (eps below the paper's) and (5,7) 1x2x4 (eps at the paper's level, node
    counts read at run time); FP64 and mixed at 1 RHS, eps on 1000 targets,
    plan time."""
    w = inputs.WORKLOADS[2]
    p = w.points()
    n = p.shape[0]
    a = w.densities()
    idx = inputs.error_subset(2, n, 1000)
    d = oracle.direct(p, a, 0.0, targets=p[idx], skip=idx)
    res = {"n": n, "kappa": 0.0, "nrhs": 1, "paper_T_acc_s": 16.9, "paper_eps": 1.27e-5}
    for deg, leaf in (((3, 5), (1, 2)), ((4, 6), (2, 4)), ((5, 7), (1, 2))):
        for prec in ("fp64", "mixed"):
            t0 = time.time()
            plan = ifgf.Plan(p, 0.0, precision=prec, max_nrhs=1, store_levels=0, degrees=deg, leaf=leaf)
            t_plan = time.time() - t0
            st = plan.stats()
            x = torch.from_numpy(a).to(torch.complex128 if prec == "fp64" else torch.complex64).cuda()
            ms = time_fn(lambda: plan.apply(x), 5)
            out = plan.apply(x).cpu().numpy()
            res[f"{prec}_deg{deg[0]}{deg[1]}_leaf{leaf[0]}x{leaf[1]}"] = {
                "matvecs_per_s": round(1000.0 / ms, 3), "ms_per_matvec": round(ms, 3), "t_plan_s": round(t_plan, 2),
                "levels": st["D"], "cones": sum(st["n_cones"]), "plan_device_bytes": st["device_bytes"],
                "eps_vs_direct": float(np.linalg.norm(out[:, idx] - d) / np.linalg.norm(d)),
                "misses": plan.misses()}
            del plan, x
            torch.cuda.empty_cache()
    log(f"laplace: {res}")
    return res


def graded_adaptive_extras(torch, ifgf, inputs, oracle, time_fn, log) -> dict:
    """The adaptive octree on a locally refined mesh: the graded sphere (N =
    393216, point density 16x the mean near one pole and 1/16 of it at the
    other), kappa = 32 pi, mixed, 1 RHS.  Uniform trees of 8 levels (leaf
    boxes about a quarter wavelength) and 9 levels against adaptive trees of
    at most 9 levels; rate, eps on 1000 targets, plan time and bytes."""
    kappa = 32.0 * math.pi
    p = inputs.graded_sphere(256)
    n = p.shape[0]
    a = inputs.densities(6, 1, n)
    x = torch.from_numpy(a).to(torch.complex64).cuda()
    idx = inputs.error_subset(6, n, 1000)
    d = oracle.direct(p, a, kappa, targets=p[idx], skip=idx)
    res = {"points": "graded sphere c = 0.25", "n": n, "kappa": kappa, "precision": "mixed", "nrhs": 1}
    for name, levels, lm in (("uniform_D8", 8, 0), ("adaptive_D8_leaf8", 8, 8), ("adaptive_D8_leaf24", 8, 24),
                             ("uniform_D9", 9, 0), ("adaptive_D9_leaf16", 9, 16)):
        t0 = time.time()
        plan = ifgf.Plan(p, kappa, levels=levels, precision="mixed", max_nrhs=1, store_levels=0, leaf_max=lm)
        t_plan = time.time() - t0
        st = plan.stats()
        plan.autotune(1)
        ms = time_fn(lambda: plan.apply(x), 10)
        out = plan.apply(x).cpu().numpy()
        res[name] = {"levels": levels, "leaf_max": lm, "matvecs_per_s": round(1000.0 / ms, 3),
                     "ms_per_matvec": round(ms, 3), "t_plan_s": round(t_plan, 2),
                     "eps_vs_direct": float(np.linalg.norm(out[:, idx] - d) / np.linalg.norm(d)),
                     "plan_device_bytes": st["device_bytes"], "cones": sum(st["n_cones"]),
                     "leaf_boxes": st["n_leaf_boxes"][2:], "near_pairs": st["n_near_pairs"],
                     "misses": plan.misses()}
        del plan
        torch.cuda.empty_cache()
    log(f"graded adaptive: {res}")
    return res


if __name__ == "__main__":
    sys.exit(main())
