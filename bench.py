"""Throughput of the fused three-field MRT step on one MI355X.

Prints one JSON line.  A step advances every node of the workload by one
time step; the library's default launch does three steps per launch
through LDS tiles (two for FP64 storage), bit-identical to one-step
launches, and the one-step kernel is timed beside it.  Workload (default:
the 8192 x 8192 cavity, Ra = 1e7, Da = 1e-5, phi = 0.9, Ste = 0.5,
lambda = 1000, FP32 storage, 67.1 M nodes, 15 GB of double-buffered
populations).  Inputs are resident in HBM before timing;
the timed region is bracketed by HIP events on the stream the kernels run
on.  MLUPS counts every node (walls included) advancing all 27 populations.

Algorithmic HBM bytes per node and step: the stored populations read once
and written once, plus the previous-step source read and written: FP64
448 B, FP32 224 B, FP32 with the FP64 rest enthalpy population 232 B,
split 16-bit 152 B, 16-bit offsets 116 B.  With the D2Q5 thermal fields of
Appendix B (--thermal-lattice 5, 19 populations per node): FP64 320 B,
FP32 160 B, FP32 with the FP64 rest enthalpy population 168 B.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PER_NODE = {"f64": 448, "f32": 224, "f32h64": 232, "f16split": 152, "bf16split": 152, "f16": 116,
                  "bf16": 116}
# The storage form the FP32 configurations are timed in: FP32 populations
# with the rest enthalpy population (which carries H) in FP64, the only
# FP32 form that holds every field within 1e-4 of the FP64 oracle over the
# 256^2 A/B run.
FP32_FORM = "f32h64"
# Algorithmic VALU instructions per node update of the timed forms: those of
# the one-step kernel (no multi-step ring), counted with rocprofv3
# (SQ_INSTS_VALU x 64 / node updates) on the 8192^2 cavity.
ALG_VALU_PER_NODE_STEP = {"f32": 436.3, "f32h64": 468.7}
# The paper's own timings (Table I, present scheme, quad-core 2.33 GHz CPU;
# precision and thread count not stated): context only.
PAPER_TABLE_I = [
    {"grid": "150x150", "Ra": 1e6, "steps": 90000, "cpu_s": 423.79, "steps_per_s": 212.37,
     "MLUPS": 150 * 150 * 212.37 / 1e6},
    {"grid": "300x300", "Ra": 1e8, "steps": 360000, "cpu_s": 11611.81, "steps_per_s": 31.0,
     "MLUPS": 300 * 300 * 31.0 / 1e6},
]
BYTES_PER_NODE_D2Q5 = {"f64": 320, "f32": 160, "f32h64": 168}


def bytes_per_node(precision: str, thermal_lattice: int = 9) -> int:
    return BYTES_PER_NODE_D2Q5[precision] if thermal_lattice == 5 else BYTES_PER_NODE[precision]
PEAK_HBM_GBPS = 8000.0
# VALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = one 64-lane wave
# instruction per CU and clock, 39.3 T lane-instructions/s (unpacked FP32; the
# 157.3 TFLOP/s vector figure counts packed FMAs, 4 flop per lane and clock)
PEAK_VALU_GIPS = 256 * 64 * 2.4
METRIC = "MLUPS (3 coupled MRT fields) + achieved HBM GB/s vs peak; FP16-store vs FP32"
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1701_00702_amd", "csrc", n)
                  for n in ("lbm_kernels.hip", "lbm_node.h", "lbm_internal.h", "lbm_api.hip", "lbm_plan.h",
                            "lbm_tiles.h")] + \
    [os.path.join(ROOT, "paper_1701_00702_amd", "build.py")]


def kernel_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def workload(name: str):
    import lbm_workloads as W
    if name == "c3":
        p, _, seed, prec = W.case_c3()
        return [p], seed, prec, "cavity 8192x8192 Ra=1e7 Da=1e-5 phi=0.9 Ste=0.5 lambda=1000 sigma=1 Nu_i=5"
    if name == "c2":
        p, _, seed, prec = W.case_c2()
        return [p], seed, prec, "cavity 1024x1024 Ra=1e6 Da=1e-4 phi=0.95 Ste=1 lambda=100 Nu_i=10"
    if name == "c4":
        p, _, seed, prec = W.case_c4()
        return [p], seed, prec, "cavity 4096x4096 Ra=1e6 Da=1e-4 phi=0.9 Ste=1 lambda=100 Nu_i=5"
    if name.startswith("bat"):
        # k identical n x n cavities in one batch (bat<k>x<n>)
        k, n = (int(v) for v in name[3:].split("x"))
        p = W.scaled_cavity(W.case_c3()[0], n)
        return [dict(p) for _ in range(k)], 0, "f32", f"{k} cavities {n}x{n}, physics of the 8192x8192 case"
    if name.startswith("sq"):
        # cavity of the 8192^2 physics at another size (sq<n> square, sq<nx>x<ny>)
        dims = [int(v) for v in name[2:].split("x")]
        nx, ny = dims[0], dims[-1]
        p = W.scaled_cavity(W.case_c3()[0], nx, ny)
        return [p], 0, "f32", f"cavity {nx}x{ny}, physics of the 8192x8192 case"
    if name == "c5":
        ps, _, seed, prec = W.case_c5()
        return ps, seed, prec, "256 cavities, sides log-U[64,512] (seed 7), 24198641 nodes"
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profile(sha: str, workload_name: str, precision: str, thermal_lattice: int = 9,
                         steps_per_launch: int = 1):
    """HBM bytes per launch measured with rocprofv3 counters, if the summary
    in profiles/ was taken on the current kernel source."""
    tag = f"{workload_name}_d2q5_{precision}" if thermal_lattice == 5 else f"{workload_name}_{precision}"
    kernel = f"stepk_kernel_k{steps_per_launch}" if steps_per_launch > 1 else "step_kernel"
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{tag}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_sha:\s*(\w+)", text)
    m_b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


def valu_from_profile(sha: str, workload_name: str, precision: str, thermal_lattice: int,
                      steps_per_launch: int):
    """VALU instructions per node and step of the timed kernel, counted with
    rocprofv3 (SQ_INSTS_VALU) on the current kernel source, if profiled."""
    if thermal_lattice != 9:
        return None
    path = os.path.join(ROOT, "profiles", f"valu_step_kernels_{workload_name}_{precision}.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernel_sha:\s*(\w+)", text)
    m_v = re.search(rf"valu_per_node_step_k{steps_per_launch}:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_v or m_sha.group(1) != sha:
        return None
    return float(m_v.group(1))


def make_solver(lbm, torch, params, precision, stream):
    nbytes = lbm.lbm_workspace_bytes(params, precision)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    s = lbm.Solver(params, precision, workspace=(base, nbytes), stream=stream.cuda_stream)
    return s, ws


def time_steps(lbm, torch, s, stream, steps, warmup, looped=False):
    step = lbm.lbm_step_per_cavity if looped else lbm.lbm_step
    step(s.h, warmup)
    lbm.lbm_synchronize(s.h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    step(s.h, steps)
    e1.record(stream)
    lbm.lbm_synchronize(s.h)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)  # ms


def cpu_baseline(params, seed, budget_s=15.0, side=1536):
    """The FP64 oracle on a side x side window of the same cavity (hot-wall
    corner), OpenMP over rows on the host cores.  At 1536^2 its two FP64
    population sets (27 x 8 B x 2 per node) take 1.0 GB, far beyond the
    host's caches, as the GPU workload's state is beyond the GPU's."""
    import oracle
    import lbm_workloads as W
    p = params[0]
    win = (0, 0, min(side, p["nx"]), min(side, p["ny"]))
    d = W.perturbation(seed, win[3], win[2])
    Tf = np.full((win[3], win[2]), p["T_init"])
    Tf[1:, 1:] += d[1:, 1:]
    Tm = np.full_like(Tf, p["T_init"])
    o = oracle.Oracle(p, window=win)
    o.set_initial(Tf, Tm)
    o.step(3)  # first touch of the populations
    t0 = time.perf_counter()
    o.step(5)
    t1 = time.perf_counter()
    per = (t1 - t0) / 5
    n = max(5, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    o.step(n)
    dt = time.perf_counter() - t0
    nodes = win[2] * win[3]
    # the oracle's OpenMP runtime: its thread count, then one thread
    gomp = ctypes.CDLL("libgomp.so.1")
    cores = int(gomp.omp_get_max_threads())
    gomp.omp_set_num_threads(1)
    n1 = max(2, int(budget_s / 3 / max(per * cores, 1e-6)))
    t0 = time.perf_counter()
    o.step(n1)
    dt1 = time.perf_counter() - t0
    gomp.omp_set_num_threads(cores)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    state_gb = nodes * 27 * 8 * 2 / 1e9
    return {"value": nodes * n / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{win[2]}x{win[3]} window at the hot-wall corner of the same cavity, "
                      f"{n} steps, {dt:.1f} s, FP64, {state_gb:.2f} GB of populations (not cache-resident)",
            "single_thread_value": nodes * n1 / dt1 / 1e6, "single_thread_sample": f"{n1} steps, {dt1:.1f} s",
            "host_cpu": model}


def errors_vs_f64(f, d, rf, rd, dT) -> dict:
    """Errors of fields f and diagnostics d against the FP64 ones (rf, rd):
    liquid fraction, melt front (units of L) absolute, hot-wall Nu relative,
    interior T in units of dT, f_l absolute, u over the largest FP64 speed."""
    inner = (slice(1, -1), slice(1, -1))
    umax = max(np.abs(rf["ux"]).max(), np.abs(rf["uy"]).max(), 1e-300)
    return {
        "liquid_fraction": abs(d["liquid_fraction"] - rd["liquid_fraction"]),
        "x_front_mid": abs(d["x_front_mid"] - rd["x_front_mid"]),
        "Nu_hot_rel": abs(d["Nu_hot"] - rd["Nu_hot"]) / max(abs(rd["Nu_hot"]), 1e-300),
        "T_pcm": float(np.abs(f["T_pcm"] - rf["T_pcm"])[inner].max() / dT),
        "T_mf": float(np.abs(f["T_mf"] - rf["T_mf"])[inner].max() / dT),
        "f_l": float(np.abs(f["f_l"] - rf["f_l"])[inner].max()),
        "u": float(max(np.abs(f["ux"] - rf["ux"]).max(), np.abs(f["uy"] - rf["uy"]).max()) / umax),
    }


def short_errors(lbm, p, seed, steps, forms) -> dict:
    """The storage forms against FP64 on the same GPU after a short run (the
    default launch of each form)."""
    import lbm_workloads as W
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    dT = p["T_hot"] - p["T_cold"]
    ref, out = None, {}
    for prec in ["f64"] + list(forms):
        s = lbm.Solver(p, prec)
        s.set_initial(0, T_pcm, T_mf)
        s.step(steps)
        f, d = s.fields(), s.diagnostics(allow_nonfinite=True)
        s.close()
        if ref is None:
            ref = (f, d)
        else:
            out[prec] = errors_vs_f64(f, d, ref[0], ref[1], dT)
    return out


def accuracy(name: str) -> dict:
    """Full-length runs of the 1024^2 (FP32 forms, 200 000 steps) or the
    4096^2 (16-bit forms, 100 000 steps) cavity next to the FP64 path on the
    same GPU, which the parity tests tie to the oracle at 1e-10; the
    oracle itself would need hours at these sizes.  Errors in liquid
    fraction, mid-row melt front, hot-wall Nusselt number and the fields."""
    from paper_1701_00702_amd import lbm
    import lbm_workloads as W
    if name == "c2":
        p, steps, seed, _ = W.case_c2()
        forms = ["f64", "f32", "f32h64"]
    elif name == "c4":
        p, steps, seed, _ = W.case_c4()
        forms = ["f64", "f32", "f32h64", "f16split", "bf16split", "f16", "bf16"]
    else:
        raise SystemExit("--accuracy takes c2 or c4")
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    dT = p["T_hot"] - p["T_cold"]
    chunk = 10000
    out, ref = {}, None
    for prec in forms:
        s = lbm.Solver(p, prec)
        s.set_initial(0, T_pcm, T_mf)
        t0 = time.perf_counter()
        for done in range(0, steps, chunk):
            s.step(min(chunk, steps - done))
            lbm.lbm_synchronize(s.h)
            print(f"accuracy {name} {prec}: {min(done + chunk, steps)} of {steps} steps", file=sys.stderr, flush=True)
        wall = time.perf_counter() - t0
        f, d = s.fields(), s.diagnostics(allow_nonfinite=True)
        s.close()
        row = {"seconds": wall, "liquid_fraction": d["liquid_fraction"], "x_front_mid": d["x_front_mid"],
               "Nu_hot": d["Nu_hot"], "energy_residual": d["energy_residual"], "nonfinite": d["nonfinite"]}
        if ref is None:
            ref = (f, d)
        else:
            row["error_vs_f64"] = errors_vs_f64(f, d, ref[0], ref[1], dT)
        out[prec] = row
        del f
    return {"accuracy": name, "nx": p["nx"], "ny": p["ny"], "steps": steps, "seed": seed,
            "reference": "f64 on the GPU (the FP64 path matches the oracle to 1e-10)", "forms": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--workload", default="c3",
                    help="c2, c3 (default), c4, c5, sq<n> for an n x n cavity (sq<nx>x<ny>), bat<k>x<n> for k of them")
    ap.add_argument("--precision", default=None, choices=[None] + list(BYTES_PER_NODE))
    ap.add_argument("--thermal-lattice", type=int, default=9, choices=[9, 5],
                    help="9: D2Q9 thermal fields (the paper's main method); 5: D2Q5 (Appendix B)")
    ap.add_argument("--block", type=int, default=512)
    ap.add_argument("--npt", type=int, default=1)
    ap.add_argument("--xcd", type=int, default=1)
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--steps-per-launch", type=int, default=0, choices=[0, 1, 2, 3],
                    help="0: the library's default (several steps per launch through LDS where available)")
    ap.add_argument("--tile-shape", type=int, default=None, choices=[0, 1, 2],
                    help="tile shape of the multi-step kernel (0 default, 1 wide, 2 tall)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--forms", action="store_true", help="also time the 16-bit and batched forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp16-store", action="store_true",
                    help="skip the 4096^2 FP16-store vs FP32 timing the default run adds")
    ap.add_argument("--accuracy", default=None, choices=["c2", "c4"],
                    help="only run the full-length error report of the 1024^2 (c2) or 4096^2 (c4) cavity")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration and its bandwidth)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is a design note only)"}))
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        # the same copy timed: the practical HBM ceiling of a pure stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"calibration": "copy", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": dst.numel() * 4, "copies": 13,
                          "copy_GBps": 2 * src.numel() * 4 / (ms * 1e-3) / 1e9}))
        return
    if args.accuracy:
        print(json.dumps(accuracy(args.accuracy)))
        return
    from paper_1701_00702_amd import lbm
    import lbm_workloads as W

    params, seed, prec, desc = workload(args.workload)
    prec = args.precision or (FP32_FORM if prec == "f32" else prec)
    qt = args.thermal_lattice
    if qt == 5:
        if prec not in BYTES_PER_NODE_D2Q5:
            raise SystemExit(f"D2Q5 thermal fields are stored as {sorted(BYTES_PER_NODE_D2Q5)}")
        params = [dict(p, thermal_lattice=5) for p in params]
        desc += ", D2Q5 thermal fields (Appendix B)"
    stream = torch.cuda.Stream()
    s, ws = make_solver(lbm, torch, params, prec, stream)
    for c, p in enumerate(params):
        T_pcm, T_mf = W.initial_temperatures(p, seed + c if len(params) > 1 else seed)
        s.set_initial(c, T_pcm, T_mf)
    if args.autotune:
        launch = lbm.lbm_autotune(s.h, 5, os.path.join(tempfile.gettempdir(), "lbmpcm_autotune_cache.txt"))
    else:
        lbm.lbm_set_launch(s.h, args.block, args.npt, args.xcd, args.persistent,
                           steps_per_launch=args.steps_per_launch or None, tile_shape=args.tile_shape)
        launch = lbm.lbm_get_launch(s.h)
    nodes = sum(p["nx"] * p["ny"] for p in params)
    ms = time_steps(lbm, torch, s, stream, args.steps, args.warmup)
    d = s.diagnostics(0, allow_nonfinite=True)
    ms_step = ms / args.steps
    mlups = nodes / (ms_step * 1e-3) / 1e6
    # A launch reads and writes the state once, whether it advances one step
    # or several (through LDS): bytes are per launch.
    spl = launch["steps_per_launch"]
    alg = bytes_per_node(prec, qt) * nodes
    launch_ms = ms_step * spl
    launch_s = launch_ms * 1e-3
    sha = kernel_sha()
    traffic = traffic_from_profile(sha, args.workload, prec, qt, spl)
    valu_k = valu_from_profile(sha, args.workload, prec, qt, spl)
    valu_1 = valu_from_profile(sha, args.workload, prec, qt, 1)
    hbm = {"algorithmic_bytes_per_launch": alg,
           "algorithmic_GBps": alg / launch_s / 1e9, "algorithmic_frac": alg / launch_s / 1e9 / PEAK_HBM_GBPS,
           "counted_bytes_per_launch": traffic,
           "counted_GBps": None if traffic is None else traffic / launch_s / 1e9,
           "counted_frac": None if traffic is None else traffic / launch_s / 1e9 / PEAK_HBM_GBPS,
           "peak_GBps": PEAK_HBM_GBPS}
    alg_instr = ALG_VALU_PER_NODE_STEP.get(prec) if qt == 9 else None
    if spl > 1 and alg_instr:
        # Several steps per launch through LDS: the launch moves the state
        # once for spl steps and is bound by instruction issue.  Algorithmic
        # work: the one-step update's VALU instructions per node x the node
        # updates of the launch (the ring's redundant updates excluded);
        # peak: one 64-lane VALU instruction per CU and clock.
        alg_ti = alg_instr * nodes * spl / launch_s / 1e12
        roof = {"bound": "alu", "achieved": alg_ti, "peak": PEAK_VALU_GIPS / 1e3, "unit": "T lane-instr/s",
                "frac": alg_ti / (PEAK_VALU_GIPS / 1e3), "traffic": traffic,
                "algorithmic_instructions_per_node_step": alg_instr}
        if valu_k is not None:
            issued = valu_k * nodes * spl / launch_s / 1e12
            roof["issued"] = {"instructions_per_node_step": valu_k, "achieved": issued,
                              "frac": issued / (PEAK_VALU_GIPS / 1e3)}
        if valu_1 is not None:
            roof["counted_one_step_instructions_per_node_step"] = valu_1
    else:
        roof = {"bound": "hbm", "achieved": alg / launch_s / 1e9, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": alg / launch_s / 1e9 / PEAK_HBM_GBPS, "traffic": traffic}
    roof.update({"hbm": hbm, "steps_per_launch": spl, "launch_ms": launch_ms, "kernel_sha": sha})
    single = None
    if spl > 1:
        # the one-step kernel on the same state, for reference
        lbm.lbm_set_launch(s.h, launch["block"], launch["nodes_per_thread"], launch["xcd_remap"],
                           launch["persistent"], steps_per_launch=1, tile_shape=0)
        t1 = time_steps(lbm, torch, s, stream, 100, 10) / 100
        single = {"MLUPS": nodes / (t1 * 1e-3) / 1e6, "ms_per_step": t1,
                  "achieved_GBps": alg / (t1 * 1e-3) / 1e9,
                  "frac": alg / (t1 * 1e-3) / 1e9 / PEAK_HBM_GBPS}
    storage_desc = {"f32h64": "FP32 populations, FP64 rest enthalpy population",
                    "f32": "FP32 populations", "f64": "FP64 populations",
                    "f16split": "FP32 rest populations and bases, FP16 remainders",
                    "bf16split": "FP32 rest populations and bases, BF16 remainders",
                    "f16": "FP16 offsets", "bf16": "BF16 offsets"}[prec]
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if prec == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": desc, "nodes": nodes, "storage": prec, "storage_detail": storage_desc,
                   "thermal_lattice": qt, "launch": launch, "seed": seed,
                   "step_kernel": (f"lbm::stepk_kernel ({launch['steps_per_launch']} fused steps per launch "
                                   "through LDS tiles)" if launch["steps_per_launch"] > 1 else
                                   "lbm::step_kernel (fused pull-stream + NEE walls + 3 MRT collisions)")},
        "roofline": roof,
        "check": {"nonfinite": d["nonfinite"], "liquid_fraction": d["liquid_fraction"],
                  "energy_residual_rel": d["energy_residual"] / max(abs(d["E_int"]), 1e-300)},
        "paper_context": {"table_I_present_scheme": PAPER_TABLE_I,
                          "hardware": "quad-core 2.33 GHz CPU (precision and threads not stated)"},
    }
    if single is not None:
        out["one_step_kernel"] = single
    s.close()
    del ws
    torch.cuda.empty_cache()

    if args.workload == "c3" and qt == 9 and not args.no_fp16_store:
        # The metric's FP16-store vs FP32 comparison on the 4096^2 precision
        # workload: the split FP16 form against the FP32 forms, default launch.
        # Also with one and two steps per launch: where a launch is bound by
        # HBM (one step) the 16-bit store pays; with three it is bound by
        # instruction issue and the codec costs more than the bytes save.
        fp16 = {"workload": workload("c4")[3], "by_steps_per_launch": {}}
        for pr in ("f16split", "f32h64", "f32"):
            ps, sd, _, _ = workload("c4")
            s2, ws2 = make_solver(lbm, torch, ps, pr, stream)
            s2.set_initial(0, *W.initial_temperatures(ps[0], sd))
            n2 = ps[0]["nx"] * ps[0]["ny"]
            l2 = lbm.lbm_get_launch(s2.h)
            for k in (l2["steps_per_launch"], 2, 1):
                lbm.lbm_set_launch(s2.h, l2["block"], l2["nodes_per_thread"], l2["xcd_remap"], l2["persistent"],
                                   steps_per_launch=k, tile_shape=0)
                t = time_steps(lbm, torch, s2, stream, 96, 12) / 96
                rec = {"MLUPS": n2 / (t * 1e-3) / 1e6, "ms_per_step": t, "steps_per_launch": k,
                       "bytes_per_node_step": bytes_per_node(pr),
                       "alg_GBps_per_launch": bytes_per_node(pr) * n2 / (t * k * 1e-3) / 1e9}
                if k == l2["steps_per_launch"]:
                    fp16[pr] = rec
                fp16["by_steps_per_launch"].setdefault(str(k), {})[pr] = rec["MLUPS"]
            s2.close()
            del ws2
            torch.cuda.empty_cache()
        fp16["f16split_over_f32h64"] = fp16["f16split"]["MLUPS"] / fp16["f32h64"]["MLUPS"]
        for k, v in fp16["by_steps_per_launch"].items():
            v["f16split_over_f32"] = v["f16split"] / v["f32"]
        # error against FP64: the same physics on 256^2 for 3000 steps (the
        # full-length 4096^2 errors take minutes: bench.py --accuracy c4)
        pe = W.scaled_cavity(workload("c4")[0][0], 256)
        fp16["error_vs_f64"] = {"workload": "the 4096^2 physics on 256x256, 3000 steps, FP64 on the same GPU",
                                "forms": short_errors(lbm, pe, workload("c4")[1], 3000, ("f16split", "f32h64", "f32"))}
        out["fp16_store_vs_fp32"] = fp16

    if args.forms:
        forms = {}
        for wl, pr, q in (("c3", "f32", 9), ("c3", "f16split", 9), ("c3", "bf16split", 9), ("c3", "f16", 9),
                          ("c3", "bf16", 9), ("c4", "f32", 9), ("c4", "f16split", 9), ("c4", "bf16split", 9),
                          ("c4", "f16", 9), ("c4", "bf16", 9),
                          ("c3", "f32", 5), ("c3", "f32h64", 5), ("c3", "f64", 5), ("c3", "f64", 9)):
            if q == qt and wl == args.workload and pr == prec:
                continue
            ps, sd, _, _ = workload(wl)
            if q == 5:
                ps = [dict(p, thermal_lattice=5) for p in ps]
            s2, ws2 = make_solver(lbm, torch, ps, pr, stream)
            T_pcm, T_mf = W.initial_temperatures(ps[0], sd)
            s2.set_initial(0, T_pcm, T_mf)
            lbm.lbm_set_launch(s2.h, args.block, args.npt, args.xcd, args.persistent,
                               steps_per_launch=args.steps_per_launch or None)
            n2 = ps[0]["nx"] * ps[0]["ny"]
            # 96 steps: whole multi-step launches for two and three steps
            t = time_steps(lbm, torch, s2, stream, 96, 12) / 96
            name = f"{wl}_d2q5_{pr}" if q == 5 else f"{wl}_{pr}"
            sp2 = lbm.lbm_get_launch(s2.h)["steps_per_launch"]
            forms[name] = {"MLUPS": n2 / (t * 1e-3) / 1e6, "ms_per_step": t, "steps_per_launch": sp2,
                           "alg_GBps_per_launch": bytes_per_node(pr, q) * n2 / (t * sp2 * 1e-3) / 1e9}
            s2.close()
            del ws2
            torch.cuda.empty_cache()
        ps, sd, _, _ = workload("c5")
        s2, ws2 = make_solver(lbm, torch, ps, "f32", stream)
        for c, q in enumerate(ps):
            s2.set_initial(c, *W.initial_temperatures(q, sd + c))
        lbm.lbm_set_launch(s2.h, args.block, args.npt, args.xcd, args.persistent,
                           steps_per_launch=args.steps_per_launch or None)
        n2 = sum(q["nx"] * q["ny"] for q in ps)
        t1 = time_steps(lbm, torch, s2, stream, 200, 10) / 200
        t2 = time_steps(lbm, torch, s2, stream, 20, 2, looped=True) / 20
        tuned = lbm.lbm_autotune(s2.h, 3, None)
        t3 = time_steps(lbm, torch, s2, stream, 198, 12) / 198
        forms["c5_batched_f32"] = {"MLUPS": n2 / (t1 * 1e-3) / 1e6, "ms_per_step": t1,
                                   "looped_single_cavity_MLUPS": n2 / (t2 * 1e-3) / 1e6,
                                   "autotuned_MLUPS": n2 / (t3 * 1e-3) / 1e6, "autotuned_launch": tuned}
        s2.close()
        del ws2
        torch.cuda.empty_cache()
        out["forms"] = forms

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, seed)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
