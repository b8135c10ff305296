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

BYTES_PER_NODE = {"f64": 448, "f32": 224, "f32h64": 232, "f16split": 152, "f16": 116, "bf16": 116}
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
    if (workload_name, precision, thermal_lattice) != ("c3", "f32", 9):
        return None
    path = os.path.join(ROOT, "profiles", "valu_step_kernels_c3_f32.md")
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


def cpu_baseline(params, seed, budget_s=15.0):
    """The FP64 oracle on a 384 x 384 window of the same cavity (hot-wall
    corner), OpenMP over rows on the host cores."""
    import oracle
    import lbm_workloads as W
    p = params[0]
    win = (0, 0, min(384, p["nx"]), min(384, p["ny"]))
    d = W.perturbation(seed, win[3], win[2])
    Tf = np.full((win[3], win[2]), p["T_init"])
    Tf[1:, 1:] += d[1:, 1:]
    Tm = np.full_like(Tf, p["T_init"])
    o = oracle.Oracle(p, window=win)
    o.set_initial(Tf, Tm)
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
    return {"value": nodes * n / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{win[2]}x{win[3]} window at the hot-wall corner of the same cavity, "
                      f"{n} steps, {dt:.1f} s, FP64",
            "single_thread_value": nodes * n1 / dt1 / 1e6, "single_thread_sample": f"{n1} steps, {dt1:.1f} s",
            "host_cpu": model}


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
        forms = ["f64", "f32", "f32h64", "f16split", "f16", "bf16"]
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
            rf, rd = ref
            inner = (slice(1, -1), slice(1, -1))
            umax = max(np.abs(rf["ux"]).max(), np.abs(rf["uy"]).max(), 1e-300)
            row["error_vs_f64"] = {
                "liquid_fraction": abs(d["liquid_fraction"] - rd["liquid_fraction"]),
                "x_front_mid": abs(d["x_front_mid"] - rd["x_front_mid"]),
                "Nu_hot_rel": abs(d["Nu_hot"] - rd["Nu_hot"]) / max(abs(rd["Nu_hot"]), 1e-300),
                "T_pcm": float(np.abs(f["T_pcm"] - rf["T_pcm"])[inner].max() / dT),
                "T_mf": float(np.abs(f["T_mf"] - rf["T_mf"])[inner].max() / dT),
                "f_l": float(np.abs(f["f_l"] - rf["f_l"])[inner].max()),
                "u": float(max(np.abs(f["ux"] - rf["ux"]).max(), np.abs(f["uy"] - rf["uy"]).max()) / umax),
            }
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
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--forms", action="store_true", help="also time the 16-bit and batched forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    prec = args.precision or prec
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
                           steps_per_launch=args.steps_per_launch or None)
        launch = lbm.lbm_get_launch(s.h)
    nodes = sum(p["nx"] * p["ny"] for p in params)
    ms = time_steps(lbm, torch, s, stream, args.steps, args.warmup)
    d = s.diagnostics(0, allow_nonfinite=True)
    ms_step = ms / args.steps
    mlups = nodes / (ms_step * 1e-3) / 1e6
    # A launch reads and writes the state once, whether it advances one step
    # or several (through LDS); the roofline is per launch.
    spl = launch["steps_per_launch"]
    alg = bytes_per_node(prec, qt) * nodes
    launch_ms = ms_step * spl
    achieved = alg / (launch_ms * 1e-3) / 1e9
    sha = kernel_sha()
    traffic = traffic_from_profile(sha, args.workload, prec, qt, spl)
    valu = valu_from_profile(sha, args.workload, prec, qt, spl)
    single = None
    if spl > 1:
        # the one-step kernel on the same state, for reference
        lbm.lbm_set_launch(s.h, launch["block"], launch["nodes_per_thread"], launch["xcd_remap"],
                           launch["persistent"], steps_per_launch=1)
        t1 = time_steps(lbm, torch, s, stream, 100, 10) / 100
        single = {"MLUPS": nodes / (t1 * 1e-3) / 1e6, "ms_per_step": t1,
                  "achieved_GBps": alg / (t1 * 1e-3) / 1e9,
                  "frac": alg / (t1 * 1e-3) / 1e9 / PEAK_HBM_GBPS}
    out = {
        "metric": METRIC, "value": mlups, "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": desc, "nodes": nodes, "storage": prec, "thermal_lattice": qt, "launch": launch,
                   "seed": seed,
                   "step_kernel": (f"lbm::stepk_kernel ({launch['steps_per_launch']} fused steps per launch "
                                   "through LDS tiles)" if launch["steps_per_launch"] > 1 else
                                   "lbm::step_kernel (fused pull-stream + NEE walls + 3 MRT collisions)")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBPS,
                     "traffic": None if traffic is None else traffic,
                     "algorithmic_bytes_per_launch": alg, "steps_per_launch": spl,
                     "launch_ms": launch_ms, "kernel_sha": sha,
                     # the bytes a one-step sweep would move per step, over the
                     # measured time per step (above peak: temporal blocking)
                     "per_step_equivalent_GBps": alg / (ms_step * 1e-3) / 1e9,
                     "per_step_equivalent_frac": alg / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBPS,
                     # the same kernel against the VALU issue rate: counted
                     # instructions per node-step x node-steps per second
                     "valu": None if valu is None else {
                         "instructions_per_node_step": valu,
                         "achieved_Ginstr_per_s": valu * mlups / 1e3, "peak_Ginstr_per_s": PEAK_VALU_GIPS,
                         "frac": valu * mlups / 1e3 / PEAK_VALU_GIPS}},
        "check": {"nonfinite": d["nonfinite"], "liquid_fraction": d["liquid_fraction"],
                  "energy_residual_rel": d["energy_residual"] / max(abs(d["E_int"]), 1e-300)},
    }
    if single is not None:
        out["one_step_kernel"] = single
    s.close()
    del ws
    torch.cuda.empty_cache()

    if args.forms:
        forms = {}
        for wl, pr, q in (("c3", "f32h64", 9), ("c3", "f16split", 9), ("c3", "f16", 9), ("c3", "bf16", 9),
                          ("c4", "f32", 9), ("c4", "f16split", 9), ("c4", "f16", 9), ("c4", "bf16", 9),
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
        forms["c5_batched_f32"] = {"MLUPS": n2 / (t1 * 1e-3) / 1e6, "ms_per_step": t1,
                                   "looped_single_cavity_MLUPS": n2 / (t2 * 1e-3) / 1e6}
        s2.close()
        del ws2
        torch.cuda.empty_cache()
        out["forms"] = forms

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(params, seed)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
