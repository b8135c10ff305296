"""CPU replay of the step kernels (tests/host_replay/replay.cpp): the GPU
kernels' own headers built with a host compiler under AddressSanitizer.

* Multi-step launches, in every tile shape: the K-step kernel's workgroups
  are emulated tile by tile (first update of every thread, the middle update's pulls of every
  thread before any of its writes, the last update) with LDS arrays of the
  kernel's exact sizes filled with NaN bit patterns and the headers' bounds
  checks on; the result must equal K one-step updates bit for bit
  (populations, previous-step sources, wall tallies), for every storage
  form with two or three steps per launch, on ragged cavities, the smallest
  cavities, tiles crossing bands of the fewest allowed rows, the periodic
  channel, mixed wall types and the bounce-back variant.
* The one-step per-node path against the oracle: FP64 to 1e-12, the FP32
  forms to 1e-5 over a short run.

No GPU is involved; this is the host-side evidence for the ring and LDS
coverage of the multi-step kernels.
"""
import hashlib
import os
import subprocess

import numpy as np
import pytest

import oracle
import lbm_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host_replay", "replay.cpp")
CSRC = os.path.join(ROOT, "paper_1701_00702_amd", "csrc")
BUILD = os.path.join(ROOT, "tests", "host_replay", "_build")
CXX = "/opt/rocm/llvm/bin/clang++"
HEADERS = ["lbm_node.h", "lbm_plan.h", "lbm_tiles.h", "lbm_internal.h"]


def _binary():
    h = hashlib.sha256(open(SRC, "rb").read())
    for n in HEADERS:
        h.update(open(os.path.join(CSRC, n), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "lbmpcm.h"), "rb").read())
    exe = os.path.join(BUILD, "replay_" + h.hexdigest()[:12])
    if not os.path.exists(exe):
        os.makedirs(BUILD, exist_ok=True)
        flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                 "-fsanitize=address,undefined", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC]
        tmp = f"{exe}.tmp{os.getpid()}"  # parallel test workers each build their own, then rename
        subprocess.check_call([CXX] + flags + ["-o", tmp, SRC])
        os.replace(tmp, exe)
    return exe


@pytest.fixture(scope="module")
def replay():
    if not os.path.exists(CXX):
        pytest.skip("no host clang++")
    return _binary()


def _job(p: dict, **kw) -> str:
    lines = []
    for k in W.PARAM_FIELDS:
        v = p[k]
        if isinstance(v, (list, tuple)):
            lines.append(f"{k} " + " ".join(repr(float(x)) if k == "wall_T" else str(int(x)) for x in v))
        elif k in ("nx", "ny", "bc_x", "gravity_axis", "thermal_lattice", "thermal_collision",
                   "solid_treatment", "band_rows", "pcm_even_rates"):
            lines.append(f"{k} {int(v)}")
        else:
            lines.append(f"{k} {float(v)!r}")
    for k, v in kw.items():
        lines.append(f"{k} {v}")
    return "\n".join(lines) + "\nend\n"


def _run(exe, job):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], input=job, capture_output=True, text=True, env=env, timeout=600)
    return r.returncode, r.stdout + r.stderr


def _geometries():
    c1 = W.case_c1()[0]
    hot = W.scaled_cavity(c1, 37, 29)
    hot["Ra"] = 1e6                       # flow near the hot wall within a few steps
    return {
        "ragged 37x29": hot,
        "smallest 4x4": W.scaled_cavity(c1, 4, 4),
        "thin 5x37": W.scaled_cavity(c1, 5, 37),
        "bands of 34 rows, 70x100": dict(W.scaled_cavity(c1, 70, 100), band_rows=34),
        "periodic channel 6x17": W.make_params(nx=6, ny=17, bc_x=1, gravity_axis=0, porosity=0.9, Ra=100.0,
                                               Pr=5.0, Da=0.05, Ste=1.0, k_ratio=1.0, cap_ratio=1.0, Nu_i=0.0,
                                               k_f=0.02, T_hot=1.0, T_cold=0.0, T_init=1.0, T_solidus=-2.0,
                                               T_liquidus=-1.0),
        "corner walls 100x100": W.case_corner(100)[0],
        "wide 200x60": dict(W.scaled_cavity(c1, 200, 60), Ra=1e6),
        "bounce-back 41x23": dict(W.scaled_cavity(c1, 41, 23), solid_treatment=1, Ra=1e6),
    }


FORMS = [("f32", 9, 3), ("f32", 9, 2), ("f32h64", 9, 3), ("f32h64", 9, 2), ("f16", 9, 3), ("bf16", 9, 3),
         ("f16split", 9, 3), ("f16split", 9, 2), ("bf16split", 9, 3), ("f64", 9, 2), ("f32", 5, 3), ("f32", 5, 2), ("f32h64", 5, 3),
         ("f64", 5, 2)]


@pytest.mark.parametrize("form", FORMS, ids=[f"{p}-q{q}-k{k}" for p, q, k in FORMS])
def test_multi_step_launch_replays_single_steps(replay, form):
    prec, qt, K = form
    for name, p in _geometries().items():
        q = dict(p, thermal_lattice=qt)
        for shape in range(3):      # every tile shape the launch can take
            code, out = _run(replay, _job(q, precision=prec, K=K, shape=shape, launches=2, mode="kstep", seed=7))
            assert code == 0 and "identical" in out, f"{name}, tile shape {shape}: {out}"


@pytest.mark.parametrize("prec,qt,tol", [("f64", 9, 1e-12), ("f64", 5, 1e-12), ("f32", 9, 1e-5),
                                         ("f32h64", 9, 1e-5), ("f32h64", 5, 1e-5)])
def test_one_step_path_matches_the_oracle(replay, tmp_path, prec, qt, tol):
    p = dict(W.scaled_cavity(W.case_c1()[0], 40, 30), thermal_lattice=qt, Ra=1e6)
    steps = 120
    out = tmp_path / "fields.bin"
    code, msg = _run(replay, _job(p, precision=prec, mode="fields", steps=steps, seed=0, out=str(out)))
    assert code == 0, msg
    f = np.fromfile(out, dtype=np.float64).reshape(6, p["ny"], p["nx"])
    # the replay perturbs the interior PCM temperature with its own generator;
    # the oracle starts from the same temperatures, read back from step 0
    code, msg = _run(replay, _job(p, precision="f64", mode="fields", steps=0, seed=0, out=str(out)))
    assert code == 0, msg
    o = oracle.Oracle(p)
    T0 = np.fromfile(out, dtype=np.float64).reshape(6, p["ny"], p["nx"])
    o.set_initial(T0[2], T0[3])
    o.step(steps)
    r = o.fields()
    umax = max(np.abs(r["ux"]).max(), np.abs(r["uy"]).max())
    assert umax > 1e-6
    err = max(np.abs(f[2] - r["T_pcm"]).max(), np.abs(f[3] - r["T_mf"]).max(), np.abs(f[4] - r["f_l"]).max(),
              np.abs(f[0] - r["ux"]).max() / umax, np.abs(f[1] - r["uy"]).max() / umax)
    assert err < tol, err
