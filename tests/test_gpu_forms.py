"""GPU checks of the full-size, full-length, 16-bit and batched forms.

* Full-size cavity (8192^2, FP32) in the benchmark's launch shape: after a
  few steps every node depends only on a small neighbourhood of the seeded
  initial state, so the CPU oracle run on small windows (with its own
  light-cone bookkeeping) gives exact expected values for sampled nodes at
  the corners, on the walls and in the interior.
* Full-length runs of the 64^2 FP64 case and the 256^2 FP32 case.
* 16-bit offset storage: errors against the FP64 oracle are measured and
  bounded; the bounds are what the storage rounding allows (the fixed
  offsets round the O(1) enthalpy offsets at 5e-4 / 4e-3 relative per
  step), not parity.
* Batched cavities: each cavity inside the packed launch is bit-identical to
  the same cavity run alone, and to the one-launch-per-cavity schedule; the
  whole 256-cavity set in the benchmark's launch, sampled cavities against
  the oracle.
"""
import numpy as np
import pytest

import lbm_workloads as W
import oracle
from test_gpu_parity import diag_errors, field_errors, run_pair

pytestmark = pytest.mark.gpu

BENCH_LAUNCH = dict(block=512, nodes_per_thread=1, xcd_remap=1, persistent=0)


@pytest.fixture(scope="module")
def lbm(require_gpu):
    import torch
    torch.cuda.set_device(0)
    from paper_1701_00702_amd import lbm as mod
    return mod


def test_fullsize_c3_sampled_windows(lbm):
    p, _, seed, _ = W.case_c3()
    nx, ny = p["nx"], p["ny"]
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    s = lbm.Solver(p, "f32")
    lbm.lbm_set_launch(s.h, **BENCH_LAUNCH)
    s.set_initial(0, T_pcm, T_mf)
    steps = 8
    s.step(steps)
    g = s.fields()
    s.close()
    w = 48
    windows = [(0, 0), (nx - w, ny - w), (0, ny // 2), (nx // 2, 0), (nx // 3, ny // 3),
               (nx - w, 0), (0, ny - w)]
    refs = []
    for (x0, y0) in windows:
        o = oracle.Oracle(p, window=(x0, y0, w, w))
        o.set_initial(T_pcm[y0:y0 + w, x0:x0 + w], T_mf[y0:y0 + w, x0:x0 + w])
        o.step(steps)
        refs.append(o.fields())
    # one velocity scale for all windows: the largest oracle speed sampled
    # (near the hot wall); far from it the flow after 8 steps is ~1e-16
    umax = max(max(np.abs(r["ux"][r["valid"]]).max(), np.abs(r["uy"][r["valid"]]).max())
               for r in refs)
    checked = 0
    for (x0, y0), r in zip(windows, refs):
        mask = r["valid"]
        assert mask.sum() > 100, (x0, y0)
        sub = {k: v[y0:y0 + w, x0:x0 + w] for k, v in g.items()}
        e = field_errors(sub, r, p, mask, umax=umax)
        assert max(e.values()) < 1e-4, ((x0, y0), e)
        checked += int(mask.sum())
    assert checked > 4000


def sampled_windows(lbm, p, seed, precision, steps, w=48):
    """Fields of a full-size cavity in the benchmark's launch next to the
    oracle on windows at the corners, the walls and the interior."""
    nx, ny = p["nx"], p["ny"]
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    s = lbm.Solver(p, precision)
    lbm.lbm_set_launch(s.h, **BENCH_LAUNCH)
    s.set_initial(0, T_pcm, T_mf)
    s.step(steps)
    g, gd = s.fields(), s.diagnostics()
    s.close()
    assert gd["nonfinite"] == 0
    windows = [(0, 0), (nx - w, ny - w), (0, ny // 2), (nx // 2, 0), (nx // 3, ny // 3),
               (nx - w, 0), (0, ny - w)]
    out = []
    for (x0, y0) in windows:
        o = oracle.Oracle(p, window=(x0, y0, w, w))
        o.set_initial(T_pcm[y0:y0 + w, x0:x0 + w], T_mf[y0:y0 + w, x0:x0 + w])
        o.step(steps)
        r = o.fields()
        assert r["valid"].sum() > 100, (x0, y0)
        out.append(({k: v[y0:y0 + w, x0:x0 + w] for k, v in g.items()}, r))
    umax = max(max(np.abs(r["ux"][r["valid"]]).max(), np.abs(r["uy"][r["valid"]]).max()) for _, r in out)
    return [field_errors(sub, r, p, r["valid"], umax=umax) for sub, r in out]


def test_fullsize_c2_sampled_windows(lbm):
    # 1024^2 FP32 case, 8 steps: two three-step launches and one two-step
    p, _, seed, prec = W.case_c2()
    for e in sampled_windows(lbm, p, seed, prec, 8):
        assert max(e.values()) < 1e-4, e


@pytest.mark.parametrize("precision", ["f16split", "bf16split", "f16", "bf16"])
def test_fullsize_c4_16bit_sampled_windows(lbm, precision):
    # 4096^2, the 16-bit forms in the benchmark's launch.  The split form is
    # held to the bars of its full-length test; the fixed-offset forms are
    # characterised (their rounding exceeds the per-step change, see the
    # full-length error test) and only bounded.
    p, _, seed, _ = W.case_c4()
    errs = sampled_windows(lbm, p, seed, precision, 8)
    worst = {k: max(e[k] for e in errs) for k in errs[0]}
    print(precision, worst)
    # measured (8 steps): T 3.4e-6 (split FP16), 1.8e-5 (split BF16),
    # 5.4e-4 (FP16 offsets), 6.9e-3 (BF16 offsets)
    if precision == "f16split":
        assert worst["T_pcm"] < 1e-5 and worst["T_mf"] < 5e-5 and worst["f_l"] < 2e-5, worst
        assert worst["ux"] < 3e-4 and worst["uy"] < 3e-4, worst
    elif precision == "bf16split":
        assert worst["T_pcm"] < 5e-5 and worst["T_mf"] < 4e-4 and worst["f_l"] < 2e-4, worst
        assert worst["ux"] < 1e-3 and worst["uy"] < 1.5e-3, worst
    elif precision == "f16":
        assert worst["T_pcm"] < 1.5e-3 and worst["T_mf"] < 2e-4, worst
    else:
        assert worst["T_pcm"] < 1.5e-2 and worst["T_mf"] < 2e-3, worst


def test_fullsize_c5_bench_launch(lbm):
    # The whole 256-cavity set (24 198 641 nodes) in the benchmark's launch
    # and seeds; 96 steps run as one captured graph of 32 three-step
    # launches.  The smallest and the largest cavity and two others are
    # checked whole against the oracle, and bit for bit against the same
    # cavity run alone; every cavity must stay finite.
    ps, _, seed, prec = W.case_c5()
    temps = [W.initial_temperatures(q, seed + c) for c, q in enumerate(ps)]
    steps = 96
    b = lbm.Solver(ps, prec)
    lbm.lbm_set_launch(b.h, **BENCH_LAUNCH)
    assert lbm.lbm_get_launch(b.h)["steps_per_launch"] == 3
    for c, (tp, tm) in enumerate(temps):
        b.set_initial(c, tp, tm)
    b.step(steps)
    for c in range(len(ps)):
        assert b.diagnostics(c)["nonfinite"] == 0, c
    size = [q["nx"] * q["ny"] for q in ps]
    pick = [int(np.argmin(size)), int(np.argmax(size)), 17, 200]
    for c in pick:
        q = ps[c]
        o = oracle.Oracle(q)
        o.set_initial(*temps[c])
        o.step(steps)
        e = field_errors(b.fields(c), o.fields(), q)
        assert max(e.values()) < 1e-4, (c, q["nx"], q["ny"], e)
        single = lbm.Solver(q, prec)
        lbm.lbm_set_launch(single.h, **BENCH_LAUNCH)
        single.set_initial(0, *temps[c])
        single.step(steps)
        assert np.array_equal(b.state(c).view(np.uint32), single.state().view(np.uint32)), c
        single.close()
    b.close()


def test_fp64_c1_full_length(lbm):
    p, steps, seed, _ = W.case_c1()
    g, gd, r, rd = run_pair(lbm, p, steps, seed)
    e = field_errors(g, r, p)
    de = diag_errors(gd, rd)
    print("C1 FP64 20000 steps", e, de)
    assert max(e.values()) < 1e-10, e
    assert max(de.values()) < 1e-10, de
    assert rd["liquid_fraction"] > 0.6        # well into the melting run
    assert abs(gd["energy_residual"]) < 1e-12 * gd["E_int"]


@pytest.mark.parametrize("precision", ["f32", "f32h64"])
def test_fp32_c2_ab_full_length(lbm, precision):
    p, steps, seed, _ = W.case_c2(256)
    assert steps == 12500
    g, gd, r, rd = run_pair(lbm, p, steps, seed, precision=precision)
    e = field_errors(g, r, p)
    print("C2 A/B 256^2", precision, "12500 steps", e, gd["liquid_fraction"], rd["liquid_fraction"])
    assert abs(gd["liquid_fraction"] - rd["liquid_fraction"]) < 1e-4
    for k in ("Nu_hot", "Nu_hot_pcm"):
        assert abs(gd[k] - rd[k]) < 1e-4 * abs(rd[k]), k
    assert abs(gd["x_front_mid"] - rd["x_front_mid"]) < 1e-4
    for k in ("T_pcm", "T_mf", "ux", "uy", "rho"):
        assert e[k] < 1e-4, (k, e)
    if precision == "f32h64":
        # the form the FP32 configurations are timed in: every field < 1e-4
        assert e["f_l"] < 1e-4, e
    else:
        # Plain FP32 storage (not the timed form) rounds the rest enthalpy
        # population (which carries H ~ 1) every step; the front integrates
        # that error, so f_l on the few front nodes drifts to 2.2e-4 by the
        # end of the run while every other field, the liquid fraction and
        # the front stay < 1e-4.  Pinned as measured.
        assert e["f_l"] < 3e-4, e


@pytest.mark.parametrize("precision", ["f16split", "bf16split", "f16", "bf16"])
def test_16bit_storage_error_vs_fp64(lbm, precision):
    p = W.scaled_cavity(W.case_c4()[0], 256)
    steps = 3000
    g, gd, r, rd = run_pair(lbm, p, steps, 0, precision=precision)
    e = field_errors(g, r, p)
    err = {"liquid_fraction": abs(gd["liquid_fraction"] - rd["liquid_fraction"]),
           "x_front_mid": abs(gd["x_front_mid"] - rd["x_front_mid"]),
           "Nu_hot": abs(gd["Nu_hot"] - rd["Nu_hot"]) / abs(rd["Nu_hot"])}
    print(precision, "fields", e, "diag", err, "fl", gd["liquid_fraction"], rd["liquid_fraction"])
    assert gd["nonfinite"] == 0
    u = max(e["ux"], e["uy"])
    if precision == "f16split":
        # FP32 rest populations and bases carry the conserved content; the
        # FP16 remainders are small, so the fields stay FP32-like (measured:
        # T 1.6e-5, f_l 8.4e-5, u 7.2e-4, liquid fraction 3.5e-6, Nu 1.3e-4)
        assert e["T_pcm"] < 5e-5 and e["T_mf"] < 6e-5 and e["f_l"] < 2e-4, e
        assert err["liquid_fraction"] < 1e-5 and err["x_front_mid"] < 1e-5 and err["Nu_hot"] < 3e-4, err
        assert u < 2e-3, e
    elif precision == "bf16split":
        # the same layout with bfloat16 remainders: eight bits of mantissa
        # (measured: T 4.5e-4, f_l 1.6e-3, u 9.6e-3, liquid fraction 2.4e-5,
        # front 2.1e-5, Nu 1.4e-4)
        assert e["T_pcm"] < 1e-3 and e["T_mf"] < 6e-4 and e["f_l"] < 4e-3, e
        assert err["liquid_fraction"] < 6e-5 and err["x_front_mid"] < 6e-5 and err["Nu_hot"] < 4e-4, err
        assert u < 2.5e-2, e
    elif precision == "f16":
        # Fixed-reference offsets: the enthalpy offsets are O(1), so each
        # step rounds them at ~5e-4 relative, above the per-step change; the
        # run stays finite but drifts.  Characterised, within a factor of
        # about two of the measured errors (T 0.167 of dT, f_l 0.50,
        # liquid fraction 0.0151 of 0.0632, front 0.0095, Nu 0.43): the form
        # fails the run, and a change in how it fails is caught.
        assert 0.08 < e["T_pcm"] < 0.3 and e["f_l"] > 0.25, e
        assert 0.007 < err["liquid_fraction"] < 0.03 and 0.004 < err["x_front_mid"] < 0.02, err
        assert 0.2 < err["Nu_hot"] < 0.9, err
    else:
        # bfloat16 offsets (~4e-3 relative): measured T 0.74, f_l 1.0,
        # liquid fraction 0.046, front 0.041, Nu 1.9
        assert 0.4 < e["T_pcm"] < 1.0 and e["f_l"] > 0.5, e
        assert 0.025 < err["liquid_fraction"] < 0.063 and 0.02 < err["x_front_mid"] < 0.08, err
        assert 1.0 < err["Nu_hot"] < 4.0, err


def test_batched_cavities_bitwise(lbm):
    ps, _, _, _ = W.case_c5()
    pick = sorted(range(len(ps)), key=lambda c: ps[c]["nx"] * ps[c]["ny"])[:5] + [0]
    batch = [ps[c] for c in pick]
    temps = [W.initial_temperatures(q, 100 + i) for i, q in enumerate(batch)]
    steps = 120
    b = lbm.Solver(batch, "f32")
    lbm.lbm_set_launch(b.h, block=256, nodes_per_thread=1, xcd_remap=1, persistent=4)
    for c, (tp, tm) in enumerate(temps):
        b.set_initial(c, tp, tm)
    b.step(steps)
    lp = lbm.Solver(batch, "f32")
    for c, (tp, tm) in enumerate(temps):
        lp.set_initial(c, tp, tm)
    lbm.lbm_step_per_cavity(lp.h, steps)
    for c, q in enumerate(batch):
        single = lbm.Solver(q, "f32")
        single.set_initial(0, *temps[c])
        single.step(steps)
        a = b.state(c).view(np.uint32)
        assert np.array_equal(a, single.state().view(np.uint32)), c
        assert np.array_equal(a, lp.state(c).view(np.uint32)), c
        db, ds = b.diagnostics(c), single.diagnostics()
        assert db["flux_E"] == ds["flux_E"] and db["E_int"] == ds["E_int"]
        single.close()
    # and the smallest cavity against the FP64 oracle
    q = batch[0]
    o = oracle.Oracle(q)
    o.set_initial(*temps[0])
    o.step(steps)
    e = field_errors(b.fields(0), o.fields(), q)
    assert max(e.values()) < 1e-4, e
    b.close()
    lp.close()


def test_autotune_keeps_state(lbm, tmp_path):
    p = W.scaled_cavity(W.case_c2()[0], 512)
    T_pcm, T_mf = W.initial_temperatures(p, 1)
    a = lbm.Solver(p, "f32")
    a.set_initial(0, T_pcm, T_mf)
    a.step(40)
    before = a.state().copy()
    cache = str(tmp_path / "tune.txt")
    cfg = lbm.lbm_autotune(a.h, 3, cache)
    assert cfg["block"] in (128, 256, 512)
    assert np.array_equal(a.state().view(np.uint32), before.view(np.uint32))
    a.step(10)
    b = lbm.Solver(p, "f32")
    b.set_initial(0, T_pcm, T_mf)
    b.step(50)
    assert np.array_equal(a.state().view(np.uint32), b.state().view(np.uint32))
    # a second handle reads the choice from the cache
    assert lbm.lbm_autotune(b.h, 3, cache) == cfg
    a.close()
    b.close()


def test_autotune_batch_picks_a_tile_shape_and_keeps_state(lbm, tmp_path):
    # a batch of uneven cavities (the first twelve of the 256-cavity set):
    # the tuner times every launch shape, tile shapes included, on the live
    # state, keeps it, and stepping on is bitwise the same as without tuning
    ps = W.case_c5()[0][:12]
    temps = [W.initial_temperatures(q, 7 + c) for c, q in enumerate(ps)]
    a = lbm.Solver(ps, "f32h64")
    b = lbm.Solver(ps, "f32h64")
    for c, t in enumerate(temps):
        a.set_initial(c, *t)
        b.set_initial(c, *t)
    a.step(31)
    before = [a.state(c).copy() for c in range(len(ps))]
    cfg = lbm.lbm_autotune(a.h, 2, str(tmp_path / "tune.txt"))
    print("batch autotune", cfg)
    assert cfg["steps_per_launch"] in (1, 2, 3) and cfg["tile_shape"] in (0, 1, 2)
    if cfg["steps_per_launch"] > 1:
        assert cfg["tile_w"] > 0 and cfg["tile_h"] > 0
    for c in range(len(ps)):
        assert np.array_equal(a.state(c).view(np.uint32), before[c].view(np.uint32))
    a.step(30)
    b.step(61)
    for c in range(len(ps)):
        assert np.array_equal(a.state(c).view(np.uint32), b.state(c).view(np.uint32)), c
    a.close()
    b.close()
