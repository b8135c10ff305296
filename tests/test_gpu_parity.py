"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Field errors are measured as: temperatures over the wall temperature
difference, liquid fraction and density absolutely, velocity over the
oracle's largest speed.  Bars: 1e-10 for the FP64 form, 1e-4 for the FP32
form (the targets the method is built to), computed on the same seeded
inputs.
"""
import os
import tempfile

import numpy as np
import pytest

import lbm_workloads as W
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm(require_gpu):
    import torch
    torch.cuda.set_device(0)
    from paper_1701_00702_amd import lbm as mod
    return mod


def field_errors(g, r, p, mask=None, umax=None):
    dT = p["T_hot"] - p["T_cold"]
    if mask is None:
        mask = np.ones_like(r["T_pcm"], dtype=bool)
    if umax is None:
        umax = max(np.abs(r["ux"][mask]).max(), np.abs(r["uy"][mask]).max(), 1e-300)
    e = {
        "T_pcm": np.abs(g["T_pcm"] - r["T_pcm"])[mask].max() / dT,
        "T_mf": np.abs(g["T_mf"] - r["T_mf"])[mask].max() / dT,
        "f_l": np.abs(g["f_l"] - r["f_l"])[mask].max(),
        "rho": np.abs(g["rho"] - r["rho"])[mask].max(),
        "ux": np.abs(g["ux"] - r["ux"])[mask].max() / umax,
        "uy": np.abs(g["uy"] - r["uy"])[mask].max() / umax,
    }
    return e


def run_pair(lbm, p, steps, seed, precision="f64", launch=None):
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    s = lbm.Solver(p, precision)
    if launch:
        lbm.lbm_set_launch(s.h, **launch)
    s.set_initial(0, T_pcm, T_mf)
    s.step(steps)
    g, gd = s.fields(), s.diagnostics()
    s.close()
    o = oracle.Oracle(p)
    o.set_initial(T_pcm, T_mf)
    o.step(steps)
    return g, gd, o.fields(), o.diagnostics()


def diag_errors(gd, rd):
    out = {}
    for k in ("liquid_fraction", "x_front_mid"):
        out[k] = abs(gd[k] - rd[k])
    # Nusselt numbers on the scale of a conduction Nusselt number (>= 1): the
    # cold-wall value is ~1e-5 before the front arrives, so a relative error
    # there would only measure cancellation
    for k in ("Nu_hot", "Nu_cold", "Nu_hot_pcm"):
        out[k] = abs(gd[k] - rd[k]) / max(abs(rd[k]), 1.0)
    for k in ("E_int", "M_int", "max_dT_LTNE"):
        out[k] = abs(gd[k] - rd[k]) / max(abs(rd[k]), 1e-300)
    for w in range(4):
        scale = max(abs(rd["E_int"] - rd["E_int0"]), 1.0)
        out[f"flux_E{w}"] = abs(gd["flux_E"][w] - rd["flux_E"][w]) / scale
    return out


def test_fp64_c1_parity(lbm):
    p, _, seed, _ = W.case_c1()
    g, gd, r, rd = run_pair(lbm, p, 2000, seed)
    e = field_errors(g, r, p)
    print("fp64 C1 2000 steps", e)
    assert max(e.values()) < 1e-10, e
    de = diag_errors(gd, rd)
    print(de)
    assert max(de.values()) < 1e-10, de
    assert gd["step"] == 2000


@pytest.mark.parametrize("launch", [dict(block=64, nodes_per_thread=1, xcd_remap=0, persistent=0, steps_per_launch=1),
                                    dict(block=128, nodes_per_thread=2, xcd_remap=1, persistent=0, steps_per_launch=1),
                                    dict(block=256, nodes_per_thread=4, xcd_remap=1, persistent=2, steps_per_launch=1),
                                    dict(block=256, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=2),
                                    dict(block=256, nodes_per_thread=1, xcd_remap=0, persistent=2, steps_per_launch=2)])
def test_fp64_ragged_tiles(lbm, launch):
    # 67 x 45 nodes: several tiles per row and a ragged tail for every shape
    p = W.scaled_cavity(W.case_c1()[0], 67, 45)
    g, gd, r, rd = run_pair(lbm, p, 300, 5, launch=launch)
    e = field_errors(g, r, p)
    assert max(e.values()) < 1e-10, e


def test_fp64_periodic_channel(lbm):
    p = W.make_params(nx=8, ny=33, bc_x=1, gravity_axis=0, porosity=0.9, Ra=30.0, Pr=5.0, Da=0.05,
                      Ste=1.0, k_ratio=10.0, cap_ratio=1.5, Nu_i=0.5, F_phi=-1.0, k_f=0.02,
                      T_hot=1.0, T_cold=0.0, T_init=0.7, T_solidus=0.4, T_liquidus=0.5)
    g, gd, r, rd = run_pair(lbm, p, 800, 9)
    e = field_errors(g, r, p)
    assert max(e.values()) < 1e-10, e
    assert np.abs(r["ux"]).max() > 1e-6


def test_fp64_energy_balance(lbm):
    p, _, seed, _ = W.case_c1()
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    s = lbm.Solver(p, "f64")
    s.set_initial(0, T_pcm, T_mf)
    for n in (1, 37, 500):
        s.step(n)
        d = s.diagnostics()
        assert abs(d["energy_residual"]) <= 1e-12 * abs(d["E_int"]), d
        assert abs(d["mass_residual"]) <= 1e-12 * abs(d["M_int"]), d
    s.close()


def test_fp32_parity_256(lbm):
    p, _, seed, _ = W.case_c2(256)
    g, gd, r, rd = run_pair(lbm, p, 1500, seed, precision="f32")
    e = field_errors(g, r, p)
    print("fp32 256^2 1500 steps", e)
    assert max(e.values()) < 1e-4, e
    assert abs(gd["liquid_fraction"] - rd["liquid_fraction"]) < 1e-4
    assert abs(gd["Nu_hot"] - rd["Nu_hot"]) < 1e-4 * abs(rd["Nu_hot"])


def test_graph_replay_matches_single_launches(lbm):
    p = W.scaled_cavity(W.case_c1()[0], 70, 50)
    T_pcm, T_mf = W.initial_temperatures(p, 3)
    a = lbm.Solver(p, "f32")
    a.set_initial(0, T_pcm, T_mf)
    a.step(101)                      # graph chunks plus single launches
    b = lbm.Solver(p, "f32")
    b.set_initial(0, T_pcm, T_mf)
    for _ in range(101):
        b.step(1)
    assert np.array_equal(a.state().view(np.uint32), b.state().view(np.uint32))
    da, db = a.diagnostics(), b.diagnostics()
    assert da["flux_E"] == db["flux_E"] and da["E_int"] == db["E_int"]
    a.close()
    b.close()


def test_launch_shapes_bitwise_and_deterministic(lbm):
    p = W.scaled_cavity(W.case_c2()[0], 300, 130)
    T_pcm, T_mf = W.initial_temperatures(p, 1)
    ref = None
    # rows of 300 nodes span several tiles for every shape, including the
    # first (non-pulling) step
    for launch in (dict(block=256, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=1),
                   dict(block=256, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=1),
                   dict(block=128, nodes_per_thread=2, xcd_remap=0, persistent=4, steps_per_launch=1),
                   dict(block=64, nodes_per_thread=4, xcd_remap=1, persistent=0, steps_per_launch=1),
                   dict(block=64, nodes_per_thread=1, xcd_remap=0, persistent=0, steps_per_launch=1),
                   dict(block=512, nodes_per_thread=4, xcd_remap=1, persistent=1, steps_per_launch=1),
                   dict(block=512, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=2),
                   dict(block=512, nodes_per_thread=1, xcd_remap=0, persistent=3, steps_per_launch=2),
                   dict(block=512, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=3),
                   dict(block=512, nodes_per_thread=1, xcd_remap=0, persistent=2, steps_per_launch=3)):
        s = lbm.Solver(p, "f32")
        lbm.lbm_set_launch(s.h, **launch)
        s.set_initial(0, T_pcm, T_mf)
        s.step(150)
        st = s.state().view(np.uint32)
        d = s.diagnostics()
        s.close()
        if ref is None:
            ref = (st, d)
        else:
            assert np.array_equal(st, ref[0]), launch
            assert d["flux_E"] == ref[1]["flux_E"]


@pytest.mark.parametrize("prec,n", [("f64", 40), ("f16split", 40), ("bf16split", 40), ("f32h64", 1024)])
def test_save_resume_bitwise(lbm, prec, n):
    # (the 1024^2 state, 117 MB, moves through the 64 MiB buffer in two parts)
    p = W.scaled_cavity(W.case_c1()[0], n, n - 4)
    T_pcm, T_mf = W.initial_temperatures(p, 2)
    a = lbm.Solver(p, prec)
    a.set_initial(0, T_pcm, T_mf)
    a.step(120)
    b = lbm.Solver(p, prec)
    b.set_initial(0, T_pcm, T_mf)
    b.step(55)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        lbm.lbm_save(b.h, path)
        c = lbm.Solver(p, prec)
        lbm.lbm_load(c.h, path)
        assert lbm.lbm_step_count(c.h) == 55
        c.step(65)
        # a file of another format, a truncated one and one with bytes to
        # spare are refused and leave the handle alone
        with open(path, "rb") as f:
            blob = f.read()
        for k, data in enumerate((b"LBMPCM02" + blob[8:], blob[:-1], blob[:len(blob) // 2], blob + b"\0")):
            bad = os.path.join(d, f"bad{k}.bin")
            with open(bad, "wb") as g:
                g.write(data)
            with pytest.raises(lbm.LbmError) as e:
                lbm.lbm_load(c.h, bad)
            assert e.value.status == lbm.LBM_EIO
        assert lbm.lbm_step_count(c.h) == 120
    assert np.array_equal(a.state().view(np.uint8), c.state().view(np.uint8))
    assert a.diagnostics()["flux_E"] == c.diagnostics()["flux_E"]
    for s in (a, b, c):
        s.close()


def test_nonfinite_is_reported(lbm):
    p = W.scaled_cavity(W.case_c1()[0], 32, 32)
    s = lbm.Solver(p, "f32")
    s.step(10)
    assert s.diagnostics()["nonfinite"] == 0
    lbm.lbm_debug_poke(s.h, 0, 10, 12, 1, 3, float("nan"))
    s.step(3)
    d = s.diagnostics(allow_nonfinite=True)
    assert d["status"] == lbm.LBM_ENONFINITE and d["nonfinite"] > 0
    with pytest.raises(lbm.LbmError):
        s.diagnostics()
    s.close()


def test_set_initial_after_step_is_rejected(lbm):
    p = W.scaled_cavity(W.case_c1()[0], 16, 16)
    s = lbm.Solver(p, "f32")
    s.step(1)
    with pytest.raises(lbm.LbmError) as e:
        s.set_initial(0, None, None)
    assert e.value.status == lbm.LBM_ESTATE
    s.close()


def test_torch_workspace_and_stream(lbm):
    import torch
    p, _, seed, _ = W.case_c1()
    nbytes = lbm.lbm_workspace_bytes(p, "f64")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) // 256 * 256
    stream = torch.cuda.Stream()
    s = lbm.Solver(p, "f64", workspace=(base, nbytes), stream=stream.cuda_stream)
    T_pcm, T_mf = W.initial_temperatures(p, seed)
    s.set_initial(0, T_pcm, T_mf)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(300)
    e1.record(stream)
    e1.synchronize()
    assert e0.elapsed_time(e1) > 0
    g = s.fields()
    s.close()
    o = oracle.Oracle(p)
    o.set_initial(T_pcm, T_mf)
    o.step(300)
    e = field_errors(g, o.fields(), p)
    assert max(e.values()) < 1e-10, e
    del ws


def test_zero_and_negative_step_counts(lbm):
    # step(0) leaves the state and the step counter alone; a negative count
    # is an error that changes nothing
    p = W.scaled_cavity(W.case_c1()[0], 16, 12)
    s = lbm.Solver(p, "f32")
    s.set_initial(0, *W.initial_temperatures(p, 0))
    s.step(5)
    a = s.state().copy()
    n = s.diagnostics()["step"]
    s.step(0)
    assert np.array_equal(s.state().view(np.uint32), a.view(np.uint32))
    assert s.diagnostics()["step"] == n
    with pytest.raises(lbm.LbmError):
        s.step(-1)
    assert np.array_equal(s.state().view(np.uint32), a.view(np.uint32))
    s.step(1)
    assert s.diagnostics()["step"] == n + 1
    s.close()
