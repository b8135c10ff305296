"""GPU parity of the thermal-model variants and wall conditions (HIP path
through the C ABI against the FP64 CPU oracle, same seeded inputs):

* D2Q5 thermal fields (Appendix B) in FP64, FP32 and FP32 with the FP64
  rest enthalpy population; ragged tiles, launch shapes, batches and
  checkpoints bit-identical;
* BGK thermal collisions (Sec. V A) on both lattices, the Sec. V D
  zeta_e sweep, and the enthalpy field's stress moments at the rate of e
  and eps, with which the solid stays at the melting temperature (Sec. V C);
* the conduction-induced solidification of Sec. IV A at the paper's
  200 x 200 grid and full length (Fo = 0.02), and mixed wall types;
* the 8192^2 cavity on D2Q5 in the benchmark's launch shape, sampled
  against oracle windows.

Bars as for the D2Q9 path: 1e-10 in FP64, 1e-4 in FP32 (errors as in
test_gpu_parity: temperatures over the wall temperature difference,
velocities over the oracle's largest speed, f_l and rho absolute).
"""
import os
import tempfile

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


def _c1(**over):
    p, _, seed, _ = W.case_c1()
    return dict(p, **over), seed


@pytest.mark.parametrize("over", [dict(thermal_lattice=5), dict(thermal_lattice=5, varpi=0.5),
                                  dict(thermal_collision=1), dict(thermal_lattice=5, thermal_collision=1),
                                  dict(zeta_e=1.8), dict(thermal_lattice=5, zeta_e=0.6), dict(pcm_even_rates=1)],
                         ids=["d2q5", "d2q5_varpi0.5", "d2q9_bgk", "d2q5_bgk", "d2q9_zeta1.8", "d2q5_zeta0.6",
                              "d2q9_even_rates"])
def test_fp64_variant_parity_c1(lbm, over):
    p, seed = _c1(**over)
    g, gd, r, rd = run_pair(lbm, p, 2000, seed)
    e = field_errors(g, r, p)
    de = diag_errors(gd, rd)
    print(over, e, de)
    assert max(e.values()) < 1e-10, e
    assert max(de.values()) < 1e-10, de
    assert abs(gd["energy_residual"]) < 1e-12 * gd["E_int"]


@pytest.mark.parametrize("launch", [dict(block=64, nodes_per_thread=1, xcd_remap=0, persistent=0),
                                    dict(block=256, nodes_per_thread=4, xcd_remap=1, persistent=2)])
def test_fp64_d2q5_ragged_tiles(lbm, launch):
    p = dict(W.scaled_cavity(W.case_c1()[0], 67, 45), thermal_lattice=5)
    g, gd, r, rd = run_pair(lbm, p, 300, 5, launch=launch)
    e = field_errors(g, r, p)
    assert max(e.values()) < 1e-10, e


@pytest.mark.parametrize("precision", ["f32", "f32h64"])
def test_fp32_d2q5_parity_256(lbm, precision):
    p, _, seed, _ = W.case_c2(256)
    p = dict(p, thermal_lattice=5)
    g, gd, r, rd = run_pair(lbm, p, 1500, seed, precision=precision)
    e = field_errors(g, r, p)
    print("d2q5", precision, e)
    assert max(e.values()) < 1e-4, e
    assert abs(gd["liquid_fraction"] - rd["liquid_fraction"]) < 1e-4
    assert abs(gd["Nu_hot"] - rd["Nu_hot"]) < 1e-4 * abs(rd["Nu_hot"])


@pytest.mark.parametrize("precision", ["f32", "f32h64"])
def test_fp32_d2q5_ab_full_length(lbm, precision):
    # the 256^2 A/B case to the same Fourier number as the 1024^2 run
    p, steps, seed, _ = W.case_c2(256)
    p = dict(p, thermal_lattice=5)
    g, gd, r, rd = run_pair(lbm, p, steps, seed, precision=precision)
    e = field_errors(g, r, p)
    print("d2q5 A/B", precision, steps, e, gd["liquid_fraction"], rd["liquid_fraction"])
    assert max(e.values()) < 1e-4, e
    assert abs(gd["liquid_fraction"] - rd["liquid_fraction"]) < 1e-4
    for k in ("Nu_hot", "Nu_hot_pcm"):
        assert abs(gd[k] - rd[k]) < 1e-4 * abs(rd[k]), k
    assert abs(gd["x_front_mid"] - rd["x_front_mid"]) < 1e-4
    inflow = sum(gd["flux_E"])
    assert abs(gd["energy_residual"]) < 1e-4 * inflow


def test_corner_solidification_full_length(lbm):
    # Sec. IV A: 200 x 200, L = 100, Fo = 0.02 (20 000 steps), FP64
    p, steps, _, _ = W.case_corner(200)
    assert steps == 20000
    T0 = np.full((200, 200), p["T_init"])
    s = lbm.Solver(p, "f64")
    s.set_initial(0, T0, T0)
    s.step(steps)
    g, gd = s.fields(), s.diagnostics()
    s.close()
    o = oracle.Oracle(p)
    o.set_initial(T0, T0)
    o.step(steps)
    r, rd = o.fields(), o.diagnostics()
    dT = 1.0
    for k in ("T_pcm", "T_mf"):
        assert np.abs(g[k] - r[k]).max() / dT < 1e-10, k
    assert np.abs(g["f_l"] - r["f_l"]).max() < 1e-10
    assert np.all(g["ux"] == 0.0) and np.all(g["uy"] == 0.0)       # u = 0 at every node
    assert np.abs(g["f_l"] - g["f_l"].T).max() < 1e-12               # symmetric about y = x
    assert abs(gd["liquid_fraction"] - rd["liquid_fraction"]) < 1e-12
    assert gd["liquid_fraction"] < 0.95                               # a solid layer has grown
    assert abs(gd["energy_residual"]) < 1e-12 * abs(gd["E_int"] - gd["E_int0"]) + 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("qt", [9, 5])
def test_mixed_walls_parity_and_wall_values(lbm, precision, qt):
    p = W.make_params(nx=70, ny=52, porosity=0.9, Ra=1e5, Pr=5.0, Da=1e-2, Ste=1.0, k_ratio=5.0,
                      cap_ratio=1.2, Nu_i=0.5, k_f=0.02, T_hot=1.0, T_cold=0.0, T_init=0.2,
                      T_solidus=0.3, T_liquidus=0.35, thermal_lattice=qt,
                      wall_type=(1, 2, 2, 1), wall_T=(1.0, 0.0, 0.0, 0.1))
    g, gd, r, rd = run_pair(lbm, p, 700, 11, precision=precision)
    e = field_errors(g, r, p)
    assert max(e.values()) < (1e-10 if precision == "f64" else 1e-4), e
    assert np.abs(r["ux"]).max() > 1e-5
    # isothermal wall nodes hold their wall temperature (left column, top row)
    tol = 1e-13 if precision == "f64" else 1e-6
    assert np.abs(g["T_pcm"][:, 0] - 1.0).max() < tol and np.abs(g["T_mf"][:, 0] - 1.0).max() < tol
    assert np.abs(g["T_pcm"][-1, 1:] - 0.1).max() < tol


@pytest.mark.parametrize("qt", [5])
def test_fullsize_c3_d2q5_sampled_windows(lbm, qt):
    p, _, seed, _ = W.case_c3()
    p = dict(p, thermal_lattice=qt)
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
    windows = [(0, 0), (nx - w, ny - w), (0, ny // 2), (nx // 2, 0), (nx // 3, ny // 3)]
    refs = []
    for (x0, y0) in windows:
        o = oracle.Oracle(p, window=(x0, y0, w, w))
        o.set_initial(T_pcm[y0:y0 + w, x0:x0 + w], T_mf[y0:y0 + w, x0:x0 + w])
        o.step(steps)
        refs.append(o.fields())
    umax = max(max(np.abs(r["ux"][r["valid"]]).max(), np.abs(r["uy"][r["valid"]]).max()) for r in refs)
    for (x0, y0), r in zip(windows, refs):
        mask = r["valid"]
        assert mask.sum() > 100
        sub = {k: v[y0:y0 + w, x0:x0 + w] for k, v in g.items()}
        e = field_errors(sub, r, p, mask, umax=umax)
        assert max(e.values()) < 1e-4, ((x0, y0), e)


def test_d2q5_launch_shapes_batches_and_checkpoints_bitwise(lbm):
    p = dict(W.scaled_cavity(W.case_c2()[0], 300, 130), thermal_lattice=5)
    T_pcm, T_mf = W.initial_temperatures(p, 1)
    ref = None
    for launch in (dict(block=256, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=1),
                   dict(block=128, nodes_per_thread=2, xcd_remap=0, persistent=4, steps_per_launch=1),
                   dict(block=512, nodes_per_thread=4, xcd_remap=1, persistent=1, steps_per_launch=1),
                   dict(block=512, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=2)):
        s = lbm.Solver(p, "f32")
        lbm.lbm_set_launch(s.h, **launch)
        s.set_initial(0, T_pcm, T_mf)
        s.step(150)
        st = s.state().view(np.uint32)
        s.close()
        if ref is None:
            ref = st
        else:
            assert np.array_equal(st, ref), launch
    # a batch of three cavities: the first is the cavity above
    q2 = dict(W.scaled_cavity(W.case_c1()[0], 90, 64), thermal_lattice=5)
    q3 = dict(W.scaled_cavity(W.case_c1()[0], 33, 70), thermal_lattice=5)
    b = lbm.Solver([p, q2, q3], "f32")
    b.set_initial(0, T_pcm, T_mf)
    b.step(150)
    assert np.array_equal(b.state(0).view(np.uint32), ref)
    b.close()
    # checkpoint and resume in FP32 with the FP64 rest enthalpy population
    a = lbm.Solver(p, "f32h64")
    a.set_initial(0, T_pcm, T_mf)
    a.step(90)
    c = lbm.Solver(p, "f32h64")
    c.set_initial(0, T_pcm, T_mf)
    c.step(40)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "ck.bin")
        lbm.lbm_save(c.h, path)
        e = lbm.Solver(p, "f32h64")
        lbm.lbm_load(e.h, path)
        e.step(50)
    assert np.array_equal(a.state(), e.state())
    for s in (a, c, e):
        s.close()


@pytest.mark.parametrize("qt", [9, 5])
def test_bounce_back_parity(lbm, qt):
    # the Sec. V B alternative on the 64^2 cavity: FP64 to the parity bar,
    # FP32 to 1e-4; solid nodes (f_l < 0.5) at rest exactly
    p, seed = _c1(solid_treatment=1, thermal_lattice=qt)
    g, gd, r, rd = run_pair(lbm, p, 2000, seed)
    e = field_errors(g, r, p)
    de = diag_errors(gd, rd)
    assert max(e.values()) < 1e-10, e
    assert max(de.values()) < 1e-10, de
    solid = g["f_l"] < 0.5
    assert solid.sum() > 1000 and np.all(g["ux"][solid] == 0.0) and np.all(g["uy"][solid] == 0.0)
    g32, gd32, _, _ = run_pair(lbm, p, 2000, seed, precision="f32")
    e32 = field_errors(g32, r, p)
    assert max(e32.values()) < 1e-4, e32


def test_bounce_back_channel_parity(lbm):
    # solid layers along both walls of a periodic porous channel
    import math
    ny, k = 37, 2
    p = W.make_params(nx=4, ny=ny, bc_x=1, gravity_axis=0, porosity=0.9, Ra=2e3, Pr=1875.0, Da=0.05,
                      Ste=1.0, k_ratio=1.0, cap_ratio=1.0, Nu_i=0.0, F_phi=0.0, k_f=1e-4,
                      T_hot=1.0, T_cold=-1.0, T_init=1e-6, T_solidus=0.0, T_liquidus=1e-7,
                      solid_treatment=1)
    T = np.full((ny, 4), 1e-6)
    T[:k + 1] = 0.0
    T[ny - 1 - k:] = 0.0
    s = lbm.Solver(p, "f64")
    s.set_initial(0, T, T)
    s.step(3000)
    g = s.fields()
    s.close()
    o = oracle.Oracle(p)
    o.set_initial(T, T)
    o.step(3000)
    r = o.fields()
    assert np.abs(r["ux"]).max() > 1e-6
    e = field_errors(g, r, p)
    assert max(e.values()) < 1e-10, e
    assert np.all(g["ux"][:k + 1] == 0.0)


@pytest.mark.parametrize("precision", ["f64", "f32h64"])
def test_solid_stays_at_the_melting_temperature(lbm, precision):
    # Sec. V C: T_melt = T_init = T_cold, no interstitial exchange, the 41^2
    # cavity of the Sec. IV B run to Fo = 0.002 in the default launch.  With
    # the stress moments of the enthalpy field at the rate of e and eps
    # (pcm_even_rates) the solid stays at the melting temperature (FP64: to
    # rounding; FP32 populations: within their rounding); with the printed
    # zeta_v = 1.2 it undershoots, as the oracle shows for both sets.
    from oracle.mapping import lattice_params, steps_for_fourier
    q = W.case_p1()[0]
    p = dict(W.scaled_cavity(q, 41), Nu_i=0.0, T_solidus=0.0, T_liquidus=0.002)
    steps = int(round(steps_for_fourier(lattice_params(p), 0.002)))
    T0 = np.full((p["ny"], p["nx"]), p["T_init"])
    low = {}
    for even in (1, 0):
        s = lbm.Solver(dict(p, pcm_even_rates=even), precision)
        s.set_initial(0, T0, T0)
        s.step(steps)
        f = s.fields()
        s.close()
        assert f["f_l"].max() > 0.5 and (f["f_l"] < 1e-9).sum() > 0.2 * f["f_l"].size
        low[even] = f["T_pcm"].min()
    print(precision, steps, low)
    bar = 1e-12 if precision == "f64" else 1e-6
    assert low[1] >= p["T_solidus"] - bar, low
    assert low[0] < p["T_solidus"] - 5e-4, low
