"""GPU checks of the K-steps-per-launch kernels (K = 2, 3; K = 2 only for FP64):
the state crosses HBM once per K steps through LDS tiles, and the result
must be the same map as K single steps, bit for bit (populations, sources,
FP64 wall tallies and diagnostics), on every geometry the single-step path
handles: walls and corners, periodic channels, ragged and batched cavities,
mixed wall types, the bounce-back alternative, the smallest cavities, both
thermal lattices, FP32, FP64, FP32 with the FP64 rest enthalpy population and
the 16-bit forms, step counts that leave a remainder and graph replays.
"""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm(require_gpu):
    import torch
    torch.cuda.set_device(0)
    from paper_1701_00702_amd import lbm as mod
    return mod


def _c1():
    return W.case_c1()[0]


CASES = {
    "c1": lambda: [_c1()],
    "ragged": lambda: [W.scaled_cavity(_c1(), 67, 45)],
    "periodic": lambda: [W.make_params(nx=9, ny=33, bc_x=1, gravity_axis=0, porosity=0.9, Ra=30.0, Pr=5.0,
                                       Da=0.05, Ste=1.0, k_ratio=10.0, cap_ratio=1.5, Nu_i=0.5, k_f=0.02,
                                       T_hot=1.0, T_cold=0.0, T_init=0.7, T_solidus=0.4, T_liquidus=0.5)],
    "corner": lambda: [W.case_corner(100)[0]],
    "mixed_bb": lambda: [dict(W.scaled_cavity(_c1(), 40, 37), wall_type=(1, 2, 2, 1),
                              wall_T=(1.0, 0.0, 0.0, 0.1), solid_treatment=1)],
    "batch": lambda: [W.scaled_cavity(_c1(), 33, 70), W.scaled_cavity(_c1(), 70, 34),
                      W.scaled_cavity(_c1(), 16, 16)],
    "wide": lambda: [W.scaled_cavity(W.case_c2()[0], 301, 97)],
    # the smallest cavities accepted (4 nodes a side) and thin ones, where
    # every node is a wall node or next to one
    "tiny": lambda: [W.scaled_cavity(_c1(), nx, ny) for (nx, ny) in ((4, 4), (4, 7), (5, 4), (33, 4), (4, 35))],
}


def _run(lbm, ps, prec, steps, spl, chunks, shape=0):
    s = lbm.Solver(ps, prec)
    cfg = lbm.lbm_get_launch(s.h)
    lbm.lbm_set_launch(s.h, cfg["block"], cfg["nodes_per_thread"], cfg["xcd_remap"], cfg["persistent"],
                       steps_per_launch=spl, tile_shape=shape if spl > 1 else 0)
    for c, q in enumerate(ps):
        s.set_initial(c, *W.initial_temperatures(q, 20 + c))
    for n in chunks(steps):
        s.step(n)
    out = [(s.state(c).copy(), s.diagnostics(c)) for c in range(len(ps))]
    s.close()
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("qt", [9, 5])
@pytest.mark.parametrize("prec", ["f32", "f64", "f32h64"])
def test_two_step_is_bitwise_two_single_steps(lbm, case, qt, prec):
    ps = [dict(q, thermal_lattice=qt) for q in CASES[case]()]
    steps = 131      # first (raw) step, graph replays of 32 launches, odd remainder
    ref = _run(lbm, ps, prec, steps, 1, lambda n: [1] * n)
    two = _run(lbm, ps, prec, steps, 2, lambda n: [n])
    mixed = _run(lbm, ps, prec, steps, 2, lambda n: [1, 2, 3, 64, 61])
    for (a, da), (b, db), (m, dm) in zip(ref, two, mixed):
        assert np.array_equal(a, b) and np.array_equal(a, m)
        for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction", "Nu_hot"):
            assert da[k] == db[k] == dm[k], k


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("qt", [9, 5])
@pytest.mark.parametrize("prec", ["f32", "f32h64"])
def test_three_steps_per_launch_are_bitwise_three_single_steps(lbm, case, qt, prec):
    ps = [dict(q, thermal_lattice=qt) for q in CASES[case]()]
    steps = 200      # first (raw) step, graph replays of 32 launches, a remaining pair
    ref = _run(lbm, ps, prec, steps, 1, lambda n: [1] * n)
    three = _run(lbm, ps, prec, steps, 3, lambda n: [n])
    mixed = _run(lbm, ps, prec, steps, 3, lambda n: [1, 2, 3, 4, 97, 93])
    for (a, da), (b, db), (m, dm) in zip(ref, three, mixed):
        assert np.array_equal(a, b) and np.array_equal(a, m)
        for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction", "Nu_hot"):
            assert da[k] == db[k] == dm[k], k


@pytest.mark.parametrize("case", ["c1", "ragged", "periodic", "corner", "batch", "tiny"])
@pytest.mark.parametrize("prec", ["f16split", "bf16split", "f16", "bf16"])
@pytest.mark.parametrize("spl", [2, 3])
def test_16bit_multi_step_is_bitwise_single_steps(lbm, case, prec, spl):
    # the LDS holds the 16-bit codes (and the split form's FP32 rest
    # populations and bases) exactly as the global state stores them
    ps = CASES[case]()
    steps = 100
    ref = _run(lbm, ps, prec, steps, 1, lambda n: [1] * n)
    got = _run(lbm, ps, prec, steps, spl, lambda n: [n])
    for (a, da), (b, db) in zip(ref, got):
        assert np.array_equal(a, b)
        for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction"):
            assert (da[k] == db[k]) or (np.isnan(da[k]) and np.isnan(db[k])), k


def test_smallest_cavities_against_oracle(lbm):
    # each tiny cavity alone, in the default launch, against the FP64 oracle
    import oracle
    from test_gpu_parity import field_errors
    for (nx, ny) in ((4, 4), (4, 7), (5, 4), (33, 4), (4, 35)):
        p = W.scaled_cavity(_c1(), nx, ny)
        T = W.initial_temperatures(p, 3)
        s = lbm.Solver(p, "f64")
        s.set_initial(0, *T)
        s.step(61)
        g = s.fields()
        s.close()
        o = oracle.Oracle(p)
        o.set_initial(*T)
        o.step(61)
        e = field_errors(g, o.fields(), p)
        assert max(e.values()) < 1e-10, (nx, ny, e)


@pytest.mark.parametrize("spl", [2, 3])
@pytest.mark.parametrize("form", [("f32", 9), ("f32h64", 9), ("f32", 5), ("f32h64", 5), ("f64", 9), ("f64", 5),
                                  ("f16split", 9), ("bf16split", 9), ("f16", 9)])
@pytest.mark.parametrize("shape", [1, 2])
def test_every_tile_shape_is_bitwise_single_steps(lbm, spl, form, shape):
    # the alternative tile shapes the autotuner chooses from: the same bits
    # as single steps on ragged, tiny, periodic and batched geometries
    prec, qt = form
    if prec == "f64" and spl == 3:
        pytest.skip("FP64 has two steps per launch at most")
    for case in ("ragged", "tiny", "periodic", "batch", "corner"):
        ps = [dict(q, thermal_lattice=qt) for q in CASES[case]()]
        steps = 101
        ref = _run(lbm, ps, prec, steps, 1, lambda n: [1] * n)
        got = _run(lbm, ps, prec, steps, spl, lambda n: [n], shape)
        for (a, da), (b, db) in zip(ref, got):
            assert np.array_equal(a, b), case
            for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction"):
                assert (da[k] == db[k]) or (np.isnan(da[k]) and np.isnan(db[k])), (case, k)


def test_tile_shape_reported_and_validated(lbm):
    s = lbm.Solver(W.scaled_cavity(_c1(), 50, 40), "f32h64")
    cfg = lbm.lbm_get_launch(s.h)
    assert (cfg["steps_per_launch"], cfg["tile_shape"], cfg["tile_w"], cfg["tile_h"]) == (3, 0, 32, 10)
    lbm.lbm_set_launch(s.h, 512, 1, 1, 0, steps_per_launch=3, tile_shape=1)
    cfg = lbm.lbm_get_launch(s.h)
    assert (cfg["tile_shape"], cfg["tile_w"], cfg["tile_h"]) == (1, 64, 4)
    for bad in (dict(steps_per_launch=3, tile_shape=3), dict(steps_per_launch=1, tile_shape=1),
                dict(steps_per_launch=3, tile_shape=2, persistent=4)):
        kw = dict(dict(persistent=0), **bad)
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_set_launch(s.h, 512, 1, 1, kw.pop("persistent"), **kw)
        assert e.value.status == lbm.LBM_EINVAL
    s.close()
