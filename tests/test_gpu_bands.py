"""GPU checks of the banded storage layout: a cavity cut into bands of a
few rows (every step-kernel tile then crosses band boundaries, and the
multi-step tiles' rings reach into the next band) must give the same
populations, sources, wall tallies and diagnostics, bit for bit, as the
same cavity stored in one band, with one, two and three steps per launch."""
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


def _min_rows(nx):
    return max(32, -(-2048 // nx) + 4)


def _c1():
    return W.case_c1()[0]


CASES = {
    "c1": lambda: [_c1()],
    "ragged": lambda: [W.scaled_cavity(_c1(), 67, 45)],
    "corner": lambda: [W.case_corner(100)[0]],
    "mixed_bb": lambda: [dict(W.scaled_cavity(_c1(), 130, 77), wall_type=(1, 2, 2, 1),
                              wall_T=(1.0, 0.0, 0.0, 0.1), solid_treatment=1)],
    "batch": lambda: [W.scaled_cavity(_c1(), 33, 70), W.scaled_cavity(_c1(), 100, 101),
                      W.scaled_cavity(_c1(), 16, 16)],
}


def _run(lbm, ps, prec, steps, spl):
    s = lbm.Solver(ps, prec)
    cfg = lbm.lbm_get_launch(s.h)
    lbm.lbm_set_launch(s.h, cfg["block"], cfg["nodes_per_thread"], cfg["xcd_remap"], cfg["persistent"],
                       steps_per_launch=spl)
    for c, q in enumerate(ps):
        s.set_initial(c, *W.initial_temperatures(q, 30 + c))
    s.step(steps)
    out = [(s.state(c).copy(), s.diagnostics(c)) for c in range(len(ps))]
    s.close()
    return out


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("qt", [9, 5])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("spl", [1, 2, 3])
def test_bands_give_the_same_bits(lbm, case, qt, prec, spl):
    if spl == 3 and prec != "f32":
        pytest.skip("three steps per launch exist for the FP32 forms")
    one = [dict(q, thermal_lattice=qt, band_rows=q["ny"]) for q in CASES[case]()]
    cut = [dict(q, band_rows=_min_rows(q["nx"])) for q in one]
    assert any(q["band_rows"] < q["ny"] for q in cut), "the case must hold more than one band"
    steps = 77
    ref = _run(lbm, one, prec, steps, spl)
    got = _run(lbm, cut, prec, steps, spl)
    for (a, da), (b, db) in zip(ref, got):
        assert np.array_equal(a, b)
        for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction", "Nu_hot", "nonfinite"):
            assert da[k] == db[k], k
        assert db["nonfinite"] == 0
