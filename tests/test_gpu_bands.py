"""GPU checks of the banded storage layout: a cavity cut into bands of a
few rows (every step-kernel tile then crosses band boundaries, and the
multi-step tiles' rings reach into the next band) must give the same
populations, sources, wall tallies and diagnostics, bit for bit, as the
same cavity stored in one band, with one, two and three steps per launch;
and the longest rows accepted, whose bands are the largest blocks the
kernels' 32-bit offsets reach."""
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


def test_longest_rows(lbm):
    # Rows of the greatest accepted length (262 144 nodes: a tile addresses
    # two band blocks by 32-bit offsets) over 70 rows, so the blocks are about
    # 1 GB and the multi-step tiles cross them: three steps per launch bit for
    # bit against single steps, and the FP64 oracle after 9 steps.
    import oracle
    from test_gpu_parity import field_errors
    p = dict(W.scaled_cavity(_c1(), 262144, 70), L_char=127.0)
    T = W.initial_temperatures(p, 4)
    out = []
    for spl in (1, 3):
        s = lbm.Solver(p, "f32h64")
        cfg = lbm.lbm_get_launch(s.h)
        lbm.lbm_set_launch(s.h, cfg["block"], cfg["nodes_per_thread"], cfg["xcd_remap"], 0, steps_per_launch=spl)
        s.set_initial(0, *T)
        s.step(9)
        out.append((s.state().copy(), s.fields()))
        s.close()
    assert np.array_equal(out[0][0].view(np.uint8), out[1][0].view(np.uint8))
    o = oracle.Oracle(p)
    o.set_initial(*T)
    o.step(9)
    e = field_errors(out[1][1], o.fields(), p)
    del o
    assert max(e["T_pcm"], e["T_mf"], e["f_l"], e["rho"]) < 1e-5, e
