"""lbm_diagnostics_noalloc (the allocation-free diagnostics, one fixed device
scratch array per GPU) against lbm_diagnostics on the same state, through
the C ABI: several calls in a row on cavities of decreasing size (each call
reuses the array the previous one wrote), every storage family, a batch
cavity, the periodic channel, the raw initial state, and the size limit.

Per-node values, the Nusselt numbers (same per-node temperatures, same sum
order over the wall rows), the melt front, maxima and counts agree bit for
bit; sums over nodes run in another order and agree to 1e-12 relative.
"""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu

EXACT = ("step", "Fo", "Nu_hot", "Nu_hot_pcm", "Nu_cold", "x_front_mid", "max_dT_LTNE", "u_max",
         "nonfinite", "E_int0", "M_int0")
SUMS = ("liquid_fraction", "E_int", "M_int")


def _compare(a, b):
    for k in EXACT:
        assert a[k] == b[k], (k, a[k], b[k])
    for k in SUMS:
        assert abs(a[k] - b[k]) <= 1e-12 * max(abs(a[k]), 1e-300), (k, a[k], b[k])
    for k in ("flux_E", "flux_M"):
        scale = max(max(abs(v) for v in a[k]), 1e-300)
        for u, v in zip(a[k], b[k]):
            assert abs(u - v) <= 1e-12 * scale, (k, a[k], b[k])
    for k, tot in (("energy_residual", "E_int"), ("mass_residual", "M_int")):
        assert abs(a[k] - b[k]) <= 1e-12 * abs(a[tot]), (k, a[k], b[k])


def _cases():
    c1 = W.case_c1()[0]
    return [
        ("cavity 300x200 FP64", [W.scaled_cavity(c1, 300, 200)], "f64", 0, 400),
        ("cavity 130x97 FP32, raw initial state", [W.scaled_cavity(c1, 130, 97)], "f32", 0, 0),
        ("batch of 3, cavity 1 (90x70) F16_SPLIT",
         [W.scaled_cavity(c1, 50, 40), W.scaled_cavity(c1, 90, 70), W.scaled_cavity(c1, 33, 33)], "f16split", 1, 150),
        ("cavity 64x48 D2Q5 FP32_H64", [dict(W.scaled_cavity(c1, 64, 48), thermal_lattice=5)], "f32h64", 0, 120),
        ("periodic channel 4x17 FP64",
         [W.make_params(nx=4, ny=17, bc_x=1, gravity_axis=0, porosity=0.9, Ra=100.0, Pr=5.0, Da=0.05,
                        Ste=1.0, k_ratio=1.0, cap_ratio=1.0, Nu_i=0.0, k_f=0.02, T_hot=1.0, T_cold=0.0,
                        T_init=1.0, T_solidus=-2.0, T_liquidus=-1.0)], "f64", 0, 60),
        ("cavity 6x5 FP32 (fewer columns than the six wall columns apart)",
         [W.scaled_cavity(c1, 6, 5)], "f32", 0, 30),
    ]


def test_noalloc_diagnostics_match_lbm_diagnostics(require_gpu):
    from paper_1701_00702_amd import lbm
    for name, ps, prec, cav, steps in _cases():
        print(f"noalloc diagnostics: {name}, {steps} steps", flush=True)
        s = lbm.Solver(ps, prec)
        for c, p in enumerate(ps):
            s.set_initial(c, *W.initial_temperatures(p, 3 + c))
        s.step(steps)
        a = s.diagnostics(cav)
        b = lbm.lbm_diagnostics_noalloc(s.h, cav)
        _compare(a, b)
        # a second call on the same state gives the same bits
        b2 = lbm.lbm_diagnostics_noalloc(s.h, cav)
        assert b2 == b
        s.close()


def test_noalloc_diagnostics_rejects_sides_beyond_its_scratch(require_gpu):
    from paper_1701_00702_amd import lbm
    p = W.scaled_cavity(W.case_c1()[0], 32769, 4)
    print("noalloc diagnostics: cavity 32769x4 FP32 (beyond the limit)", flush=True)
    s = lbm.Solver(p, "f32")
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_diagnostics_noalloc(s.h, 0)
    assert e.value.status == lbm.LBM_EINVAL and "32768" in str(e.value)
    s.diagnostics()   # the workspace path still serves it
    s.close()
