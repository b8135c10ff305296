"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and its host-only parameter mapping
and validation agree with the paper's printed numbers and with the CPU
oracle's mapping."""
import os
import re

import pytest

import lbm_workloads as W
from oracle.mapping import lattice_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbmpcm.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char \*|lbm_status|int64_t)\s*(lbm_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1701_00702_amd import lbm
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lbm._lib, n), n
        assert n in lbm.EXPORTED, f"binding lacks {n}"
        assert callable(getattr(lbm, n)), f"binding wrapper {n} missing"


def test_host_mapping_matches_paper_and_oracle():
    from paper_1701_00702_amd import lbm
    p, _, _, _ = W.case_p1()
    l = lbm.lbm_lattice_of(p, "f64")
    assert round(l["zeta"][1], 4) == 0.0296          # Sec. V D
    lo = lattice_params(p)
    for k in ("L", "k_f", "k_m", "nu_f", "nu_e", "K", "F_phi", "gbeta", "h_v", "L_a", "d_p", "z",
              "H_fs", "H_fl"):
        assert l[k] == pytest.approx(lo[k], rel=1e-14, abs=1e-300), k
    for k in ("s", "zeta", "eta"):
        assert l[k] == pytest.approx(lo[k], rel=1e-14), k
    # every named workload maps, and the rule for k_f gives the
    # paper's value (tau_h = 2) at lambda = 1000
    for case in (W.case_c1, W.case_c2, W.case_c3, W.case_c4):
        q = case()[0]
        a, b = lbm.lbm_lattice_of(q, "f32"), lattice_params(q)
        assert a["k_f"] == pytest.approx(b["k_f"], rel=1e-14)
        assert a["tau_h"] <= 2.0 + 1e-12 and a["z"] <= 0.5 + 1e-12
    c5, _, _, _ = W.case_c5()
    for q in c5:
        a, b = lbm.lbm_lattice_of(q, "f32"), lattice_params(q)
        assert a["k_f"] == pytest.approx(b["k_f"], rel=1e-14)
        assert a["gbeta"] == pytest.approx(b["gbeta"], rel=1e-14)


@pytest.mark.parametrize("over", [dict(thermal_lattice=5), dict(thermal_lattice=5, varpi=0.4),
                                  dict(thermal_collision=1), dict(thermal_lattice=5, thermal_collision=1),
                                  dict(zeta_e=1.2), dict(thermal_lattice=5, zeta_e=0.6),
                                  dict(wall_type=(1, 2, 1, 0), wall_T=(-1.0, 0.0, 0.5, 0.0)),
                                  dict(L_char=40.0), dict(solid_treatment=1), dict(pcm_even_rates=1),
                                  dict(pcm_even_rates=1, zeta_e=1.5)])
def test_host_mapping_of_variants_matches_oracle(over):
    from paper_1701_00702_amd import lbm
    p = dict(W.case_c1()[0], **over)
    prec = "f64"
    a, b = lbm.lbm_lattice_of(p, prec), lattice_params(p)
    for k in ("L", "k_f", "k_m", "h_v", "d_p", "z", "gbeta", "K", "tau_g", "tau_h", "varpi"):
        assert a[k] == pytest.approx(b[k], rel=1e-14, abs=1e-300), k
    for k in ("s", "zeta", "eta", "wall_T"):
        assert a[k] == pytest.approx(b[k], rel=1e-14), k
    assert a["wall_type"] == b["wall_type"] and a["q_thermal"] == b["qt"]
    assert a["solid_treatment"] == b["solid_treatment"]


def test_corner_case_maps_like_the_oracle():
    from paper_1701_00702_amd import lbm
    p = W.case_corner()[0]
    a, b = lbm.lbm_lattice_of(p, "f64"), lattice_params(p)
    assert a["L"] == 100.0 and a["wall_type"] == [1, 2, 1, 2] and a["wall_T"][0] == -1.0
    assert a["h_v"] == pytest.approx(b["h_v"], rel=1e-14) and a["z"] == pytest.approx(b["z"], rel=1e-14)


def test_host_validation_rejects_bad_sets():
    from paper_1701_00702_amd import lbm
    base = W.case_c1()[0]
    bad = [dict(base, porosity=1.0), dict(base, nx=3), dict(base, cf_ref=1.9), dict(base, Ste=0.0),
           dict(base, k_f=5e-3, Nu_i=60.0), dict(base, T_hot=0.0), dict(base, T_liquidus=-1.0),
           dict(base, bc_x=2), dict(base, thermal_lattice=7), dict(base, thermal_collision=2),
           dict(base, thermal_lattice=5, varpi=1.5), dict(base, thermal_collision=1, zeta_e=1.0),
           dict(base, wall_type=(3, 0, 0, 0)),
           dict(base, bc_x=1, wall_type=(1, 0, 0, 0)), dict(base, solid_treatment=2),
           dict(base, nx=262145, ny=4), dict(base, pcm_even_rates=2),
           dict(base, pcm_even_rates=1, thermal_lattice=5), dict(base, pcm_even_rates=1, thermal_collision=1)]
    for q in bad:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_lattice_of(q, "f32")
        assert e.value.status == lbm.LBM_EINVAL
        assert lbm.lbm_last_error()
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes([base], 7)
    # D2Q5 storage exists in FP64, FP32 and FP32 with the FP64 rest enthalpy
    q5 = dict(base, thermal_lattice=5)
    for prec in ("f16", "bf16", "f16split", "bf16split"):
        with pytest.raises(lbm.LbmError):
            lbm.lbm_lattice_of(q5, prec)
    # a batch shares one thermal lattice
    with pytest.raises(lbm.LbmError):
        lbm.lbm_workspace_bytes([base, q5], "f32")
    # an empty batch, and calls on a NULL handle (any step count)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_workspace_bytes([], "f32")
    assert e.value.status == lbm.LBM_EINVAL
    for call in (lambda: lbm.lbm_step(None, 1), lambda: lbm.lbm_step(None, -1), lambda: lbm.lbm_step(None, 0),
                 lambda: lbm.lbm_synchronize(None)):
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.status == lbm.LBM_EINVAL


def test_workspace_plan_sizes():
    from paper_1701_00702_amd import lbm
    p3 = W.case_c3()[0]
    b32 = lbm.lbm_workspace_bytes(p3, "f32")
    b16 = lbm.lbm_workspace_bytes(p3, "f16")
    n = p3["nx"] * p3["ny"]
    assert b32 >= 2 * 27 * 4 * n and b16 >= 2 * 27 * 2 * n
    assert b32 - b16 >= 2 * 27 * 2 * n * 0.99
    c5 = W.case_c5()[0]
    nodes = sum(q["nx"] * q["ny"] for q in c5)
    assert nodes == 24198641
    assert lbm.lbm_workspace_bytes(c5, "f32") >= 2 * 27 * 4 * nodes
    # D2Q5: 19 populations per node
    q5 = dict(p3, thermal_lattice=5)
    b5 = lbm.lbm_workspace_bytes(q5, "f32")
    assert b5 >= 2 * 19 * 4 * n and b32 - b5 >= 2 * 8 * 4 * n * 0.99
    assert lbm.state_bytes_per_node("f32h64", 5) == 80 and lbm.state_bytes_per_node("f64", 5) == 152


def test_workspace_is_the_state_and_little_else():
    """No per-node scratch beside the state: at 32768^2 the workspace is the
    two state buffers and the two source planes plus under 1% (tile tables,
    wall tallies, a staging area of 2^22 nodes x six doubles), so a 32768^2
    FP32_H64 cavity fits one 288 GiB GPU."""
    from paper_1701_00702_amd import lbm
    n = 32768
    p = W.scaled_cavity(W.case_c1()[0], n, n)
    for prec, sr in (("f32h64", 4), ("f32", 4), ("f16split", 4), ("f16", 4), ("f64", 8)):
        core = (2 * lbm.state_bytes_per_node(prec) + 2 * sr) * n * n
        b = lbm.lbm_workspace_bytes(p, prec)
        assert core <= b <= 1.01 * core, (prec, b, core)
    assert lbm.lbm_workspace_bytes(p, "f32h64") < 0.9 * 288 * 2**30
    # a small cavity stages all its rows at once: six doubles per node
    q = W.case_c1()[0]
    nq = q["nx"] * q["ny"]
    assert lbm.lbm_workspace_bytes(q, "f32") >= (2 * 108 + 8 + 48) * nq


def test_band_rows_validation_and_sizes():
    """Storage bands: 0 (automatic), at least max(32, ceil(2048 / nx) + 4)
    rows, or the whole cavity; a cut layout never needs less memory."""
    from paper_1701_00702_amd import lbm
    p = W.case_c1()[0]                                   # 64 x 64: minimum 36 rows
    b_one = lbm.lbm_workspace_bytes(dict(p, band_rows=64), "f32")
    b_cut = lbm.lbm_workspace_bytes(dict(p, band_rows=36), "f32")
    assert b_cut >= b_one == lbm.lbm_workspace_bytes(p, "f32")
    assert lbm.lbm_workspace_bytes(dict(p, band_rows=500), "f32") == b_one   # clipped to ny
    for bad in (-1, 5, 35):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_workspace_bytes(dict(p, band_rows=bad), "f32")
        assert e.value.status == lbm.LBM_EINVAL


def test_binding_structs_match_the_header_layout(tmp_path):
    """The ctypes mirrors of lbm_params, lbm_lattice, lbm_diag and
    lbm_launch_config have the header's sizes and field offsets (a C99
    program built against the header prints them; no library call)."""
    import ctypes
    import shutil
    import subprocess
    from paper_1701_00702_amd import lbm
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"lbm_params": lbm.lbm_params, "lbm_lattice": lbm.lbm_lattice, "lbm_diag": lbm.lbm_diag,
               "lbm_launch_config": lbm.lbm_launch_config}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lbmpcm.h"', "int main(void) {"]
    for s, py in structs.items():
        lines.append(f'    printf("{s} size %zu\\n", sizeof({s}));')
        for name, _ in py._fields_:
            lines.append(f'    printf("{s} {name} %zu\\n", offsetof({s}, {name}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        parts = line.split()
        s, py = parts[0], structs[parts[0]]
        if parts[1] == "size":
            assert ctypes.sizeof(py) == int(parts[2]), line
        else:
            assert getattr(py, parts[1]).offset == int(parts[2]), line
        seen += 1
    assert seen == len(structs) + sum(len(py._fields_) for py in structs.values())


def test_lent_workspace_is_checked_before_any_device_call():
    """lbm_create_ext refuses a NULL, short or misaligned workspace with
    LBM_EINVAL before it touches the device (the pointers below are never
    dereferenced)."""
    from paper_1701_00702_amd import lbm
    p = W.case_c1()[0]
    need = lbm.lbm_workspace_bytes(p, "f32")
    for ptr, size in ((0, need), (1 << 40, need - 1), ((1 << 40) + 128, need)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_create_ext([p], "f32", ptr, size, 0)
        assert e.value.status == lbm.LBM_EINVAL, (ptr, size)


def test_every_entry_point_refuses_a_null_handle():
    """Each call on a NULL handle returns LBM_EINVAL with a message and no
    device call; lbm_destroy(NULL) is a no-op and lbm_step_count(NULL) is -1."""
    import ctypes
    from paper_1701_00702_amd import lbm
    L = lbm._lib
    d, lat, cfg = lbm.lbm_diag(), lbm.lbm_lattice(), lbm.lbm_launch_config()
    buf = (ctypes.c_double * 4)()
    dp = ctypes.cast(buf, ctypes.POINTER(ctypes.c_double))
    calls = {
        "lbm_set_stream": lambda: L.lbm_set_stream(None, None),
        "lbm_set_initial": lambda: L.lbm_set_initial(None, 0, None, None),
        "lbm_step": lambda: L.lbm_step(None, 1),
        "lbm_step_per_cavity": lambda: L.lbm_step_per_cavity(None, 1),
        "lbm_synchronize": lambda: L.lbm_synchronize(None),
        "lbm_fields": lambda: L.lbm_fields(None, 0, dp, dp, dp, dp, dp, dp),
        "lbm_fields_rows": lambda: L.lbm_fields_rows(None, 0, 0, 1, dp, dp, dp, dp, dp, dp),
        "lbm_diagnostics": lambda: L.lbm_diagnostics(None, 0, ctypes.byref(d)),
        "lbm_diagnostics_noalloc": lambda: L.lbm_diagnostics_noalloc(None, 0, ctypes.byref(d)),
        "lbm_get_lattice": lambda: L.lbm_get_lattice(None, 0, ctypes.byref(lat)),
        "lbm_get_launch": lambda: L.lbm_get_launch(None, ctypes.byref(cfg)),
        "lbm_set_launch": lambda: L.lbm_set_launch(None, ctypes.byref(cfg)),
        "lbm_autotune": lambda: L.lbm_autotune(None, 2, None, ctypes.byref(cfg)),
        "lbm_save": lambda: L.lbm_save(None, b"/nonexistent/x"),
        "lbm_load": lambda: L.lbm_load(None, b"/nonexistent/x"),
        "lbm_copy_state": lambda: L.lbm_copy_state(None, 0, ctypes.cast(buf, ctypes.c_void_p), 32),
        "lbm_debug_poke": lambda: L.lbm_debug_poke(None, 0, 1, 1, 0, 1, 0.0),
    }
    for name, call in calls.items():
        assert call() == lbm.LBM_EINVAL, name
        assert lbm.lbm_last_error(), name
    assert L.lbm_destroy(None) == lbm.LBM_OK
    assert L.lbm_step_count(None) == -1
    missing = [n for n in lbm.EXPORTED if n not in calls and n not in (
        "lbm_create", "lbm_create_batch", "lbm_workspace_bytes", "lbm_create_ext", "lbm_lattice_of",
        "lbm_destroy", "lbm_step_count", "lbm_last_error")]
    assert not missing, missing
