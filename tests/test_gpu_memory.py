"""GPU checks of the memory plan: the staging area that lbm_set_initial and
lbm_fields pass whole rows through (runs of at most 2^22 nodes, so no
per-node copy of the fields sits beside the state), reading row ranges, the
largest square power-of-two cavity of the timed storage form that one GPU
holds, and the largest cavity the library accepts (just under 2^31 nodes)."""
import numpy as np
import pytest

import lbm_workloads as W

pytestmark = pytest.mark.gpu

STAGE_NODES = 1 << 22


@pytest.fixture(scope="module")
def lbm(require_gpu):
    import torch
    torch.cuda.set_device(0)
    from paper_1701_00702_amd import lbm as mod
    return mod


def _c1():
    return W.case_c1()[0]


def _window_errors(p, T_pcm, T_mf, steps, windows, rows_of, w=48):
    """Oracle windows (with their light-cone masks) next to the GPU fields
    that rows_of(y0, w) returns for rows [y0, y0 + w); None for a
    temperature array means T_init everywhere."""
    import oracle
    from test_gpu_parity import field_errors
    out = []
    for (x0, y0) in windows:
        o = oracle.Oracle(p, window=(x0, y0, w, w))
        uniform = np.full((w, w), float(p["T_init"]))
        tf = uniform if T_pcm is None else T_pcm[y0:y0 + w, x0:x0 + w]
        tm = uniform if T_mf is None else T_mf[y0:y0 + w, x0:x0 + w]
        o.set_initial(tf, tm)
        o.step(steps)
        r = o.fields()
        assert r["valid"].sum() > 100, (x0, y0)
        g = rows_of(y0, w)
        out.append(({k: v[:, x0:x0 + w] for k, v in g.items()}, r))
    umax = max(max(np.abs(r["ux"][r["valid"]]).max(), np.abs(r["uy"][r["valid"]]).max()) for _, r in out)
    return [field_errors(sub, r, p, r["valid"], umax=umax) for sub, r in out]


def test_staged_rows(lbm):
    # 2100 x 2100 nodes (4.41e6 > 2^22): the staging area holds 1997 rows,
    # so the seeded initial temperatures go in and the fields come out in
    # two runs; any row range reads the same bits as the whole field, and
    # oracle windows across the run boundary agree
    n = 2100
    p = W.scaled_cavity(_c1(), n, n)
    rows_per_run = STAGE_NODES // n
    assert rows_per_run < n
    T_pcm, T_mf = W.initial_temperatures(p, 6)
    s = lbm.Solver(p, "f32h64")
    s.set_initial(0, T_pcm, T_mf)
    steps = 5
    s.step(steps)
    g = s.fields()
    for (y0, rows) in ((0, n), (0, 1), (n - 1, 1), (rows_per_run - 10, 20), (rows_per_run - 1, 2),
                       (17, rows_per_run), (5, n - 5), (1, rows_per_run + 1)):
        r = s.fields_rows(y0, rows)
        for k in g:
            assert np.array_equal(r[k], g[k][y0:y0 + rows]), (y0, rows, k)
    for (y0, rows) in ((-1, 5), (0, 0), (n - 10, 11), (0, n + 1)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_fields_rows(s.h, 0, n, y0, rows)
        assert e.value.status == lbm.LBM_EINVAL
    d, dn = s.diagnostics(), lbm.lbm_diagnostics_noalloc(s.h, 0)
    s.close()
    assert d["nonfinite"] == 0
    for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction", "Nu_hot", "x_front_mid"):
        assert d[k] == dn[k], k
    b = rows_per_run - 24
    windows = [(0, b), (n // 2, b), (n - 48, b), (0, 0), (n - 48, n - 48)]
    errs = _window_errors(p, T_pcm, T_mf, steps, windows, lambda y0, w: {k: v[y0:y0 + w] for k, v in g.items()})
    for (x0, y0), e in zip(windows, errs):
        assert max(e.values()) < 1e-4, ((x0, y0), e)


def test_staged_rows_in_a_batch(lbm):
    # a batch whose largest cavity (2100 x 2100) sizes the staging area:
    # the wide cavity goes in and out in two runs, the others (one wider
    # than the first is tall, one narrow) in one; every cavity's fields,
    # whole and by row ranges, are those of the same cavity run alone
    ps = [W.scaled_cavity(_c1(), 2100, 2100), W.scaled_cavity(_c1(), 3000, 40), W.scaled_cavity(_c1(), 37, 900)]
    Ts = [W.initial_temperatures(q, 50 + c) for c, q in enumerate(ps)]
    b = lbm.Solver(ps, "f32h64")
    for c, T in enumerate(Ts):
        b.set_initial(c, *T)
    b.step(4)
    for c, (q, T) in enumerate(zip(ps, Ts)):
        a = lbm.Solver(q, "f32h64")
        a.set_initial(0, *T)
        a.step(4)
        ga, gb = a.fields(), b.fields(c)
        a.close()
        for k in ga:
            assert np.array_equal(ga[k], gb[k]), (c, k)
        ny = q["ny"]
        for (y0, rows) in ((0, ny), (ny // 3, ny // 2), (ny - 1, 1)):
            r = b.fields_rows(y0, rows, c)
            for k in ga:
                assert np.array_equal(r[k], ga[k][y0:y0 + rows]), (c, y0, rows, k)
    b.close()


def test_largest_timed_form_cavity(lbm):
    # 32768^2 nodes (1.07e9) in FP32_H64: 250 GB with both state buffers,
    # the largest power-of-two square of that form one GPU's memory holds.
    # The default launch (three steps per launch, graph runs) for 9 steps;
    # oracle windows at the walls, the corners and the interior, read as row
    # ranges; both diagnostics entry points agree bit for bit.  The lattice
    # constants are those of a 128^2 cavity (L = 127), so the flow the hot
    # wall starts in 9 steps is as fast as in the small cases; with
    # L = 32767 the buoyancy (g beta ~ 1/L^3) leaves it ~1e-7 of that, at
    # the floor of FP32 arithmetic.
    import torch
    n = 32768
    p = dict(W.scaled_cavity(_c1(), n, n), L_char=127.0)
    need = lbm.lbm_workspace_bytes(p, "f32h64")
    assert need < 251e9, need
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    print(f"workspace {need / 1e9:.1f} GB, device free {free / 1e9:.1f} of {total / 1e9:.1f} GB", flush=True)
    if total < need * 1.05 or free < need * 1.02:
        pytest.skip(f"the cavity needs {need * 1.02 / 1e9:.0f} GB of free device memory "
                    f"({free / 1e9:.0f} of {total / 1e9:.0f} GB free)")
    w = 48
    windows = [(0, 0), (0, n // 2), (n - w, n - w), (n // 2, 0), (n // 3, n // 3), (n - w, n // 2), (0, n - w)]
    # the seeded perturbation inside the windows only: every other node
    # starts at T_init, and each window's valid nodes depend on the window
    # alone
    T_pcm = np.full((n, n), float(p["T_init"]))
    for k, (x0, y0) in enumerate(windows):
        d = W.perturbation(40 + k, w, w, 1e-6)
        ys, xs = slice(max(y0, 1), min(y0 + w, n - 1)), slice(max(x0, 1), min(x0 + w, n - 1))
        T_pcm[ys, xs] += d[ys.start - y0:ys.stop - y0, xs.start - x0:xs.stop - x0]
    s = lbm.Solver(p, "f32h64")
    cfg = lbm.lbm_get_launch(s.h)
    assert cfg["steps_per_launch"] == 3
    s.set_initial(0, T_pcm, None)
    steps = 9
    s.step(steps)
    d, dn = s.diagnostics(), lbm.lbm_diagnostics_noalloc(s.h, 0)
    assert d["nonfinite"] == 0
    for k in ("flux_E", "flux_M", "E_int", "M_int", "liquid_fraction", "Nu_hot", "x_front_mid"):
        assert d[k] == dn[k], k
    errs = _window_errors(p, T_pcm, None, steps, windows, lambda y0, w: s.fields_rows(y0, w))
    s.close()
    del T_pcm
    for (x0, y0), e in zip(windows, errs):
        assert max(e["T_pcm"], e["T_mf"], e["f_l"], e["rho"]) < 1e-5, ((x0, y0), e)
        assert max(e["ux"], e["uy"]) < 1e-4, ((x0, y0), e)


def test_largest_accepted_cavity(lbm):
    # 46336 x 46344 nodes, just under the 2^31 nodes one cavity may hold, in
    # the FP16 offset form (117 B per node: a 251 GB workspace): node
    # indices, tile tables and reductions at the top of their range.  The
    # default launch for 9 steps from the uniform initial state; oracle
    # windows at the walls and corners within that form's characterised
    # error (its offsets round at 5e-4 relative each step); the
    # allocation-free diagnostics refuse sides above their scratch.
    import torch
    nx, ny = 46336, 46344
    assert ((nx + 63) // 64 * 64) * ny < 2**31 - 4096 and nx * ny > 2**31 - 2**17
    p = dict(W.scaled_cavity(_c1(), nx, ny), L_char=127.0)
    need = lbm.lbm_workspace_bytes(p, "f16")
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    print(f"workspace {need / 1e9:.1f} GB, device free {free / 1e9:.1f} of {total / 1e9:.1f} GB", flush=True)
    if total < need * 1.05 or free < need * 1.02:
        pytest.skip(f"the cavity needs {need * 1.02 / 1e9:.0f} GB of free device memory "
                    f"({free / 1e9:.0f} of {total / 1e9:.0f} GB free)")
    s = lbm.Solver(p, "f16")
    assert lbm.lbm_get_launch(s.h)["steps_per_launch"] == 3
    steps = 9
    s.step(steps)
    d = s.diagnostics()
    assert d["nonfinite"] == 0 and d["liquid_fraction"] > 0
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_diagnostics_noalloc(s.h, 0)
    assert e.value.status == lbm.LBM_EINVAL
    w = 48
    windows = [(0, 0), (0, ny // 2), (nx - w, ny - w), (nx // 2, 0), (nx - w, ny // 2), (0, ny - w)]
    errs = _window_errors(p, None, None, steps, windows, lambda y0, w: s.fields_rows(y0, w))
    s.close()
    worst = {k: max(e[k] for e in errs) for k in errs[0]}
    print(worst)
    # measured: T_pcm 9.7e-5, T_mf 1.2e-4, f_l 6.1e-4, rho 1.4e-8, u 9.3e-5
    assert worst["T_pcm"] < 2.5e-4 and worst["T_mf"] < 2.5e-4 and worst["f_l"] < 1.5e-3, worst
    assert worst["rho"] < 1e-6 and worst["ux"] < 2.5e-4 and worst["uy"] < 2.5e-4, worst
