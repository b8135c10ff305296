"""Pins of the oracle's thermal-model variants and wall conditions.

* D2Q5 thermal models (Appendix B): the velocity-space equilibria (Eqs. B3,
  B5) against their moment forms (Eqs. B2, B4) through the transformation
  of Eq. (B1); the sound speed c_sT^2 = varpi/2 stated after Eq. (B3); the
  source direction; the collision's conservation and relaxation.
* BGK thermal models (Sec. V A): every thermal rate equal to 1/tau makes the
  moment-space collision the velocity-space BGK update with the source
  spread like the rest equilibrium.
* A fixed zeta_e (Sec. V D) and the rate mapping of both lattices.
* Wall conditions: the default cavity, per-wall isothermal/adiabatic types.
"""
import math

import numpy as np
import pytest

import oracle
from lbm_workloads import case_p1, make_params
from oracle.mapping import lattice_params

EX, EY, W, M9, _ = oracle.lattice_tables()
M5, M5INV = oracle.lattice5_tables()
EX5, EY5 = EX[:5], EY[:5]


def _lp(**over):
    p = make_params(nx=64, ny=64, porosity=0.9, Ra=1e4, Da=1e-4, Ste=1.0, Nu_i=5.0)
    p.update(over)
    return lattice_params(p)


def _weights5(varpi):
    return np.array([1 - varpi] + [varpi / 4] * 4)


# ---------------------------------------------------------------------------
# D2Q5 lattice algebra
# ---------------------------------------------------------------------------

def test_d2q5_transform_rows_and_inverse():
    # Rows of Eq. (B1) as polynomials of the five velocities of Eq. (11):
    # energy density, the two fluxes, |e|^2 and e_x^2 - e_y^2.
    rows = [np.ones(5), EX5, EY5, EX5 ** 2 + EY5 ** 2, EX5 ** 2 - EY5 ** 2]
    np.testing.assert_array_equal(M5, np.array(rows, dtype=float))
    np.testing.assert_allclose(M5INV @ M5, np.eye(5), atol=1e-15)
    np.testing.assert_allclose(M5 @ M5INV, np.eye(5), atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_d2q5_enthalpy_equilibrium_moments(seed):
    # Eq. (B3) against Eq. (B2).
    r = np.random.default_rng(300 + seed)
    H, T, ux, uy = r.uniform(0, 2), r.uniform(-1, 1), 0.05 * r.standard_normal(), 0.05 * r.standard_normal()
    phi, cf, cpl, vp = r.uniform(0.3, 0.99), r.uniform(0.05, 1.7), 1.0, r.uniform(0.1, 0.9)
    n = M5 @ oracle.geq5(H, T, ux, uy, phi, cf, cpl, vp)
    neq = np.array([H, cpl * T * ux / phi, cpl * T * uy / phi, vp * cf * T, 0.0])
    np.testing.assert_allclose(n, neq, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_d2q5_metal_equilibrium_moments(seed):
    # Eq. (B5) against Eq. (B4).
    r = np.random.default_rng(400 + seed)
    Tm, cpm, cm, vp = r.uniform(-1, 2), 1.0, r.uniform(0.05, 1.7), r.uniform(0.1, 0.9)
    n = M5 @ oracle.heq5(Tm, cpm, cm, vp)
    np.testing.assert_allclose(n, [cpm * Tm, 0, 0, vp * cm * Tm, 0], atol=1e-15)


def test_d2q5_sound_speed():
    # The second moment of the equilibrium at rest is c_sT^2 c_f,ref T times
    # the identity with c_sT^2 = varpi / 2, the statement after Eq. (B3).
    for vp in (0.3, 2.0 / 3.0, 0.9):
        g = oracle.geq5(0.7, 0.4, 0.0, 0.0, 0.8, 0.5, 1.0, vp)
        assert abs((EX5 ** 2 * g).sum() - vp / 2 * 0.5 * 0.4) < 1e-16
        assert abs((EY5 ** 2 * g).sum() - vp / 2 * 0.5 * 0.4) < 1e-16
        assert (EX5 * EY5 * g).sum() == 0.0


def test_d2q5_source_direction_is_rest_shape():
    # S (1, 0, 0, varpi, 0) in moment space is S times the rest-state weights
    # (1 - varpi, varpi/4, ...) in velocity space, the shape of Eq. (B5).
    for vp in (0.25, 2.0 / 3.0):
        v = M5INV @ np.array([1.0, 0.0, 0.0, vp, 0.0])
        np.testing.assert_allclose(v, _weights5(vp), atol=1e-16)
        np.testing.assert_allclose(v, oracle.heq5(1.0, 1.0, 1.0, vp), atol=1e-16)


def _node5(r, lp, T=0.5):
    rho = 1 + 1e-3 * r.standard_normal()
    u = 0.02 * r.standard_normal(2)
    fplus = oracle.feq(rho, u[0], u[1], lp["phi"]) + 1e-4 * r.standard_normal(9)
    H = oracle.enthalpy_of_T(lp, T)
    g = np.zeros(9)
    h = np.zeros(9)
    g[:5] = oracle.geq5(H, T, u[0], u[1], lp["phi"], lp["c_fref"], lp["c_pl"], lp["varpi"])
    g[:5] += 1e-5 * r.standard_normal(5)
    Tm = T + 0.01 * r.standard_normal()
    h[:5] = oracle.heq5(Tm, lp["c_pm"], lp["c_mref"], lp["varpi"]) + 1e-5 * r.standard_normal(5)
    return fplus, g, h


@pytest.mark.parametrize("seed", range(4))
def test_d2q5_collision_conserves_and_relaxes(seed):
    lp = _lp(thermal_lattice=5, varpi=0.6, Ra=1e8)
    r = np.random.default_rng(500 + seed)
    fplus, g, h = _node5(r, lp)
    sp, smp = 1e-3 * r.standard_normal(), 1e-3 * r.standard_normal()
    fo, go, ho, sr = oracle.collide_node(lp, fplus, g, h, sp, smp)
    m = oracle.node_macros(lp, fplus, g, h)
    assert np.all(go[5:] == 0) and np.all(ho[5:] == 0)
    S_pcm = sr[0] + 0.5 * (sr[0] - sp)
    S_met = sr[1] + 0.5 * (sr[1] - smp)
    # zeroth moments change by exactly the sources
    assert abs(go.sum() - (m["H"] + S_pcm)) < 1e-14
    assert abs(ho.sum() - (lp["c_pm"] * m["T_m"] + S_met)) < 1e-14
    # fluxes relax at zeta_alpha toward c_pl T u / phi; metal toward zero
    za, ea, vp = lp["zeta"][1], lp["eta"][1], lp["varpi"]
    for e, u in ((EX5, m["ux"]), (EY5, m["uy"])):
        j = (e * g[:5]).sum()
        target = lp["c_pl"] * m["T_f"] * u / lp["phi"]
        assert abs((e * go[:5]).sum() - (j - za * (j - target))) < 1e-15
        assert abs((e * ho[:5]).sum() - (1 - ea) * (e * h[:5]).sum()) < 1e-15
    # |e|^2 moment relaxes at zeta_e toward varpi c_f,ref T, plus varpi S
    ze = lp["zeta"][3]
    e2 = EX5 ** 2 + EY5 ** 2
    n3 = (e2 * g[:5]).sum()
    assert abs((e2 * go[:5]).sum() - (n3 - ze * (n3 - vp * lp["c_fref"] * m["T_f"]) + vp * S_pcm)) < 1e-14


# ---------------------------------------------------------------------------
# Rates: BGK, fixed zeta_e, D2Q5 mapping
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("qt", [9, 5])
def test_bgk_is_velocity_space_bgk(qt):
    # Sec. V A: zeta_i = 1/tau_g and eta_i = 1/tau_h for every moment turns
    # the collision into g* = g - (g - g_eq)/tau_g + w_i S (and likewise h).
    lp = _lp(thermal_lattice=qt, thermal_collision=1, Ra=1e8)
    r = np.random.default_rng(9)
    if qt == 9:
        rho, u = 1.001, (0.01, -0.02)
        fplus = oracle.feq(rho, *u, lp["phi"]) + 1e-4 * r.standard_normal(9)
        H = oracle.enthalpy_of_T(lp, 0.6)
        g = oracle.geq(H, 0.6, *u, lp["phi"], lp["c_fref"], lp["c_pl"]) + 1e-5 * r.standard_normal(9)
        h = oracle.heq(0.55, lp["c_pm"], lp["c_mref"]) + 1e-5 * r.standard_normal(9)
        w = W
    else:
        fplus, g, h = _node5(r, lp, T=0.6)
        w = np.concatenate([_weights5(lp["varpi"]), np.zeros(4)])
    m = oracle.node_macros(lp, fplus, g, h)
    sp, smp = 2e-3, -1e-3
    fo, go, ho, sr = oracle.collide_node(lp, fplus, g, h, sp, smp)
    S_pcm = sr[0] + 0.5 * (sr[0] - sp)
    S_met = sr[1] + 0.5 * (sr[1] - smp)
    tg, th = lp["tau_g"], lp["tau_h"]
    if qt == 9:
        geq = oracle.geq(m["H"], m["T_f"], m["ux"], m["uy"], lp["phi"], lp["c_fref"], lp["c_pl"])
        heq = oracle.heq(m["T_m"], lp["c_pm"], lp["c_mref"])
    else:
        geq = np.concatenate([oracle.geq5(m["H"], m["T_f"], m["ux"], m["uy"], lp["phi"], lp["c_fref"],
                                          lp["c_pl"], lp["varpi"]), np.zeros(4)])
        heq = np.concatenate([oracle.heq5(m["T_m"], lp["c_pm"], lp["c_mref"], lp["varpi"]), np.zeros(4)])
    np.testing.assert_allclose(go, g - (g - geq) / tg + w * S_pcm, rtol=0, atol=1e-15)
    np.testing.assert_allclose(ho, h - (h - heq) / th + w * S_met, rtol=0, atol=1e-15)


def test_fixed_zeta_e_and_rate_tables():
    base = _lp()
    za = base["zeta"][3]
    # a given zeta_e moves the pair zeta_e = zeta_eps that Sec. III C sets
    # together; everything else keeps its Sec. III C value
    lp = _lp(zeta_e=1.8)
    assert lp["zeta"][1] == 1.8 and lp["zeta"][2] == 1.8
    assert base["zeta"][1] == base["zeta"][2] == 2.0 - za
    assert lp["zeta"][3:] == base["zeta"][3:] and lp["eta"] == base["eta"]
    lp5 = _lp(thermal_lattice=5, zeta_e=0.6)
    assert lp5["zeta"][:5] == [1.0, za, za, 0.6, 0.6]
    assert lp5["eta"][:5] == [1.0, base["eta"][3], base["eta"][3], 1.1, 1.1]
    with pytest.raises(ValueError):
        _lp(thermal_collision=1, zeta_e=1.2)
    with pytest.raises(ValueError):
        _lp(thermal_lattice=5, varpi=1.0)
    with pytest.raises(ValueError):
        _lp(thermal_lattice=7)


def test_d2q5_rate_mapping():
    # alpha_ref = c_sT^2 (1/zeta_alpha - 1/2) with c_sT^2 = varpi/2 (App. B);
    # varpi = 2/3 gives the D2Q9 sound speed, so the paper's Sec. IV B rates
    # (zeta_e = 0.0296, Sec. V D) are the same on both lattices.
    p, _, _, _ = case_p1()
    l9 = lattice_params(p)
    l5 = lattice_params(dict(p, thermal_lattice=5))
    assert abs(l5["zeta"][1] - l9["zeta"][3]) < 1e-15
    assert round(l5["zeta"][3], 4) == 0.0296
    l5b = lattice_params(dict(p, thermal_lattice=5, varpi=0.5))
    a_ref = l5b["k_f"] / l5b["c_fref"]
    assert abs(0.25 * (1 / l5b["zeta"][1] - 0.5) - a_ref) < 1e-15
    am_ref = l5b["k_m"] / (l5b["rho_m"] * l5b["c_mref"])
    assert abs(0.25 * (1 / l5b["eta"][1] - 0.5) - am_ref) < 1e-15


def test_wall_mapping():
    lp = _lp()
    assert lp["wall_type"] == [1, 1, 2, 2] and lp["wall_T"][:2] == [1.0, 0.0]
    lp = _lp(wall_type=(1, 2, 1, 0), wall_T=(-1.0, 5.0, -0.5, 3.0))
    assert lp["wall_type"] == [1, 2, 1, 2] and lp["wall_T"] == [-1.0, 0.0, -0.5, 0.0]
    with pytest.raises(ValueError):
        lattice_params(make_params(nx=8, ny=16, bc_x=1, porosity=0.9, Ra=1.0, Da=0.1, Ste=1.0,
                                   Nu_i=0.0, wall_type=(1, 0, 0, 0)))
    with pytest.raises(ValueError):
        _lp(wall_type=(3, 0, 0, 0))
    assert _lp(L_char=100.0)["L"] == 100.0


def test_bounce_back_solid_node_reflects():
    # Sec. V B alternative: a node below f_l = 0.5 returns every flow
    # population along the opposite link; a liquid node collides as usual.
    lp = _lp(solid_treatment=1, Ra=1e8)
    r = np.random.default_rng(21)
    fplus = oracle.feq(1.0, 0.01, -0.02, lp["phi"]) + 1e-4 * r.standard_normal(9)
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    for i in range(9):
        assert EX[opp[i]] == -EX[i] and EY[opp[i]] == -EY[i]
    Hs = oracle.enthalpy_of_T(lp, -0.5)
    g = oracle.geq(Hs, -0.5, 0.0, 0.0, lp["phi"], lp["c_fref"], lp["c_pl"])
    h = oracle.heq(-0.5, lp["c_pm"], lp["c_mref"])
    m = oracle.node_macros(lp, fplus, g, h)
    assert m["f_l"] == 0.0 and m["ux"] == 0.0 and m["uy"] == 0.0
    fo, _, _, _ = oracle.collide_node(lp, fplus, g, h, 0.0, 0.0)
    np.testing.assert_array_equal(fo, fplus[opp])
    # the same node in the volumetric scheme is the rest equilibrium instead
    fv, _, _, _ = oracle.collide_node(_lp(Ra=1e8), fplus, g, h, 0.0, 0.0)
    np.testing.assert_allclose(fv, W * fplus.sum(), rtol=0, atol=2e-16)
    # a liquid node is unaffected by the switch
    Hl = oracle.enthalpy_of_T(lp, 0.6)
    gl = oracle.geq(Hl, 0.6, 0.0, 0.0, lp["phi"], lp["c_fref"], lp["c_pl"])
    hl = oracle.heq(0.6, lp["c_pm"], lp["c_mref"])
    a, _, _, _ = oracle.collide_node(lp, fplus, gl, hl, 0.0, 0.0)
    b, _, _, _ = oracle.collide_node(_lp(Ra=1e8), fplus, gl, hl, 0.0, 0.0)
    np.testing.assert_array_equal(a, b)
