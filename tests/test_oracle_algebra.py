"""Pins of the oracle's per-node algebra against what the paper fixes.

Each check compares two independent statements of the paper (a velocity
form against its moment form, an explicit root against the implicit
equation it solves, a conservation law against the collision) or a printed
number, so that a transcription slip in either place fails.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from lbm_workloads import case_p1, make_params
from oracle.mapping import lattice_params, steps_for_fourier

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))

EX, EY, W, M, MINV = oracle.lattice_tables()


def test_velocities_follow_eq11():
    # Eq. (11): axis links at angles (i-1) pi/2, diagonal links at (2i-9) pi/4, length sqrt(2).
    for i in range(9):
        if i == 0:
            ex, ey = 0.0, 0.0
        elif i <= 4:
            ex, ey = math.cos((i - 1) * math.pi / 2), math.sin((i - 1) * math.pi / 2)
        else:
            a = (2 * i - 9) * math.pi / 4
            ex, ey = math.sqrt(2) * math.cos(a), math.sqrt(2) * math.sin(a)
        assert EX[i] == round(ex) and EY[i] == round(ey)


def test_weights_isotropy():
    # The weights listed after Eq. (27) must give c_s^2 = 1/3 and a fourth-order
    # isotropic tensor, the properties the Chapman-Enskog analysis relies on.
    assert abs(W.sum() - 1.0) < 1e-15
    assert abs((W * EX * EX).sum() - 1.0 / 3.0) < 1e-15
    assert abs((W * EX * EY).sum()) < 1e-15
    assert abs((W * EX ** 4).sum() - 1.0 / 3.0) < 1e-15
    assert abs((W * EX ** 2 * EY ** 2).sum() - 1.0 / 9.0) < 1e-15
    assert abs((W * EX).sum()) < 1e-15 and abs((W * EY).sum()) < 1e-15


def test_transform_rows_are_the_standard_moments():
    # Rows of Eq. (13) as polynomials of the lattice velocities (density,
    # energy, energy square, momentum, energy flux, stress components).
    e2 = EX ** 2 + EY ** 2
    rows = [np.ones(9), -4 + 3 * e2, 4 - 10.5 * e2 + 4.5 * e2 ** 2, EX, (-5 + 3 * e2) * EX,
            EY, (-5 + 3 * e2) * EY, EX ** 2 - EY ** 2, EX * EY]
    np.testing.assert_array_equal(M, np.array(rows))


def test_transform_orthogonal_and_inverse():
    G = M @ M.T
    np.testing.assert_allclose(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.abs(G - np.diag(np.diag(G))).max() == 0
    np.testing.assert_allclose(MINV @ M, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(MINV, M.T / np.diag(G), atol=1e-15)


def test_source_direction_maps_to_weights():
    # M^-1 (1,-2,1,0,...) = w: the interstitial sources (Eqs. 35, 46) add
    # w_i S in velocity space, i.e. a density change only.
    np.testing.assert_allclose(MINV @ np.array([1, -2, 1, 0, 0, 0, 0, 0, 0.0]), W, atol=1e-16)


@pytest.mark.parametrize("seed", range(5))
def test_flow_equilibrium_moments(seed):
    # Eq. (27) (velocity space) against Eq. (18) (moment space, alpha1=1, alpha2=-3).
    r = np.random.default_rng(seed)
    rho, ux, uy, phi = 1 + 0.1 * r.standard_normal(), 0.05 * r.standard_normal(), \
        0.05 * r.standard_normal(), r.uniform(0.3, 0.99)
    m = M @ oracle.feq(rho, ux, uy, phi)
    uu = ux * ux + uy * uy
    meq = rho * np.array([1, -2 + 3 * uu / phi, 1 - 3 * uu / phi, ux, -ux, uy, -uy,
                          (ux * ux - uy * uy) / phi, ux * uy / phi])
    np.testing.assert_allclose(m, meq, atol=2e-16)


@pytest.mark.parametrize("seed", range(5))
def test_enthalpy_equilibrium_moments(seed):
    # Eq. (40) against Eq. (34).
    r = np.random.default_rng(100 + seed)
    H, T, ux, uy = r.uniform(0, 2), r.uniform(-1, 1), 0.05 * r.standard_normal(), 0.05 * r.standard_normal()
    phi, cf, cpl = r.uniform(0.3, 0.99), r.uniform(0.05, 1.7), 1.0
    n = M @ oracle.geq(H, T, ux, uy, phi, cf, cpl)
    neq = np.array([H, -4 * H + 2 * cf * T, 4 * H - 3 * cf * T, cpl * T * ux / phi,
                    -cpl * T * ux / phi, cpl * T * uy / phi, -cpl * T * uy / phi, 0, 0])
    np.testing.assert_allclose(n, neq, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_metal_equilibrium_moments(seed):
    # Eq. (49) against Eq. (45).
    r = np.random.default_rng(200 + seed)
    Tm, cpm, cm = r.uniform(-1, 2), 1.0, r.uniform(0.05, 1.7)
    n = M @ oracle.heq(Tm, cpm, cm)
    neq = np.array([cpm * Tm, -4 * cpm * Tm + 2 * cm * Tm, 4 * cpm * Tm - 3 * cm * Tm, 0, 0, 0, 0, 0, 0])
    np.testing.assert_allclose(n, neq, atol=1e-15)


def _c1_lattice(**over):
    p = make_params(nx=64, ny=64, porosity=0.9, Ra=1e4, Da=1e-4, Ste=1.0, Nu_i=5.0)
    p.update(over)
    return lattice_params(p)


def _random_node(r, lp, T=None, liquid=True):
    rho = 1 + 1e-3 * r.standard_normal()
    u = 0.02 * r.standard_normal(2)
    fplus = oracle.feq(rho, u[0], u[1], lp["phi"]) + 1e-4 * r.standard_normal(9)
    if T is None:
        T = r.uniform(0.05, 1.0) if liquid else -0.5
    H = oracle.enthalpy_of_T(lp, T)
    g = oracle.geq(H, T, u[0], u[1], lp["phi"], lp["c_fref"], lp["c_pl"]) + 1e-5 * r.standard_normal(9)
    Tm = T + 0.01 * r.standard_normal()
    h = oracle.heq(Tm, lp["c_pm"], lp["c_mref"]) + 1e-5 * r.standard_normal(9)
    return fplus, g, h


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("F_phi", [0.0, -1.0])
def test_explicit_velocity_solves_implicit_eq22(seed, F_phi):
    # Eq. (23) is the explicit root of Eq. (22): rho u = sum e_i f_i + rho F(u)/2
    # with F from Eq. (3); large G makes the nonlinear term matter.
    lp = _c1_lattice(F_phi=F_phi, Ra=1e9)
    r = np.random.default_rng(seed)
    fplus, g, h = _random_node(r, lp)
    m = oracle.node_macros(lp, fplus, g, h)
    assert m["f_l"] == 1.0
    fb = fplus  # liquid node: the blend of Eq. (20) is the identity
    rho, ux, uy = m["rho"], m["ux"], m["uy"]
    umag = math.hypot(ux, uy)
    phi, K = lp["phi"], lp["K"]
    Fx = -phi * lp["nu_f"] / K * ux - phi * lp["F_phi"] / math.sqrt(K) * umag * ux + phi * m["Gx"]
    Fy = -phi * lp["nu_f"] / K * uy - phi * lp["F_phi"] / math.sqrt(K) * umag * uy + phi * m["Gy"]
    rx = rho * ux - ((EX * fb).sum() + 0.5 * rho * Fx)
    ry = rho * uy - ((EY * fb).sum() + 0.5 * rho * Fy)
    assert abs(rx) < 1e-15 and abs(ry) < 1e-15
    assert abs(m["Gy"]) > 0 and m["Gx"] == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_collision_conservation_and_impulse(seed):
    # Mass is conserved, momentum changes by the impulse rho F dt (Guo forcing
    # with s_j = 1), enthalpy and metal energy change by exactly the sources.
    lp = _c1_lattice(Ra=1e8)
    r = np.random.default_rng(50 + seed)
    fplus, g, h = _random_node(r, lp)
    srf_prev, srm_prev = 1e-3 * r.standard_normal(), 1e-3 * r.standard_normal()
    fo, go, ho, sr = oracle.collide_node(lp, fplus, g, h, srf_prev, srm_prev)
    m = oracle.node_macros(lp, fplus, g, h)
    rho, ux, uy = m["rho"], m["ux"], m["uy"]
    phi, K = lp["phi"], lp["K"]
    umag = math.hypot(ux, uy)
    Fx = -phi * lp["nu_f"] / K * ux - phi * lp["F_phi"] / math.sqrt(K) * umag * ux + phi * m["Gx"]
    Fy = -phi * lp["nu_f"] / K * uy - phi * lp["F_phi"] / math.sqrt(K) * umag * uy + phi * m["Gy"]
    assert abs(fo.sum() - fplus.sum()) < 1e-14
    assert abs((EX * fo).sum() - (EX * fplus).sum() - rho * Fx) < 1e-15
    assert abs((EY * fo).sum() - (EY * fplus).sum() - rho * Fy) < 1e-15
    # interstitial sources of Eqs. (36), (47)
    srf = lp["h_v"] * (m["T_m"] - m["T_f"]) / (phi * lp["rho_l"])
    srm = lp["h_v"] * (m["T_f"] - m["T_m"]) / ((1 - phi) * lp["rho_m"])
    assert abs(sr[0] - srf) < 1e-17 and abs(sr[1] - srm) < 1e-17
    S_pcm = srf + 0.5 * (srf - srf_prev)
    S_met = srm + 0.5 * (srm - srm_prev)
    assert abs(go.sum() - (m["H"] + S_pcm)) < 1e-14
    assert abs(ho.sum() - (lp["c_pm"] * m["T_m"] + S_met)) < 1e-14
    # the sources exchange energy only: phi rho_l Sr_f + (1-phi) rho_m Sr_m = 0
    assert abs(phi * lp["rho_l"] * srf + (1 - phi) * lp["rho_m"] * srm) < 1e-17


def test_thermal_flux_relaxes_toward_advective_flux():
    # The first moments of g relax at zeta_alpha toward c_pl T u / phi (Eq. 34),
    # which is what yields the diffusivity of Eq. (A19).
    lp = _c1_lattice()
    r = np.random.default_rng(7)
    fplus, g, h = _random_node(r, lp)
    fo, go, ho, _ = oracle.collide_node(lp, fplus, g, h, 0.0, 0.0)
    m = oracle.node_macros(lp, fplus, g, h)
    za = lp["zeta"][3]
    jx = (EX * g).sum()
    target = lp["c_pl"] * m["T_f"] * m["ux"] / lp["phi"]
    assert abs((EX * go).sum() - (jx - za * (jx - target))) < 1e-15
    # metal field: no advection, flux relaxes toward zero at eta_alpha
    ea = lp["eta"][3]
    assert abs((EX * ho).sum() - (1 - ea) * (EX * h).sum()) < 1e-15


def test_solid_node_is_at_rest():
    # Sec. V B: in the solid (f_l = 0) the velocity is zero at every node; the
    # volumetric scheme (Eq. 20) makes the flow populations the rest
    # equilibrium w_i rho.
    lp = _c1_lattice(Ra=1e8)
    r = np.random.default_rng(3)
    fplus, g, h = _random_node(r, lp, liquid=False)
    m = oracle.node_macros(lp, fplus, g, h)
    assert m["f_l"] == 0.0 and m["ux"] == 0.0 and m["uy"] == 0.0
    fo, _, _, _ = oracle.collide_node(lp, fplus, g, h, 0.0, 0.0)
    np.testing.assert_allclose(fo, W * fplus.sum(), rtol=0, atol=2e-16)


def test_eos_continuity_and_inverse():
    # Eqs. (38)-(39): T and f_l are continuous at H_fs and H_fl; the inverse
    # enthalpy map round-trips in all three branches.
    lp = _c1_lattice(T_solidus=0.299, T_liquidus=0.301, Ste=0.7)
    for Hb in (lp["H_fs"], lp["H_fl"]):
        for d in (1e-12, -1e-12):
            T1, f1 = oracle.eos(lp, Hb + d)
            T0, f0 = oracle.eos(lp, Hb)
            assert abs(T1 - T0) < 1e-11 and abs(f1 - f0) < 1e-10
    assert oracle.eos(lp, lp["H_fs"]) == (lp["T_fs"], 0.0)
    assert oracle.eos(lp, lp["H_fl"]) == (lp["T_fl"], 1.0)
    for T in np.linspace(-1, 2, 61):
        H = oracle.enthalpy_of_T(lp, T)
        T2, fl = oracle.eos(lp, H)
        assert abs(T2 - T) < 1e-14
    # latent heat: the enthalpy jump across the band is L_a plus the sensible part
    Hs, Hl = oracle.enthalpy_of_T(lp, 0.299), oracle.enthalpy_of_T(lp, 0.301)
    assert abs((Hl - Hs) - (lp["L_a"] + 0.002)) < 1e-14
    # the liquid fraction is monotone in H
    Hs_ = np.linspace(lp["H_fs"] - 0.1, lp["H_fl"] + 0.1, 401)
    fls = [oracle.eos(lp, H)[1] for H in Hs_]
    assert np.all(np.diff(fls) >= 0)


def test_paper_zeta_e_and_table1_steps():
    # Sec. V D prints zeta_e = 0.0296 for the Sec. IV B parameters; Table I
    # prints the step counts to Fo = 0.002 on the 150^2 and 300^2 grids.
    g = GOLD["zeta_e_sec_IVB"]
    p, _, _, _ = case_p1()
    lp = lattice_params(p)
    assert round(lp["zeta"][1], g["digits"]) == g["value"]
    assert lp["zeta"][1] == lp["zeta"][2]
    # Eq. (53): (1/zeta_e - 1/2)(1/zeta_alpha - 1/2) = 1/4
    assert abs((1 / lp["zeta"][1] - 0.5) * (1 / lp["zeta"][3] - 0.5) - 0.25) < 1e-12
    for row in GOLD["table_I_steps"]["rows"]:
        q = dict(p, nx=row["grid"] + 1, ny=row["grid"] + 1)
        lq = lattice_params(q)
        assert round(steps_for_fourier(lq, GOLD["table_I_steps"]["parameters"]["Fo"])) == row["steps"]


def test_mapping_rejects_unstable_sets():
    base = dict(nx=64, ny=64, porosity=0.9, Ra=1e4, Da=1e-4, Ste=1.0, Nu_i=5.0)
    with pytest.raises(ValueError):
        lattice_params(make_params(**dict(base, porosity=1.0)))
    with pytest.raises(ValueError):  # Remark I bound
        lattice_params(make_params(**dict(base, cf_ref=1.9)))
    with pytest.raises(ValueError):  # explicit interstitial source unstable
        lattice_params(make_params(**dict(base, k_f=5e-3, Nu_i=50.0)))
    with pytest.raises(ValueError):  # tau_h <= 0.5 impossible; tau too large -> rate ok; k_f huge
        lattice_params(make_params(**dict(base, k_f=-1.0, Ste=0.0)))
    with pytest.raises(ValueError):
        lattice_params(make_params(**dict(base, nx=3)))
