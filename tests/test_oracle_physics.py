"""Pins of the oracle's full update against closed forms and invariants the
paper's model fixes (no implementation of the paper exists to compare with).

* Brinkman channel: steady porous channel flow, closed form for F_phi = 0
  (Eqs. 2-3), a library BVP solve for F_phi > 0.
* LTNE conduction: Eqs. (5)-(6) without flow and without phase change are
  linear; each sine mode follows a 2x2 ODE solved by a matrix exponential.
* Stefan problem: in the local-thermal-equilibrium limit (Eq. 10) the
  melting front follows Neumann's similarity solution.
* LTE collapse: the PCM/foam temperature difference shrinks as h_v grows.
* Steady conduction: linear profiles, Nusselt number exactly 1.
* Energy and mass balance: the change of the interior totals equals the
  tallied wall link fluxes, because the interstitial sources cancel and the
  collisions keep the zeroth moments.
* Solid at rest: zero velocity wherever f_l = 0 (Sec. V B); the Eq. (53)
  rate choice reduces the solid-side undershoot (Secs. V C, V D), and BGK
  thermal collisions leave a larger one (Sec. V A).
* Solid at the melting temperature (Sec. V C): exact on D2Q5 and on D2Q9
  with every even non-conserved enthalpy moment relaxed at 2 - zeta_alpha;
  not with the printed zeta_v = 1.2 (the undershoot is pinned as measured).
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_bvp
from scipy.linalg import expm
from scipy.optimize import brentq
from scipy.special import erf

import oracle
from lbm_workloads import case_c1, case_p1, initial_temperatures, make_params, scaled_cavity
from oracle.mapping import lattice_params, steps_for_fourier
from paper_groups import groups


# ---------------------------------------------------------------------------
# Brinkman-Forchheimer channel
# ---------------------------------------------------------------------------

def _channel_params(ny, F_phi, target_u):
    p = make_params(nx=4, ny=ny, bc_x=1, gravity_axis=0, porosity=0.9, Ra=1.0, Pr=5.0, Da=0.05,
                    Ste=1.0, k_ratio=1.0, cap_ratio=1.0, Nu_i=0.0, F_phi=F_phi, k_f=0.02,
                    T_hot=1.0, T_cold=0.0, T_init=1.0, T_solidus=-2.0, T_liquidus=-1.0)
    g = groups(p)
    gb = target_u * g["nu_f"] / g["K"]            # Darcy velocity G K / nu_f = target_u
    p["Ra"] = gb * g["L"] ** 3 / (g["nu_f"] * g["alpha_f"])   # Eq. (54), dT = 1
    return p, groups(p)


def _steady_channel(p, g):
    """Advance to steady state: 40 e-folds of the slowest viscous/Darcy mode,
    rate nu_e (pi/H)^2 + phi nu_f / K.  (Non-equilibrium extrapolation does
    not conserve mass, so a sheared wall leaks mass at a rate ~u^2 and the
    velocity never stops changing in the last digits; that drift is far
    below the discretisation error checked here.)"""
    ny = p["ny"]
    H = ny - 1
    rate = g["nu_e"] * (math.pi / H) ** 2 + g["phi"] * g["nu_f"] / g["K"]
    o = oracle.Oracle(p)
    T = np.ones((ny, 4))
    o.set_initial(T, T)
    o.step(int(40.0 / rate))
    return o.fields()["ux"][:, 1].copy()


def _brinkman_closed_form(g, y):
    H = g["L"]    # the channel's walls sit on rows 0 and ny - 1
    r = math.sqrt(g["phi"] * g["nu_f"] / (g["K"] * g["nu_e"]))
    uinf = g["gbeta"] * g["K"] / g["nu_f"]
    return uinf * (1 - np.cosh(r * (y - H / 2)) / np.cosh(r * H / 2))


def test_brinkman_channel_closed_form():
    errs = []
    for ny in (17, 33):
        p, g = _channel_params(ny, 0.0, 1e-3)
        u = _steady_channel(p, g)
        ue = _brinkman_closed_form(g, np.arange(ny, dtype=float))
        errs.append(np.abs(u - ue).max() / np.abs(ue).max())
        assert abs(u[0]) < 1e-3 * ue.max() and abs(u[-1]) < 1e-3 * ue.max()
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 2.8   # second-order convergence


def test_brinkman_forchheimer_channel_bvp():
    errs = []
    for ny in (17, 33):
        p, g = _channel_params(ny, 2.0, 5e-3)
        u = _steady_channel(p, g)
        H = ny - 1
        phi, K, nu, nue, Fp, G = g["phi"], g["K"], g["nu_f"], g["nu_e"], g["F_phi"], g["gbeta"]
        # nu_e u'' - phi nu/K u - phi F/sqrt(K) |u| u + phi G = 0, u(0) = u(H) = 0
        def rhs(y, s):
            return np.vstack([s[1], (phi * nu / K * s[0] + phi * Fp / math.sqrt(K) * np.abs(s[0]) * s[0]
                                     - phi * G) / nue])
        yy = np.linspace(0, H, 801)
        guess = np.vstack([_brinkman_closed_form(g, yy), np.zeros_like(yy)])
        sol = solve_bvp(rhs, lambda a, b: np.array([a[0], b[0]]), yy, guess, tol=1e-10, max_nodes=100000)
        assert sol.success
        ue = sol.sol(np.arange(ny, dtype=float))[0]
        # the inertial term must matter for this check to pin it
        assert np.abs(ue - _brinkman_closed_form(g, np.arange(ny, dtype=float))).max() > 0.05 * ue.max()
        errs.append(np.abs(u - ue).max() / np.abs(ue).max())
    assert errs[1] < 5e-3
    assert errs[0] / errs[1] > 2.8


# ---------------------------------------------------------------------------
# LTNE conduction (no flow, no phase change)
# ---------------------------------------------------------------------------

def _ltne_params(nx, Nu_i, k_f=0.02):
    return make_params(nx=nx, ny=4, porosity=0.9, Ra=0.0, Pr=5.0, Da=1.0, Ste=1.0, k_ratio=10.0,
                       cap_ratio=2.0, Nu_i=Nu_i, k_f=k_f, cf_ref=0.3, cm_ref=0.7,
                       T_hot=1.0, T_cold=0.0, T_init=0.0, T_solidus=-2.0, T_liquidus=-1.0)


def _ltne_exact(g, x, t, kmax=3000):
    """Linear steady profile plus sine modes of the two-temperature system
    (Eqs. 5-6 without flow or phase change), from the problem's groups."""
    L = g["L"]
    af = g["alpha_f"]
    am = g["alpha_m"]
    a = g["h_v"] / g["phi"]                      # h_v / (phi rho_l c_pl)
    b = g["h_v"] / ((1 - g["phi"]) * g["rc_m"])  # h_v / ((1 - phi) rho_m c_pm)
    Tf = 1 - x / L
    Tm = 1 - x / L
    for k in range(1, kmax + 1):
        kap = k * math.pi / L
        A = np.array([[-af * kap ** 2 - a, a], [b, -am * kap ** 2 - b]])
        c = -2 / (k * math.pi)
        v = expm(A * t) @ np.array([c, c])
        s = np.sin(kap * x)
        Tf = Tf + v[0] * s
        Tm = Tm + v[1] * s
    return Tf, Tm


def _ltne_run(nx, Nu_i, Fo):
    p = _ltne_params(nx, Nu_i)
    g = groups(p)
    o = oracle.Oracle(p)
    T0 = np.zeros((4, nx))
    o.set_initial(T0, T0)
    n = int(round(Fo * g["L"] ** 2 / g["alpha_f"]))
    o.step(n)
    f = o.fields()
    x = np.arange(nx, dtype=float)
    Tf, Tm = _ltne_exact(g, x, n)
    assert np.abs(f["T_pcm"][1] - f["T_pcm"][2]).max() < 1e-14   # stays one-dimensional
    return (np.abs(f["T_pcm"][1] - Tf).max(), np.abs(f["T_mf"][1] - Tm).max(),
            np.abs(Tf - Tm).max(), np.abs(f["T_pcm"][1] - f["T_mf"][1]).max())


@pytest.mark.parametrize("Nu_i", [0.0, 0.002])
def test_ltne_conduction_modes(Nu_i):
    e33 = _ltne_run(33, Nu_i, 0.05)
    e65 = _ltne_run(65, Nu_i, 0.05)
    assert e65[2] > 0.1            # strongly non-equilibrium: T_f and T_m differ
    assert e65[0] < 5e-4 and e65[1] < 5e-4
    assert e33[0] / e65[0] > 3.5 and e33[1] / e65[1] > 3.5


def test_lte_collapse_with_interstitial_exchange():
    dts = []
    nus = [0.0125, 0.025, 0.05, 0.1, 0.2, 0.4]
    for nu in nus:
        p = _ltne_params(33, nu)
        assert lattice_params(p)["z"] <= 0.5 + 1e-12
        dts.append(_ltne_run(33, nu, 0.05)[3])
    assert all(b < a for a, b in zip(dts, dts[1:]))
    slope = math.log(dts[-1] / dts[-2]) / math.log(nus[-1] / nus[-2])
    assert -1.3 < slope < -0.7


def test_steady_conduction_nusselt_is_one():
    p = _ltne_params(33, 0.05)
    lp = lattice_params(p)
    o = oracle.Oracle(p)
    T0 = np.zeros((4, 33))
    o.set_initial(T0, T0)
    o.step(int(steps_for_fourier(lp, 2.0)))
    d = o.diagnostics()
    assert abs(d["Nu_hot"] - 1) < 1e-8 and abs(d["Nu_cold"] - 1) < 1e-8
    assert abs(d["Nu_hot_pcm"] - 1) < 1e-8
    f = o.fields()
    np.testing.assert_allclose(f["T_pcm"][1], 1 - np.arange(33) / 32.0, atol=1e-10)


# ---------------------------------------------------------------------------
# Stefan problem in the LTE limit
# ---------------------------------------------------------------------------

def test_stefan_front_neumann():
    nx = 129
    p = make_params(nx=nx, ny=4, porosity=0.9, Ra=0.0, Pr=5.0, Da=1.0, Ste=1.0, k_ratio=10.0,
                    cap_ratio=1.0, Nu_i=8.0, k_f=0.02, T_hot=1.0, T_cold=0.0, T_init=0.0,
                    T_solidus=0.0, T_liquidus=0.002)
    g = groups(p)
    assert 0.5 < g["h_v"] * (1 / g["phi"] + 1 / ((1 - g["phi"]) * g["rc_m"])) < 0.7
    o = oracle.Oracle(p)
    T0 = np.zeros((4, nx))
    o.set_initial(T0, T0)
    n = int(round(0.02 * g["L"] ** 2 / g["alpha_f"]))
    o.step(n)
    fl = o.fields()["f_l"][1]
    s_int = fl[1:-1].sum() + 0.5       # melted length: integral of f_l from the wall
    i = int(np.where(fl < 0.5)[0][0])
    s_half = (i - 1) + (fl[i - 1] - 0.5) / (fl[i - 1] - fl[i])
    # Neumann: s = 2 lam sqrt(alpha_e t), lam e^{lam^2} erf(lam) = St_e / sqrt(pi)
    phi = g["phi"]
    rc = phi + (1 - phi) * g["rc_m"]               # rho c_p-bar of Eq. (10), all liquid
    ke = phi * g["k_f"] + (1 - phi) * g["k_m"]     # k_e of Eq. (10)
    St_e = rc * (p["T_hot"] - p["T_solidus"]) / (phi * g["L_a"])
    lam = brentq(lambda l: l * math.exp(l * l) * erf(l) - St_e / math.sqrt(math.pi), 1e-6, 5)
    s_ex = 2 * lam * math.sqrt(ke / rc * n)
    assert s_ex > 25
    assert abs(s_int - s_ex) < 0.05
    assert abs(s_half - s_ex) < 0.1
    # the diagnostics report the same front and melted fraction
    d = o.diagnostics()
    assert abs(d["x_front_mid"] * g["L"] - s_half) < 1e-12
    assert abs(d["liquid_fraction"] * (nx - 2) - fl[1:-1].sum()) < 1e-9


# ---------------------------------------------------------------------------
# Energy / mass balance on the C1 cavity
# ---------------------------------------------------------------------------

def test_energy_and_mass_balance_c1():
    p, _, seed, _ = case_c1()
    Tf, Tm = initial_temperatures(p, seed)
    o = oracle.Oracle(p)
    o.set_initial(Tf, Tm)
    o.step(1500)
    d = o.diagnostics()
    assert d["E_int"] - d["E_int0"] > 100          # heat did enter
    assert abs(d["energy_residual"]) <= 1e-12 * abs(d["E_int"])
    assert abs(d["mass_residual"]) <= 1e-12 * abs(d["M_int"])
    # the hot wall supplies it; the cold wall and the adiabatic walls carry little
    assert d["flux_E"][0] > 0.99 * (d["E_int"] - d["E_int0"])
    assert d["nonfinite"] == 0


# ---------------------------------------------------------------------------
# Solid at rest and the rate choice of Eq. (53)
# ---------------------------------------------------------------------------

def _p1_small(zeta_e=None):
    p, _, _, _ = case_p1()
    q = scaled_cavity(p, 41)
    q.update(Nu_i=0.0, T_solidus=0.0, T_liquidus=0.002, zeta_e=zeta_e or 0.0)
    lp = lattice_params(q)
    o = oracle.Oracle(q)
    T0 = np.zeros((41, 41))
    o.set_initial(T0, T0)
    o.step(int(round(steps_for_fourier(lp, 0.002))))
    return o.fields()


def test_solid_at_rest_and_rate_choice_reduces_undershoot():
    f = _p1_small()
    solid = f["f_l"] == 0.0
    assert solid.sum() > 500
    assert np.all(f["ux"][solid] == 0.0) and np.all(f["uy"][solid] == 0.0)
    assert np.hypot(f["ux"], f["uy"]).max() > 1e-5          # the liquid does move
    under = -f["T_pcm"].min()
    for ze in (1.0, 1.8):
        g = _p1_small(ze)
        assert -g["T_pcm"].min() > 2.0 * under


def _two_rate(lp):
    """The rate set with the stress moments of the enthalpy field (p_xx,
    p_xy, moments 7 and 8) relaxed at 2 - zeta_alpha like e and eps, instead
    of the printed zeta_v = 1.2 of Sec. III C: every even non-conserved
    moment then relaxes at 2 - zeta_alpha and every odd one at zeta_alpha,
    so Eq. (53) is the product of the two rates' (1/rate - 1/2).  D2Q5
    (Appendix B) has this structure with its printed rates."""
    za = lp["zeta"][3]
    lp["zeta"][7] = lp["zeta"][8] = 2.0 - za
    return lp


def _min_solid_T(p, modify=None):
    lp = lattice_params(p)
    if modify:
        lp = modify(lp)
    o = oracle.Oracle(p, lattice=lp)
    T0 = np.full((p["ny"], p["nx"]), p["T_init"])
    o.set_initial(T0, T0)
    o.step(int(round(steps_for_fourier(lp, 0.02 if p["ny"] == 4 else 0.002))))
    f = o.fields()
    assert f["f_l"].max() > 0.5 and (f["f_l"] < 1e-9).sum() > 0.2 * f["f_l"].size   # a front and a solid
    return f["T_pcm"].min()


def test_solid_stays_at_the_melting_temperature():
    # Sec. V C (Fig. 13): with T_melt = T_init = T_cold and H_v = 0 the
    # present scheme keeps the solid at T_melt.  It holds exactly (to
    # rounding) on D2Q5 and on D2Q9 when the stress moments of the enthalpy
    # field relax at 2 - zeta_alpha; with the printed zeta_v = 1.2 the D2Q9
    # solid undershoots (1-D Stefan run: -7.7e-4 of dT; 41^2 Sec. V C run:
    # -1.6e-2; 151^2: -8.0e-3, -6.1e-3 on the middle row), so the claim
    # does not hold for the printed rate set.
    stefan = make_params(nx=129, ny=4, porosity=0.9, Ra=0.0, Pr=5.0, Da=1.0, Ste=1.0, k_ratio=10.0,
                         cap_ratio=1.0, Nu_i=0.0, k_f=0.02, T_hot=1.0, T_cold=0.0, T_init=0.0,
                         T_solidus=0.0, T_liquidus=0.002)
    q, _, _, _ = case_p1()
    cavity = scaled_cavity(q, 41)
    cavity.update(Nu_i=0.0, T_solidus=0.0, T_liquidus=0.002)
    for p in (stefan, cavity):
        T_fs = p["T_solidus"]
        assert _min_solid_T(p, _two_rate) >= T_fs - 1e-12
        # the library's option for this rate set (pcm_even_rates) maps to it
        even = lattice_params(dict(p, pcm_even_rates=1))
        assert even["zeta"] == _two_rate(lattice_params(p))["zeta"]
        assert _min_solid_T(dict(p, pcm_even_rates=1)) >= T_fs - 1e-12
        assert _min_solid_T(dict(p, thermal_lattice=5)) >= T_fs - 1e-12
        assert _min_solid_T(p) < T_fs - 5e-4          # the printed zeta_v = 1.2


def test_bgk_thermal_collisions_spoil_the_interface():
    # Sec. V A: single-relaxation-time thermal collisions smear the phase
    # interface that the MRT rates of Eq. (53) keep sharp.  On the same run
    # the BGK switch (every thermal rate 1/tau) leaves a solid-side
    # undershoot several times the MRT one; on D2Q5 the MRT run has none.
    def undershoot(**kw):
        p, _, _, _ = case_p1()
        q = scaled_cavity(p, 41)
        q.update(Nu_i=0.0, T_solidus=0.0, T_liquidus=0.002, **kw)
        lp = lattice_params(q)
        o = oracle.Oracle(q)
        T0 = np.zeros((41, 41))
        o.set_initial(T0, T0)
        o.step(int(round(steps_for_fourier(lp, 0.002))))
        return -o.fields()["T_pcm"].min()
    mrt, bgk = undershoot(), undershoot(thermal_collision=1)
    assert bgk > 2.5 * mrt > 0
    mrt5, bgk5 = undershoot(thermal_lattice=5), undershoot(thermal_lattice=5, thermal_collision=1)
    assert mrt5 < 1e-3 and bgk5 > 0.02


def test_zeta_e_sweep_of_sec_VD_runs():
    # Sec. V D runs the Sec. IV B problem at zeta_e = 1.8, 1.2, 0.6, 0.1 and
    # 2 - zeta_alpha = 0.0296 to Fo = 0.002: every run stays finite and the
    # melted fraction barely moves (the rate shapes the interface only).
    p, _, _, _ = case_p1()
    q0 = scaled_cavity(p, 41)
    fls = []
    for ze in (1.8, 1.2, 0.6, 0.1, 0.0):
        q = dict(q0, zeta_e=ze)
        lp = lattice_params(q)
        assert lp["zeta"][1] == lp["zeta"][2] == (ze if ze > 0 else 2 - lp["zeta"][3])
        o = oracle.Oracle(q)
        T0 = np.zeros((41, 41))
        o.set_initial(T0, T0)
        o.step(int(round(steps_for_fourier(lp, 0.002))))
        d = o.diagnostics()
        assert d["nonfinite"] == 0
        fls.append(d["liquid_fraction"])
    assert max(fls) - min(fls) < 0.01 * fls[-1]
