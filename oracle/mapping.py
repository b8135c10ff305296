"""Oracle-side mapping from the dimensionless problem to lattice units.

Test infrastructure only (see the package docstring).  Written from the
paper's definitions:

* lattice units dx = dt = c = 1, c_s^2 = 1/3 (Sec. IV parameter list);
* dimensionless groups Ra, Pr, Da, J, lambda, sigma, H_v, Fo, St (Eq. 54);
* rho_l = rho_s = 1, c_pl = c_ps = c_pm = 1, so the capacity ratio sigma
  equals rho_m (Sec. IV parameter list);
* viscosity <-> rate (Eq. 26 and the rate rule of Sec. III C);
* thermal diffusivities <-> rates (Eq. A19 and the metal analogue after
  Eq. 51), free rates of Sec. III C, Eq. (53) for zeta_e;
* Forchheimer coefficient from the porosity, Eq. (4), unless given;
* characteristic length L = nx - 1 (walls on the first and last node
  columns; for the periodic-in-x channel, the distance between the two
  horizontal walls, ny - 1) unless given, reference temperature
  T_0 = T_cold (Sec. IV B);
* thermal lattice D2Q9 (Sec. III B/C) or D2Q5 (Appendix B, c_sT^2 = varpi/2,
  zeta_e = 2 - zeta_alpha), MRT or BGK thermal collisions (Sec. V A), an
  optional fixed zeta_e (Sec. V D);
* walls: isothermal or adiabatic, each of the four; by default the cavity
  of Sec. IV B (hot left, cold right, adiabatic top and bottom);
* solid phase: the volumetric scheme of Eq. (20), or the bounce-back
  alternative of Sec. V B.
"""
from __future__ import annotations

import math


WALL_DEFAULT, WALL_ISOTHERMAL, WALL_ADIABATIC = 0, 1, 2


def char_length(p: dict) -> float:
    """Distance between the two walls that carry the imposed temperature
    difference (cavity) or the no-slip condition (periodic channel), unless
    the problem gives its own length."""
    if p.get("L_char", 0.0) > 0:
        return float(p["L_char"])
    return float(p["ny"] - 1) if int(p["bc_x"]) == 1 else float(p["nx"] - 1)


def thermal_lattice(p: dict):
    """(number of thermal velocities, varpi, c_sT^2)."""
    qt = int(p.get("thermal_lattice", 0)) or 9
    if qt not in (5, 9):
        raise ValueError("thermal_lattice must be 9 or 5")
    if qt == 9:
        return 9, 0.0, 1.0 / 3.0
    varpi = float(p.get("varpi", 0.0))
    if varpi <= 0:
        varpi = 2.0 / 3.0
    if not varpi < 1.0:
        raise ValueError("varpi must lie in (0, 1) (Eq. B2)")
    return 5, varpi, varpi / 2.0


def walls(p: dict):
    """Resolved (types, temperatures) of the left, right, bottom and top walls."""
    types = [int(t) for t in p.get("wall_type", (0, 0, 0, 0))]
    temps = [float(t) for t in p.get("wall_T", (0.0, 0.0, 0.0, 0.0))]
    if len(types) != 4 or len(temps) != 4 or any(t not in (0, 1, 2) for t in types):
        raise ValueError("wall_type needs four entries among 0 (default), 1 (isothermal), 2 (adiabatic)")
    if int(p["bc_x"]) == 1 and (types[0] or types[1]):
        raise ValueError("a periodic-in-x problem has no left or right wall")
    default = [(WALL_ISOTHERMAL, float(p["T_hot"])), (WALL_ISOTHERMAL, float(p["T_cold"])),
               (WALL_ADIABATIC, 0.0), (WALL_ADIABATIC, 0.0)]
    if int(p["bc_x"]) == 1:
        default[0] = default[1] = (WALL_ADIABATIC, 0.0)
    out_t, out_T = [], []
    for w in range(4):
        if types[w] == WALL_DEFAULT:
            t, T = default[w]
        else:
            t, T = types[w], (temps[w] if types[w] == WALL_ISOTHERMAL else 0.0)
        out_t.append(t)
        out_T.append(T)
    return out_t, out_T


def stable_k_f(p: dict) -> float:
    """Largest lattice PCM diffusivity keeping every thermal/viscous
    relaxation time at or below 2 and the interstitial-exchange number
    z = h_v dt (1/(phi rho_l c_pl) + 1/((1-phi) rho_m c_pm)) at or below 0.5.
    """
    phi = p["porosity"]
    J = p["J"] if p["J"] > 0 else 1.0
    c_fref = p["cf_ref"] if p["cf_ref"] > 0 else 0.2
    c_mref = p["cm_ref"] if p["cm_ref"] > 0 else 1.0
    rho_m = p["cap_ratio"]
    lam = p["k_ratio"]
    L = char_length(p)
    dpL = p["dp_over_L"] if p["dp_over_L"] > 0 else 0.0135
    d_p = dpL * L
    _, _, cs2T = thermal_lattice(p)
    # tau = 0.5 + alpha_ref / c_s^2 <= 2  <=>  alpha_ref <= 1.5 c_s^2
    limits = [0.5 / (J * p["Pr"]), 1.5 * cs2T * c_fref]
    if lam > 0:
        limits.append(1.5 * cs2T * rho_m * c_mref / lam)
    if p["Nu_i"] > 0:
        limits.append(0.5 * d_p * d_p / (p["Nu_i"] * (1.0 / phi + 1.0 / ((1.0 - phi) * rho_m))))
    return min(limits)


def lattice_params(p: dict) -> dict:
    """Map a problem description (see lbm_workloads.PARAM_FIELDS) to the
    lattice constants the update uses.  Raises ValueError for parameter sets
    the scheme cannot run."""
    nx, ny = int(p["nx"]), int(p["ny"])
    if nx < 4 or ny < 4:
        raise ValueError("grid must be at least 4 x 4")
    phi = float(p["porosity"])
    if not 0.0 < phi < 1.0:
        raise ValueError("porosity must lie in (0, 1)")
    rho_l = 1.0
    c_pl = c_ps = c_pm = 1.0
    rho_m = float(p["cap_ratio"])
    c_fref = p["cf_ref"] if p["cf_ref"] > 0 else 0.2 * c_pl
    c_mref = p["cm_ref"] if p["cm_ref"] > 0 else 1.0 * c_pm
    # Remark I: c_f,ref < 9/5 c_pf and c_m,ref < 9/5 c_pm.
    if not c_fref < 1.8 * c_pl or not c_mref < 1.8 * c_pm:
        raise ValueError("reference specific heats must stay below 9/5 of c_p (Remark I)")
    J = p["J"] if p["J"] > 0 else 1.0
    L = char_length(p)
    dT = float(p["T_hot"]) - float(p["T_cold"])
    if not dT > 0:
        raise ValueError("T_hot must exceed T_cold")
    k_f = p["k_f"] if p["k_f"] > 0 else stable_k_f(p)
    alpha_f = k_f / (rho_l * c_pl)
    nu_f = p["Pr"] * alpha_f
    nu_e = J * nu_f
    k_m = p["k_ratio"] * k_f
    dpL = p["dp_over_L"] if p["dp_over_L"] > 0 else 0.0135
    d_p = dpL * L
    h_v = p["Nu_i"] * k_f / (d_p * d_p)
    F_phi = p["F_phi"] if p["F_phi"] >= 0 else 1.75 / math.sqrt(150.0 * phi ** 3)
    K = p["Da"] * L * L
    if not K > 0:
        raise ValueError("Da must be positive")
    gbeta = p["Ra"] * nu_f * alpha_f / (dT * L ** 3)
    if not p["Ste"] > 0:
        raise ValueError("Ste must be positive")
    L_a = c_pl * dT / p["Ste"]
    T_fs, T_fl = float(p["T_solidus"]), float(p["T_liquidus"])
    if not T_fl > T_fs:
        raise ValueError("liquidus must lie above solidus")

    qt, varpi, cs2T = thermal_lattice(p)
    wall_type, wall_T = walls(p)
    collision = int(p.get("thermal_collision", 0))
    if collision not in (0, 1):
        raise ValueError("thermal_collision must be 0 (MRT) or 1 (BGK)")
    zeta_e_given = float(p.get("zeta_e", 0.0))
    even_rates = int(p.get("pcm_even_rates", 0))
    if even_rates not in (0, 1):
        raise ValueError("pcm_even_rates must be 0 or 1")
    if even_rates and (collision == 1 or qt == 5):
        raise ValueError("pcm_even_rates applies to D2Q9 MRT thermal fields only")
    solid_treatment = int(p.get("solid_treatment", 0))
    if solid_treatment not in (0, 1):
        raise ValueError("solid_treatment must be 0 (volumetric, Eq. 20) or 1 (bounce-back, Sec. V B)")

    # Eq. (26) / Sec. III C: s_v^-1 = 0.5 + nu_e / c_s^2.
    s_v = 1.0 / (0.5 + 3.0 * nu_e)
    # Eq. (A19): alpha_f,ref = k_f/(rho_l c_f,ref) = c_s^2 (1/zeta_alpha - 1/2),
    # with the thermal lattice's sound speed (c_sT^2 = varpi/2 for D2Q5).
    alpha_fref = k_f / (rho_l * c_fref)
    zeta_a = 1.0 / (0.5 + alpha_fref / cs2T)
    # After Eq. (51): alpha_m,ref = k_m/(rho_m c_m,ref) = c_s^2 (1/eta_alpha - 1/2).
    alpha_mref = k_m / (rho_m * c_mref)
    eta_a = 1.0 / (0.5 + alpha_mref / cs2T)
    # Sec. III C free rates; zeta_e = zeta_eps = 2 - zeta_alpha (Eq. 53) unless
    # zeta_e is given (Sec. V D), which then sets the pair zeta_e = zeta_eps
    # as Sec. III C does (moving zeta_e alone is unstable with flow even at
    # the Sec. IV B parameters, where Sec. V D reports runs up to 1.8); the
    # conserved-moment rates zeta_0 and s_rho multiply zero and are 1.  D2Q5 (Appendix B): Theta = diag(zeta_0,
    # zeta_a, zeta_a, zeta_e, zeta_eps), Q = diag(eta_0, eta_a, eta_a, eta_e,
    # eta_eps), the free rates as for D2Q9; entries 5..8 unused (1).  BGK
    # (Sec. V A): every thermal rate 1/tau_g or 1/tau_h.
    s = [1.0, 1.1, 1.1, 1.0, 1.2, 1.0, 1.2, s_v, s_v]
    if collision == 1:
        if zeta_e_given > 0:
            raise ValueError("zeta_e cannot be set for BGK thermal collisions")
        zeta = [zeta_a] * qt + [1.0] * (9 - qt)
        eta = [eta_a] * qt + [1.0] * (9 - qt)
    else:
        ze = zeta_e_given if zeta_e_given > 0 else 2.0 - zeta_a
        if qt == 9:
            # zeta_v = 1.2 (Sec. III C) for the stress moments, or on request
            # the rate of e and eps, which puts every even non-conserved
            # moment at one rate and every odd one at zeta_alpha
            zv = ze if even_rates else 1.2
            zeta = [1.0, ze, ze, zeta_a, zeta_a, zeta_a, zeta_a, zv, zv]
            eta = [1.0, 1.1, 1.1, eta_a, eta_a, eta_a, eta_a, 1.2, 1.2]
        else:
            zeta = [1.0, zeta_a, zeta_a, ze, ze, 1.0, 1.0, 1.0, 1.0]
            eta = [1.0, eta_a, eta_a, 1.1, 1.1, 1.0, 1.0, 1.0, 1.0]
    for name, r in (("s", s), ("zeta", zeta), ("eta", eta)):
        if not all(0.0 < v < 2.0 for v in r):
            raise ValueError(f"relaxation rates {name} must lie in (0, 2): {r}")
    z = h_v * (1.0 / (phi * rho_l * c_pl) + 1.0 / ((1.0 - phi) * rho_m * c_pm))
    if not z < 1.0:
        raise ValueError(f"interstitial exchange number z = {z} >= 1 (explicit source unstable)")
    return dict(
        nx=nx, ny=ny, periodic_x=int(p["bc_x"]), gravity_axis=int(p["gravity_axis"]),
        phi=phi, rho_l=rho_l, rho_m=rho_m, c_pl=c_pl, c_ps=c_ps, c_pm=c_pm,
        c_fref=c_fref, c_mref=c_mref, nu_f=nu_f, nu_e=nu_e, K=K, F_phi=F_phi, gbeta=gbeta,
        T0=float(p["T_cold"]), h_v=h_v, L_a=L_a, T_fs=T_fs, T_fl=T_fl,
        H_fs=c_ps * T_fs, H_fl=c_pl * T_fl + L_a,
        T_hot=float(p["T_hot"]), T_cold=float(p["T_cold"]),
        k_f=k_f, k_m=k_m, L=L, alpha_f=alpha_f, d_p=d_p, z=z,
        tau_v=1.0 / s_v, tau_g=1.0 / zeta_a, tau_h=1.0 / eta_a,
        s=s, zeta=zeta, eta=eta, qt=qt, varpi=varpi, cs2T=cs2T,
        wall_type=wall_type, wall_T=wall_T, thermal_collision=collision,
        solid_treatment=solid_treatment,
    )


def steps_for_fourier(lp: dict, Fo: float) -> float:
    """t = Fo L^2 / alpha_f (Eq. 54)."""
    return Fo * lp["L"] ** 2 / lp["alpha_f"]
