"""Lattice quantities of a test problem, written out in the tests from the
paper's definitions, for the expectations of the oracle's physics pins.

The oracle maps a problem description to lattice units on its own
(oracle/mapping.py).  A pin whose expected value came from that mapping
would hide a slip in it (K = Da L instead of Da L^2 would cancel out), so
the pins compute their expectations from the problem's dimensionless
groups here instead:

* Eq. (54): Ra = g beta dT L^3 / (nu_f alpha_f), Pr = nu_f / alpha_f,
  Da = K / L^2, J = nu_e / nu_f, lambda = k_m / k_f,
  sigma = (rho c_p)_m / (rho c_p)_f, H_v = h_v d_p^2 / k_f,
  Fo = t alpha_f / L^2, St = c_pl dT / L_a;
* Sec. IV parameter list: rho_0 = 1, c_pl = c_ps = c_pf = c_pm = 1,
  d_p / L = 0.0135, dx = dt = 1;
* Eq. (4) for the Forchheimer coefficient when the problem gives none;
* the characteristic length is the distance between the two walls that
  carry the imposed temperature difference (nx - 1), or between the no-slip
  walls of the periodic channel (ny - 1), unless the problem gives its own.

Every test problem passes its lattice diffusivity k_f explicitly, so no
stability rule enters.
"""
from __future__ import annotations

import math

DP_OVER_L = 0.0135   # Sec. IV parameter list


def groups(p: dict) -> dict:
    if not p["k_f"] > 0:
        raise ValueError("pins pass their lattice k_f explicitly")
    if p.get("L_char", 0.0) > 0:
        L = float(p["L_char"])
    else:
        L = float(p["ny"] - 1) if int(p["bc_x"]) == 1 else float(p["nx"] - 1)
    phi = float(p["porosity"])
    k_f = float(p["k_f"])
    alpha_f = k_f                       # k_f / (rho_l c_pl), rho_l = c_pl = 1
    nu_f = p["Pr"] * alpha_f            # Pr = nu_f / alpha_f
    J = p["J"] if p["J"] > 0 else 1.0
    nu_e = J * nu_f                     # J = nu_e / nu_f
    K = p["Da"] * L * L                 # Da = K / L^2
    dT = float(p["T_hot"]) - float(p["T_cold"])
    gbeta = p["Ra"] * nu_f * alpha_f / (dT * L ** 3)   # Ra
    rc_m = float(p["cap_ratio"])        # (rho c_p)_m with (rho c_p)_f = 1
    k_m = p["k_ratio"] * k_f            # lambda = k_m / k_f
    dpL = p["dp_over_L"] if p["dp_over_L"] > 0 else DP_OVER_L
    d_p = dpL * L
    h_v = p["Nu_i"] * k_f / (d_p * d_p)  # H_v = h_v d_p^2 / k_f
    F_phi = p["F_phi"] if p["F_phi"] >= 0 else 1.75 / math.sqrt(150.0 * phi ** 3)  # Eq. (4)
    L_a = dT / p["Ste"]                 # St = c_pl dT / L_a
    return dict(L=L, phi=phi, k_f=k_f, alpha_f=alpha_f, nu_f=nu_f, nu_e=nu_e, K=K, gbeta=gbeta,
                dT=dT, rc_m=rc_m, k_m=k_m, alpha_m=k_m / rc_m, d_p=d_p, h_v=h_v, F_phi=F_phi,
                L_a=L_a)
