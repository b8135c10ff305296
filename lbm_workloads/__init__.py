"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only describes problems: grid sizes, dimensionless groups,
boundary temperatures and seeded random perturbations of the initial PCM
temperature.  It holds none of the method's arithmetic (no parameter
mapping, no equilibria, no update); both the GPU library and the CPU
oracle consume the plain dictionaries returned here and do their own
mapping.

Cases follow the square-cavity melting problem of the paper (Sec. IV B:
hot left wall, cold right wall, adiabatic horizontal walls, PCM initially
solid) with the grid sizes and groups of the benchmark configurations, the
paper's own Ra = 1e6 run (Sec. IV B parameter list), and the batched set of
256 uneven cavities.
"""
from __future__ import annotations

import math

import numpy as np

# Field order of the C parameter struct (include/lbmpcm.h, struct lbm_params).
PARAM_FIELDS = (
    "nx", "ny", "bc_x", "gravity_axis",
    "porosity", "Ra", "Pr", "Da", "Ste", "k_ratio", "cap_ratio", "Nu_i",
    "F_phi", "dp_over_L", "k_f", "cf_ref", "cm_ref", "J",
    "T_hot", "T_cold", "T_init", "T_solidus", "T_liquidus",
    "thermal_lattice", "thermal_collision", "varpi", "zeta_e", "wall_type", "wall_T", "L_char",
    "solid_treatment", "band_rows", "pcm_even_rates",
)

_DEFAULTS = dict(
    bc_x=0, gravity_axis=1,
    Pr=50.0, k_ratio=100.0, cap_ratio=1.0,
    F_phi=-1.0,        # negative: Ergun/Vafai correlation, Eq. (4)
    dp_over_L=0.0,     # <= 0: pore size d_p / L = 0.0135 (Sec. IV parameter list)
    k_f=0.0,           # <= 0: largest stable lattice diffusivity (stability rule)
    cf_ref=0.0, cm_ref=0.0, J=0.0,   # <= 0: 0.2 c_pl, 1.0 c_pm, 1.0
    T_hot=1.0, T_cold=0.0, T_init=0.0,
    # Mushy band: solidus at the cold/initial temperature, liquidus 0.002 above,
    # so the initial state T = 0 sits exactly at the solidus (solid).
    T_solidus=0.0, T_liquidus=0.002,
    thermal_lattice=9,      # 9: D2Q9 thermal fields; 5: D2Q5 (Appendix B)
    thermal_collision=0,    # 0: MRT; 1: BGK thermal collisions (Sec. V A)
    varpi=0.0,              # <= 0: 2/3 (D2Q5 only)
    zeta_e=0.0,             # <= 0: zeta_e = 2 - zeta_alpha (Eq. 53)
    wall_type=(0, 0, 0, 0),  # left, right, bottom, top; 0: the cavity's own
                             # (hot left, cold right, adiabatic top/bottom),
                             # 1: isothermal at wall_T, 2: adiabatic
    wall_T=(0.0, 0.0, 0.0, 0.0),
    L_char=0.0,             # <= 0: nx - 1 (periodic channel: ny - 1)
    solid_treatment=0,      # 0: volumetric scheme (Eq. 20); 1: bounce-back (Sec. V B)
    band_rows=0,            # storage only (GPU library): rows per state band, 0 automatic
    pcm_even_rates=0,       # 0: enthalpy stress moments at zeta_v = 1.2 (Sec. III C);
                            # 1: at the rate of e and eps (D2Q9 MRT only)
)


def make_params(**kw) -> dict:
    """Complete a parameter dictionary with the documented defaults."""
    p = dict(_DEFAULTS)
    p.update(kw)
    missing = [k for k in PARAM_FIELDS if k not in p]
    if missing:
        raise KeyError(f"missing parameters: {missing}")
    unknown = [k for k in p if k not in PARAM_FIELDS]
    if unknown:
        raise KeyError(f"unknown parameters: {unknown}")
    p["nx"] = int(p["nx"])
    p["ny"] = int(p["ny"])
    return p


# --------------------------------------------------------------------------
# Named cases.  Each returns (params, steps, seed, storage) where storage is
# the precision the case is quoted in.
# --------------------------------------------------------------------------

def case_c1():
    """64 x 64 cavity, FP64, 20 000 steps (the small oracle-sized case)."""
    p = make_params(nx=64, ny=64, porosity=0.9, Ra=1e4, Pr=50.0, Da=1e-4,
                    Ste=1.0, k_ratio=100.0, cap_ratio=1.0, Nu_i=5.0)
    return p, 20000, 0, "f64"


def case_c2(n=1024):
    """1024 x 1024 cavity, FP32, 200 000 steps; n=256 gives the A/B case."""
    p = make_params(nx=n, ny=n, porosity=0.95, Ra=1e6, Pr=50.0, Da=1e-4,
                    Ste=1.0, k_ratio=100.0, cap_ratio=1.0, Nu_i=10.0)
    steps = 200000 if n == 1024 else int(round(200000 * (n / 1024.0) ** 2))
    return p, steps, 1, "f32"


def case_c3():
    """8192 x 8192 cavity (67.1 M nodes), FP32, bandwidth case."""
    p = make_params(nx=8192, ny=8192, porosity=0.9, Ra=1e7, Pr=50.0, Da=1e-5,
                    Ste=0.5, k_ratio=1000.0, cap_ratio=1.0, Nu_i=5.0)
    return p, 10000, 0, "f32"


def case_c4():
    """4096 x 4096 cavity, FP16/BF16 offset storage, 100 000 steps."""
    p = make_params(nx=4096, ny=4096, porosity=0.9, Ra=1e6, Pr=50.0, Da=1e-4,
                    Ste=1.0, k_ratio=100.0, cap_ratio=1.0, Nu_i=5.0)
    return p, 100000, 0, "f16"


def case_p1():
    """The paper's Sec. IV B run at Ra = 1e6 (151 x 151 nodes, L = 150)."""
    p = make_params(nx=151, ny=151, porosity=0.8, Ra=1e6, Pr=50.0, Da=1e-4,
                    Ste=1.0, k_ratio=1000.0, cap_ratio=1.0, Nu_i=5.9,
                    F_phi=0.068, k_f=5e-4, cf_ref=0.2, cm_ref=1.0, J=1.0,
                    T_hot=1.0, T_cold=0.0, T_init=0.0,
                    T_solidus=0.299, T_liquidus=0.301)
    return p, 90000, 0, "f64"


def case_corner(n=200):
    """Conduction-induced solidification in a corner (Sec. IV A): liquid PCM
    at T_i = 0.3 in an n x n box, the left and bottom walls lowered to
    T_c = -1 (isothermal), the right and top walls adiabatic (far field of
    the semi-infinite domain), no flow (Ra = 0), L = n/2, lambda = 10,
    St = 4, k_f = 0.01, c_f,ref = 0.5 c_pf, band [-0.05, 0.05] around
    T_melt = 0, H_v = 5.9.  Runs to Fo = 0.02 (20 000 steps at n = 200)."""
    L = n / 2.0
    p = make_params(nx=n, ny=n, porosity=0.8, Ra=0.0, Pr=1.0, Da=1.0, Ste=4.0,
                    k_ratio=10.0, cap_ratio=1.0, Nu_i=5.9, F_phi=0.068, k_f=0.01,
                    cf_ref=0.5, cm_ref=1.0, T_hot=0.0, T_cold=-1.0, T_init=0.3,
                    T_solidus=-0.05, T_liquidus=0.05, wall_type=(1, 2, 1, 2),
                    wall_T=(-1.0, 0.0, -1.0, 0.0), L_char=L)
    steps = int(round(0.02 * L * L / 0.01))
    return p, steps, 0, "f64"


def case_c5(n_cavities=256, seed=7):
    """256 independent cavities of uneven size and physics (seed 7).

    Draw order (vectorised, one call per quantity): side length log-uniform
    in [64, 512] rounded to an integer, aspect ratio in {1, 2} (tall
    cavities: ny = aspect * nx), porosity U[0.85, 0.97], Ra log-U[1e4, 1e6],
    Da log-U[1e-5, 1e-3], Ste U[0.2, 2], interstitial Nu U[1, 20].
    """
    rng = np.random.default_rng(seed)
    n = n_cavities
    side = np.rint(np.exp(rng.uniform(math.log(64), math.log(512), n))).astype(int)
    aspect = rng.choice([1, 2], n)
    phi = rng.uniform(0.85, 0.97, n)
    Ra = 10.0 ** rng.uniform(4, 6, n)
    Da = 10.0 ** rng.uniform(-5, -3, n)
    Ste = rng.uniform(0.2, 2.0, n)
    Nu = rng.uniform(1.0, 20.0, n)
    out = []
    for c in range(n):
        out.append(make_params(nx=int(side[c]), ny=int(side[c] * aspect[c]),
                               porosity=float(phi[c]), Ra=float(Ra[c]),
                               Pr=50.0, Da=float(Da[c]), Ste=float(Ste[c]),
                               k_ratio=100.0, cap_ratio=1.0, Nu_i=float(Nu[c])))
    return out, 50000, seed, "f32"


def scaled_cavity(p: dict, nx: int, ny: int | None = None) -> dict:
    """Same dimensionless groups on another grid."""
    q = dict(p)
    q["nx"] = int(nx)
    q["ny"] = int(ny if ny is not None else nx)
    return q


# --------------------------------------------------------------------------
# Initial temperature fields.
# --------------------------------------------------------------------------

def perturbation(seed: int, ny: int, nx: int, amplitude: float = 1e-6) -> np.ndarray:
    """Seeded uniform perturbation U(-a, a) of shape (ny, nx), float64."""
    return np.random.default_rng(seed).uniform(-amplitude, amplitude, size=(ny, nx))


def initial_temperatures(p: dict, seed: int | None, amplitude: float = 1e-6):
    """(T_pcm0, T_mf0) as (ny, nx) float64 arrays.

    Every node starts at T_init; with a seed, the interior nodes of the PCM
    field get the seeded perturbation.  Boundary values are left at T_init
    here: the solvers themselves impose the wall temperatures on the
    isothermal walls.
    """
    ny, nx = p["ny"], p["nx"]
    t_pcm = np.full((ny, nx), float(p["T_init"]))
    t_mf = np.full((ny, nx), float(p["T_init"]))
    if seed is not None:
        d = perturbation(seed, ny, nx, amplitude)
        if p["bc_x"] == 1:
            t_pcm[1:-1, :] += d[1:-1, :]
        else:
            t_pcm[1:-1, 1:-1] += d[1:-1, 1:-1]
    return t_pcm, t_mf
