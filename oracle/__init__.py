"""FP64 CPU oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps the plain C implementation in
``lbm_oracle.c`` and maps the dimensionless problem description to lattice
units on its own (``mapping.py``); it shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

from .mapping import lattice_params  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_liboracle.so")
_lib = None

Q = 9


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over rows)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared",
           "-fPIC", "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("gx0", ctypes.c_int), ("gy0", ctypes.c_int),
        ("NX", ctypes.c_int), ("NY", ctypes.c_int), ("periodic_x", ctypes.c_int),
        ("gravity_axis", ctypes.c_int),
        ("phi", ctypes.c_double), ("rho_l", ctypes.c_double), ("rho_m", ctypes.c_double),
        ("c_pl", ctypes.c_double), ("c_ps", ctypes.c_double), ("c_pm", ctypes.c_double),
        ("c_fref", ctypes.c_double), ("c_mref", ctypes.c_double),
        ("nu_f", ctypes.c_double), ("K", ctypes.c_double), ("F_phi", ctypes.c_double),
        ("gbeta", ctypes.c_double), ("T0", ctypes.c_double),
        ("h_v", ctypes.c_double), ("L_a", ctypes.c_double), ("T_fs", ctypes.c_double),
        ("T_fl", ctypes.c_double), ("T_hot", ctypes.c_double), ("T_cold", ctypes.c_double),
        ("k_f", ctypes.c_double), ("k_m", ctypes.c_double), ("L", ctypes.c_double),
        ("s", ctypes.c_double * Q), ("zeta", ctypes.c_double * Q), ("eta", ctypes.c_double * Q),
        ("qt", ctypes.c_int), ("varpi", ctypes.c_double), ("wall_type", ctypes.c_int * 4),
        ("wall_T", ctypes.c_double * 4), ("bounce_back", ctypes.c_int),
    ]


_DIAG_NAMES = ["step", "Fo", "liquid_fraction", "Nu_hot", "Nu_hot_pcm", "Nu_cold",
               "E_int", "E_int0", "flux_E", "energy_residual",
               "M_int", "M_int0", "flux_M", "mass_residual",
               "x_front_mid", "max_dT_LTNE", "u_max", "nonfinite"]


class OracleDiag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double * 4) if n in ("flux_E", "flux_M") else (n, ctypes.c_double)
                for n in _DIAG_NAMES]


def load():
    """Load the compiled oracle, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    P = ctypes.POINTER(OracleParams)
    lib.oracle_new.argtypes = [P]
    lib.oracle_new.restype = vp
    lib.oracle_free.argtypes = [vp]
    lib.oracle_set_initial.argtypes = [vp, dp, dp]
    lib.oracle_step.argtypes = [vp, ctypes.c_long]
    lib.oracle_fields.argtypes = [vp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(ctypes.c_ubyte)]
    lib.oracle_populations.argtypes = [vp, dp, dp, dp, dp]
    lib.oracle_diagnostics.argtypes = [vp, ctypes.POINTER(OracleDiag)]
    lib.oracle_poke.argtypes = [vp, ctypes.c_long, ctypes.c_int, ctypes.c_int, ctypes.c_double]
    lib.oracle_step_count.argtypes = [vp]
    lib.oracle_step_count.restype = ctypes.c_long
    lib.oracle_feq.argtypes = [ctypes.c_double] * 4 + [dp]
    lib.oracle_geq.argtypes = [ctypes.c_double] * 7 + [dp]
    lib.oracle_heq.argtypes = [ctypes.c_double] * 3 + [dp]
    lib.oracle_geq5.argtypes = [ctypes.c_double] * 8 + [dp]
    lib.oracle_heq5.argtypes = [ctypes.c_double] * 4 + [dp]
    lib.oracle_lattice5.argtypes = [dp, dp]
    lib.oracle_eos.argtypes = [P, ctypes.c_double, dp, dp]
    lib.oracle_enthalpy_of_T.argtypes = [P, ctypes.c_double]
    lib.oracle_enthalpy_of_T.restype = ctypes.c_double
    lib.oracle_node_macros.argtypes = [P, dp, dp, dp, dp]
    lib.oracle_collide_node.argtypes = [P, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                        dp, dp, dp, dp]
    lib.oracle_lattice.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                   dp, dp, dp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_struct(lp: dict, window=None) -> OracleParams:
    """Fill the C parameter struct from a lattice-parameter dict."""
    s = OracleParams()
    NX, NY = lp["nx"], lp["ny"]
    if window is None:
        gx0, gy0, nx, ny = 0, 0, NX, NY
    else:
        gx0, gy0, nx, ny = window
    s.nx, s.ny, s.gx0, s.gy0, s.NX, s.NY = nx, ny, gx0, gy0, NX, NY
    s.periodic_x = lp["periodic_x"]
    s.gravity_axis = lp["gravity_axis"]
    for k in ("phi", "rho_l", "rho_m", "c_pl", "c_ps", "c_pm", "c_fref", "c_mref", "nu_f", "K",
              "F_phi", "gbeta", "T0", "h_v", "L_a", "T_fs", "T_fl", "T_hot", "T_cold", "k_f",
              "k_m", "L"):
        setattr(s, k, float(lp[k]))
    for k in ("s", "zeta", "eta"):
        arr = getattr(s, k)
        for i, v in enumerate(lp[k]):
            arr[i] = float(v)
    s.qt = int(lp.get("qt", 9))
    s.varpi = float(lp.get("varpi", 0.0))
    wt = lp.get("wall_type", [1, 1, 2, 2])
    wT = lp.get("wall_T", [lp["T_hot"], lp["T_cold"], 0.0, 0.0])
    for w in range(4):
        s.wall_type[w] = int(wt[w])
        s.wall_T[w] = float(wT[w])
    s.bounce_back = int(lp.get("solid_treatment", 0))
    return s


class Oracle:
    """One cavity (or a window of one) advanced by the plain FP64 update."""

    def __init__(self, params: dict, window=None, lattice: dict | None = None):
        self.lib = load()
        self.lp = lattice if lattice is not None else lattice_params(params)
        self.struct = make_struct(self.lp, window)
        self.nx, self.ny = self.struct.nx, self.struct.ny
        self.h = self.lib.oracle_new(ctypes.byref(self.struct))
        if not self.h:
            raise ValueError("oracle_new rejected the geometry")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_free(h)
            self.h = None

    def set_initial(self, T_f0: np.ndarray, T_m0: np.ndarray):
        a = np.ascontiguousarray(T_f0, dtype=np.float64).reshape(self.ny, self.nx)
        b = np.ascontiguousarray(T_m0, dtype=np.float64).reshape(self.ny, self.nx)
        self.lib.oracle_set_initial(self.h, _ptr(a), _ptr(b))

    def step(self, n: int):
        self.lib.oracle_step(self.h, int(n))

    @property
    def step_count(self) -> int:
        return int(self.lib.oracle_step_count(self.h))

    def fields(self) -> dict:
        shp = (self.ny, self.nx)
        out = {k: np.zeros(shp) for k in ("ux", "uy", "T_pcm", "T_mf", "f_l", "rho")}
        valid = np.zeros(shp, dtype=np.uint8)
        self.lib.oracle_fields(self.h, _ptr(out["ux"]), _ptr(out["uy"]), _ptr(out["T_pcm"]),
                               _ptr(out["T_mf"]), _ptr(out["f_l"]), _ptr(out["rho"]),
                               valid.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)))
        out["valid"] = valid.astype(bool)
        return out

    def populations(self) -> dict:
        shp = (self.ny, self.nx, Q)
        f, g, h = np.zeros(shp), np.zeros(shp), np.zeros(shp)
        sr = np.zeros((self.ny, self.nx))
        self.lib.oracle_populations(self.h, _ptr(f), _ptr(g), _ptr(h), _ptr(sr))
        return {"f": f, "g": g, "h": h, "sr_f": sr}

    def diagnostics(self) -> dict:
        d = OracleDiag()
        self.lib.oracle_diagnostics(self.h, ctypes.byref(d))
        out = {}
        for n in _DIAG_NAMES:
            v = getattr(d, n)
            out[n] = list(v) if n in ("flux_E", "flux_M") else float(v)
        return out

    def poke(self, node: int, field: int, direction: int, value: float):
        self.lib.oracle_poke(self.h, int(node), int(field), int(direction), float(value))


# ---------------------------------------------------------------------------
# Single-node entry points used by the algebra pins.
# ---------------------------------------------------------------------------

def lattice_tables():
    lib = load()
    ex = (ctypes.c_int * Q)()
    ey = (ctypes.c_int * Q)()
    w = np.zeros(Q)
    M = np.zeros(Q * Q)
    Minv = np.zeros(Q * Q)
    lib.oracle_lattice(ex, ey, _ptr(w), _ptr(M), _ptr(Minv))
    return np.array(ex[:]), np.array(ey[:]), w, M.reshape(Q, Q), Minv.reshape(Q, Q)


def lattice5_tables():
    """D2Q5 transformation matrix (Eq. B1) and its numerical inverse."""
    M = np.zeros(25)
    Minv = np.zeros(25)
    load().oracle_lattice5(_ptr(M), _ptr(Minv))
    return M.reshape(5, 5), Minv.reshape(5, 5)


def geq5(H, T, ux, uy, phi, c_fref, c_pl, varpi):
    out = np.zeros(5)
    load().oracle_geq5(H, T, ux, uy, phi, c_fref, c_pl, varpi, _ptr(out))
    return out


def heq5(T_m, c_pm, c_mref, varpi):
    out = np.zeros(5)
    load().oracle_heq5(T_m, c_pm, c_mref, varpi, _ptr(out))
    return out


def feq(rho, ux, uy, phi):
    out = np.zeros(Q)
    load().oracle_feq(rho, ux, uy, phi, _ptr(out))
    return out


def geq(H, T, ux, uy, phi, c_fref, c_pl):
    out = np.zeros(Q)
    load().oracle_geq(H, T, ux, uy, phi, c_fref, c_pl, _ptr(out))
    return out


def heq(T_m, c_pm, c_mref):
    out = np.zeros(Q)
    load().oracle_heq(T_m, c_pm, c_mref, _ptr(out))
    return out


def eos(lp: dict, H: float):
    s = make_struct(lp)
    T = ctypes.c_double()
    fl = ctypes.c_double()
    load().oracle_eos(ctypes.byref(s), H, ctypes.byref(T), ctypes.byref(fl))
    return T.value, fl.value


def enthalpy_of_T(lp: dict, T: float) -> float:
    s = make_struct(lp)
    return load().oracle_enthalpy_of_T(ctypes.byref(s), T)


def node_macros(lp: dict, fplus, g, h) -> dict:
    s = make_struct(lp)
    out = np.zeros(9)
    a, b, c = (np.ascontiguousarray(x, dtype=np.float64) for x in (fplus, g, h))
    load().oracle_node_macros(ctypes.byref(s), _ptr(a), _ptr(b), _ptr(c), _ptr(out))
    return dict(zip(["H", "T_f", "f_l", "T_m", "rho", "ux", "uy", "Gx", "Gy"], out))


def collide_node(lp: dict, fplus, g, h, srf_prev, srm_prev):
    s = make_struct(lp)
    a, b, c = (np.ascontiguousarray(x, dtype=np.float64) for x in (fplus, g, h))
    fo, go, ho, sr = np.zeros(Q), np.zeros(Q), np.zeros(Q), np.zeros(2)
    load().oracle_collide_node(ctypes.byref(s), _ptr(a), _ptr(b), _ptr(c), float(srf_prev),
                               float(srm_prev), _ptr(fo), _ptr(go), _ptr(ho), _ptr(sr))
    return fo, go, ho, sr


def run_case(params: dict, steps: int, T_f0, T_m0, window=None):
    """Convenience: build, initialise and advance one oracle instance."""
    o = Oracle(params, window=window)
    o.set_initial(T_f0, T_m0)
    o.step(steps)
    return o
