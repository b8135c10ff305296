"""Thin ctypes binding of liblbmpcm.so (include/lbmpcm.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Function names match the C entry points.  Importing this
module loads the shared library and raises if it has not been built, so
that nothing can silently run without the GPU code.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# LBMPCM_LIBRARY selects another build of the same sources (e.g. a variant
# compiled with other cache hints); the default is the in-tree library.
LIB_PATH = os.environ.get("LBMPCM_LIBRARY") or os.path.join(_HERE, "liblbmpcm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_ENONFINITE, LBM_ESTATE, LBM_EIO = 0, -1, -2, -3, -4, -5, -6
LBM_F64, LBM_F32, LBM_F16_OFFSET, LBM_BF16_OFFSET, LBM_F16_SPLIT, LBM_F32_H64, LBM_BF16_SPLIT = 0, 1, 2, 3, 4, 5, 6
PRECISIONS = {"f64": LBM_F64, "f32": LBM_F32, "f16": LBM_F16_OFFSET, "bf16": LBM_BF16_OFFSET,
              "f16split": LBM_F16_SPLIT, "f32h64": LBM_F32_H64, "bf16split": LBM_BF16_SPLIT}
STATE_BYTES_PER_NODE = {LBM_F64: 216, LBM_F32: 108, LBM_F16_OFFSET: 54, LBM_BF16_OFFSET: 54,
                        LBM_F16_SPLIT: 72, LBM_F32_H64: 112, LBM_BF16_SPLIT: 72}
# with D2Q5 thermal fields (19 populations per node)
STATE_BYTES_PER_NODE_D2Q5 = {LBM_F64: 152, LBM_F32: 76, LBM_F32_H64: 80}


def state_bytes_per_node(precision, thermal_lattice=9) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    if int(thermal_lattice) == 5:
        return STATE_BYTES_PER_NODE_D2Q5[prec]
    return STATE_BYTES_PER_NODE[prec]


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("bc_x", ctypes.c_int32),
        ("gravity_axis", ctypes.c_int32),
        ("porosity", ctypes.c_double), ("Ra", ctypes.c_double), ("Pr", ctypes.c_double),
        ("Da", ctypes.c_double), ("Ste", ctypes.c_double), ("k_ratio", ctypes.c_double),
        ("cap_ratio", ctypes.c_double), ("Nu_i", ctypes.c_double), ("F_phi", ctypes.c_double),
        ("dp_over_L", ctypes.c_double), ("k_f", ctypes.c_double), ("cf_ref", ctypes.c_double),
        ("cm_ref", ctypes.c_double), ("J", ctypes.c_double), ("T_hot", ctypes.c_double),
        ("T_cold", ctypes.c_double), ("T_init", ctypes.c_double), ("T_solidus", ctypes.c_double),
        ("T_liquidus", ctypes.c_double),
        ("thermal_lattice", ctypes.c_int32), ("thermal_collision", ctypes.c_int32),
        ("varpi", ctypes.c_double), ("zeta_e", ctypes.c_double),
        ("wall_type", ctypes.c_int32 * 4), ("wall_T", ctypes.c_double * 4),
        ("L_char", ctypes.c_double), ("solid_treatment", ctypes.c_int32),
        ("band_rows", ctypes.c_int32), ("pcm_even_rates", ctypes.c_int32),
    ]


class lbm_lattice(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("L", "k_f", "k_m", "nu_f", "nu_e", "K", "F_phi", "gbeta", "h_v", "L_a", "d_p", "z",
                 "tau_v", "tau_g", "tau_h")] + \
               [("s", ctypes.c_double * 9), ("zeta", ctypes.c_double * 9), ("eta", ctypes.c_double * 9)] + \
               [(n, ctypes.c_double) for n in ("H_fs", "H_fl", "T_ref", "H_ref")] + \
               [("scale_exp", ctypes.c_double * 3), ("q_thermal", ctypes.c_double),
                ("varpi", ctypes.c_double), ("wall_type", ctypes.c_double * 4),
                ("wall_T", ctypes.c_double * 4), ("solid_treatment", ctypes.c_double)]


DIAG_NAMES = ["step", "Fo", "liquid_fraction", "Nu_hot", "Nu_hot_pcm", "Nu_cold",
              "E_int", "E_int0", "flux_E", "energy_residual",
              "M_int", "M_int0", "flux_M", "mass_residual",
              "x_front_mid", "max_dT_LTNE", "u_max", "nonfinite"]


class lbm_diag(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double * 4) if n in ("flux_E", "flux_M") else (n, ctypes.c_double)
                for n in DIAG_NAMES]


class lbm_launch_config(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("nodes_per_thread", ctypes.c_int32),
                ("xcd_remap", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("steps_per_launch", ctypes.c_int32), ("tile_shape", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    H = ctypes.c_void_p
    PP = ctypes.POINTER(lbm_params)
    dp = ctypes.POINTER(ctypes.c_double)
    st = ctypes.c_int
    sig = {
        "lbm_create": ([PP, ctypes.c_int, ctypes.POINTER(H)], st),
        "lbm_create_batch": ([PP, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(H)], st),
        "lbm_workspace_bytes": ([PP, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)], st),
        "lbm_create_ext": ([PP, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                            ctypes.c_void_p, ctypes.POINTER(H)], st),
        "lbm_set_stream": ([H, ctypes.c_void_p], st),
        "lbm_set_initial": ([H, ctypes.c_int32, dp, dp], st),
        "lbm_step": ([H, ctypes.c_int64], st),
        "lbm_step_per_cavity": ([H, ctypes.c_int64], st),
        "lbm_synchronize": ([H], st),
        "lbm_step_count": ([H], ctypes.c_int64),
        "lbm_fields": ([H, ctypes.c_int32, dp, dp, dp, dp, dp, dp], st),
        "lbm_fields_rows": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, dp, dp, dp, dp, dp, dp], st),
        "lbm_diagnostics": ([H, ctypes.c_int32, ctypes.POINTER(lbm_diag)], st),
        "lbm_diagnostics_noalloc": ([H, ctypes.c_int32, ctypes.POINTER(lbm_diag)], st),
        "lbm_get_lattice": ([H, ctypes.c_int32, ctypes.POINTER(lbm_lattice)], st),
        "lbm_lattice_of": ([PP, ctypes.c_int, ctypes.POINTER(lbm_lattice)], st),
        "lbm_get_launch": ([H, ctypes.POINTER(lbm_launch_config)], st),
        "lbm_set_launch": ([H, ctypes.POINTER(lbm_launch_config)], st),
        "lbm_autotune": ([H, ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(lbm_launch_config)], st),
        "lbm_save": ([H, ctypes.c_char_p], st),
        "lbm_load": ([H, ctypes.c_char_p], st),
        "lbm_copy_state": ([H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64], st),
        "lbm_debug_poke": ([H, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int32, ctypes.c_double], st),
        "lbm_destroy": ([H], st),
        "lbm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ("lbm_create", "lbm_create_batch", "lbm_workspace_bytes", "lbm_create_ext",
            "lbm_set_stream", "lbm_set_initial", "lbm_step", "lbm_step_per_cavity",
            "lbm_synchronize", "lbm_step_count", "lbm_fields", "lbm_fields_rows", "lbm_diagnostics",
            "lbm_diagnostics_noalloc",
            "lbm_get_lattice", "lbm_lattice_of", "lbm_get_launch", "lbm_set_launch", "lbm_autotune", "lbm_save",
            "lbm_load", "lbm_copy_state", "lbm_debug_poke", "lbm_destroy", "lbm_last_error")


def _check(status: int):
    if status != LBM_OK:
        raise LbmError(status, (_lib.lbm_last_error() or b"").decode())


def _params_array(params):
    if isinstance(params, dict):
        params = [params]
    arr = (lbm_params * len(params))()
    for i, p in enumerate(params):
        for name, typ in lbm_params._fields_:
            if hasattr(typ, "_length_"):
                dst = getattr(arr[i], name)
                vals = list(p[name])
                if len(vals) != typ._length_:
                    raise ValueError(f"{name} needs {typ._length_} entries")
                for k, v in enumerate(vals):
                    dst[k] = v
            else:
                # band_rows (storage only) and pcm_even_rates may be absent (0)
                setattr(arr[i], name, p.get(name, 0) if name in ("band_rows", "pcm_even_rates") else p[name])
    return arr


def _dptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prec(p):
    return PRECISIONS[p] if isinstance(p, str) else int(p)


# ---------------------------------------------------------------------------
# Same-name wrappers of the C entry points (handles are opaque ints).
# ---------------------------------------------------------------------------

def lbm_create(params: dict, precision="f32") -> int:
    h = ctypes.c_void_p()
    _check(_lib.lbm_create(_params_array(params), _prec(precision), ctypes.byref(h)))
    return h.value


def lbm_create_batch(params: list, precision="f32") -> int:
    h = ctypes.c_void_p()
    arr = _params_array(params)
    _check(_lib.lbm_create_batch(arr, len(params), _prec(precision), ctypes.byref(h)))
    return h.value


def lbm_workspace_bytes(params, precision="f32") -> int:
    arr = _params_array(params)
    b = ctypes.c_uint64()
    _check(_lib.lbm_workspace_bytes(arr, len(arr), _prec(precision), ctypes.byref(b)))
    return int(b.value)


def lbm_create_ext(params, precision, workspace_ptr: int, workspace_bytes: int, stream_ptr: int) -> int:
    arr = _params_array(params)
    h = ctypes.c_void_p()
    _check(_lib.lbm_create_ext(arr, len(arr), _prec(precision), ctypes.c_void_p(workspace_ptr),
                               workspace_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h)))
    return h.value


def lbm_set_stream(h: int, stream_ptr: int):
    _check(_lib.lbm_set_stream(h, ctypes.c_void_p(stream_ptr)))


def lbm_set_initial(h: int, cavity: int, T_pcm0=None, T_mf0=None):
    a = None if T_pcm0 is None else np.ascontiguousarray(T_pcm0, dtype=np.float64)
    b = None if T_mf0 is None else np.ascontiguousarray(T_mf0, dtype=np.float64)
    _check(_lib.lbm_set_initial(h, cavity, _dptr(a), _dptr(b)))


def lbm_step(h: int, n: int):
    _check(_lib.lbm_step(h, int(n)))


def lbm_step_per_cavity(h: int, n: int):
    _check(_lib.lbm_step_per_cavity(h, int(n)))


def lbm_synchronize(h: int):
    _check(_lib.lbm_synchronize(h))


def lbm_step_count(h: int) -> int:
    return int(_lib.lbm_step_count(h))


def lbm_fields(h: int, cavity: int, shape) -> dict:
    ny, nx = shape
    out = {k: np.empty((ny, nx)) for k in ("ux", "uy", "T_pcm", "T_mf", "f_l", "rho")}
    _check(_lib.lbm_fields(h, cavity, _dptr(out["ux"]), _dptr(out["uy"]), _dptr(out["T_pcm"]),
                           _dptr(out["T_mf"]), _dptr(out["f_l"]), _dptr(out["rho"])))
    return out


def lbm_fields_rows(h: int, cavity: int, nx: int, y0: int, rows: int) -> dict:
    out = {k: np.empty((max(rows, 0), nx)) for k in ("ux", "uy", "T_pcm", "T_mf", "f_l", "rho")}
    _check(_lib.lbm_fields_rows(h, cavity, y0, rows, _dptr(out["ux"]), _dptr(out["uy"]), _dptr(out["T_pcm"]),
                                _dptr(out["T_mf"]), _dptr(out["f_l"]), _dptr(out["rho"])))
    return out


def lbm_diagnostics(h: int, cavity: int = 0, allow_nonfinite: bool = False) -> dict:
    d = lbm_diag()
    st = _lib.lbm_diagnostics(h, cavity, ctypes.byref(d))
    if not (allow_nonfinite and st == LBM_ENONFINITE):
        _check(st)
    out = {n: (list(getattr(d, n)) if n in ("flux_E", "flux_M") else float(getattr(d, n)))
           for n in DIAG_NAMES}
    out["status"] = st
    return out


def lbm_diagnostics_noalloc(h: int, cavity: int = 0, allow_nonfinite: bool = False) -> dict:
    d = lbm_diag()
    st = _lib.lbm_diagnostics_noalloc(h, cavity, ctypes.byref(d))
    if not (allow_nonfinite and st == LBM_ENONFINITE):
        _check(st)
    out = {n: (list(getattr(d, n)) if n in ("flux_E", "flux_M") else float(getattr(d, n)))
           for n in DIAG_NAMES}
    out["status"] = st
    return out


def lbm_get_lattice(h: int, cavity: int = 0) -> dict:
    l = lbm_lattice()
    _check(_lib.lbm_get_lattice(h, cavity, ctypes.byref(l)))
    out = {}
    for n, t in lbm_lattice._fields_:
        v = getattr(l, n)
        out[n] = list(v) if hasattr(v, "__len__") else float(v)
    return out


def lbm_lattice_of(params: dict, precision="f32") -> dict:
    l = lbm_lattice()
    _check(_lib.lbm_lattice_of(_params_array(params), _prec(precision), ctypes.byref(l)))
    out = {}
    for n, t in lbm_lattice._fields_:
        v = getattr(l, n)
        out[n] = list(v) if hasattr(v, "__len__") else float(v)
    return out


def lbm_get_launch(h: int) -> dict:
    c = lbm_launch_config()
    _check(_lib.lbm_get_launch(h, ctypes.byref(c)))
    return {n: int(getattr(c, n)) for n, _ in lbm_launch_config._fields_}


def lbm_set_launch(h: int, block=256, nodes_per_thread=1, xcd_remap=1, persistent=0, steps_per_launch=None,
                   tile_shape=None):
    """steps_per_launch and tile_shape None keep the handle's current setting."""
    cur = lbm_get_launch(h)
    if steps_per_launch is None:
        steps_per_launch = cur["steps_per_launch"]
    if tile_shape is None:
        tile_shape = cur["tile_shape"] if steps_per_launch == cur["steps_per_launch"] else 0
    c = lbm_launch_config(block, nodes_per_thread, xcd_remap, persistent, steps_per_launch, tile_shape, 0, 0)
    _check(_lib.lbm_set_launch(h, ctypes.byref(c)))


def lbm_autotune(h: int, steps_per_trial: int = 5, cache_path: str | None = None) -> dict:
    c = lbm_launch_config()
    _check(_lib.lbm_autotune(h, steps_per_trial, None if cache_path is None else cache_path.encode(),
                             ctypes.byref(c)))
    return {n: int(getattr(c, n)) for n, _ in lbm_launch_config._fields_}


def lbm_save(h: int, path: str):
    _check(_lib.lbm_save(h, path.encode()))


def lbm_load(h: int, path: str):
    _check(_lib.lbm_load(h, path.encode()))


def lbm_copy_state(h: int, cavity: int, shape, precision, thermal_lattice=9) -> np.ndarray:
    """Raw stored bytes of one cavity (uint8, planes in storage order)."""
    ny, nx = shape
    a = np.empty(state_bytes_per_node(precision, thermal_lattice) * ny * nx, dtype=np.uint8)
    _check(_lib.lbm_copy_state(h, cavity, a.ctypes.data_as(ctypes.c_void_p), a.nbytes))
    return a


def lbm_debug_poke(h: int, cavity: int, x: int, y: int, field: int, direction: int, value: float):
    _check(_lib.lbm_debug_poke(h, cavity, x, y, field, direction, float(value)))


def lbm_destroy(h: int):
    _check(_lib.lbm_destroy(h))


def lbm_last_error() -> str:
    return (_lib.lbm_last_error() or b"").decode()


class Solver:
    """Convenience owner of one handle (single cavity or a batch)."""

    def __init__(self, params, precision="f32", workspace=None, stream=None):
        self.params = [params] if isinstance(params, dict) else list(params)
        self.precision = _prec(precision)
        if workspace is not None:
            self.h = lbm_create_ext(self.params, self.precision, workspace[0], workspace[1],
                                    stream or 0)
        elif len(self.params) == 1:
            self.h = lbm_create(self.params[0], self.precision)
        else:
            self.h = lbm_create_batch(self.params, self.precision)

    def close(self):
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, c=0):
        return (self.params[c]["ny"], self.params[c]["nx"])

    def set_initial(self, c, T_pcm0=None, T_mf0=None):
        lbm_set_initial(self.h, c, T_pcm0, T_mf0)

    def step(self, n):
        lbm_step(self.h, n)

    def fields(self, c=0):
        return lbm_fields(self.h, c, self.shape(c))

    def fields_rows(self, y0, rows, c=0):
        return lbm_fields_rows(self.h, c, self.shape(c)[1], y0, rows)

    def diagnostics(self, c=0, allow_nonfinite=False):
        return lbm_diagnostics(self.h, c, allow_nonfinite)

    def state(self, c=0):
        return lbm_copy_state(self.h, c, self.shape(c), self.precision,
                              self.params[c].get("thermal_lattice", 9) or 9)
