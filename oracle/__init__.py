"""Plain FP64 CPU oracle of the DS-PHD/MIB particle recursion (arXiv 1605.02406).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path (the HIP
library and its binding) never imports, links or calls it.

This module is argument marshalling for ``dogm_oracle.c`` (numpy arrays <-> C pointers);
all arithmetic of the oracle lives in the C file, which cites the paper for each step.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dogm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the same source (a planted-mistake copy).
_LIB_OVERRIDE = os.environ.get("DOGM_ORACLE_LIB")

C_CONFLICT = 1
C_NOCARRIER = 2
C_NONFINITE = 4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-ffp-contract=off: no fused multiply-adds, so each FP64
    expression rounds exactly as written)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off", "-fPIC",
             "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ct.Structure):
    _fields_ = [("nx", ct.c_int32), ("ny", ct.c_int32), ("cell_size", ct.c_double),
                ("dt", ct.c_double), ("p_s", ct.c_double), ("p_b", ct.c_double),
                ("sigma_pos", ct.c_double), ("sigma_vel", ct.c_double),
                ("sigma_birth_vel", ct.c_double), ("alpha_free", ct.c_double),
                ("n_pers", ct.c_int64), ("n_born", ct.c_int64), ("seed", ct.c_uint64),
                ("grid_id", ct.c_uint32)]


@dataclass
class Params:
    """Filter parameters.  Float fields are the FP32 values the GPU library receives,
    widened to FP64 (so both sides start from identical parameter values)."""
    nx: int
    ny: int
    cell_size: float
    dt: float
    p_s: float
    p_b: float
    sigma_pos: float
    sigma_vel: float
    sigma_birth_vel: float
    alpha_free: float
    n_pers: int
    n_born: int
    seed: int = 0
    grid_id: int = 0

    @property
    def C(self) -> int:
        return self.nx * self.ny

    def _c(self) -> _Params:
        f = lambda v: float(np.float32(v))  # noqa: E731
        return _Params(self.nx, self.ny, f(self.cell_size), f(self.dt), f(self.p_s),
                       f(self.p_b), f(self.sigma_pos), f(self.sigma_vel),
                       f(self.sigma_birth_vel), f(self.alpha_free), self.n_pers,
                       self.n_born, self.seed, self.grid_id)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ct.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=False)
            L = ct.CDLL(_LIB)
        P = ct.POINTER(_Params)
        d, u32, u64, i64, u8 = (ct.POINTER(ct.c_double), ct.POINTER(ct.c_uint32),
                                ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_int64),
                                ct.POINTER(ct.c_uint8))
        f = ct.POINTER(ct.c_float)
        sig = {
            "or_philox4x32_10": (None, [u32, ct.c_uint64, u32]),
            "or_uniform": (ct.c_double, [ct.c_uint32]),
            "or_box_muller": (None, [ct.c_double, ct.c_double, d, d]),
            "or_predict_noise": (None, [P, ct.c_uint32, ct.c_int64, d]),
            "or_cell_key_f64": (ct.c_uint32, [P, ct.c_double, ct.c_double]),
            "or_cell_keys_f32": (None, [ct.c_int32, ct.c_int32, ct.c_float, ct.c_int64, f, f,
                                        u32]),
            "or_predict": (None, [P, ct.c_uint32, ct.c_int64, d, d, d, d, d, d, u32]),
            "or_assign": (ct.c_int, [ct.c_int64, ct.c_int64, u32, i64, u32, u32]),
            "or_dempster": (ct.c_int, [ct.c_double] * 4 + [d, d]),
            "or_cell_update": (ct.c_uint32, [P, ct.c_int64, d, u32, u32, d, d, d, d, d, d, d,
                                             d, d, d, d]),
            "or_cell_update_bayes": (ct.c_uint32, [P, ct.c_int64, d, u32, u32, d, d, d, d, d,
                                                   d, d, d, d, d, d]),
            "or_velocity_likelihood": (ct.c_double, [ct.c_double] * 5),
            "or_persistent_update": (None, [ct.c_int64, d, d, d, u32, u32, d, d, d, d, d, d,
                                            d]),
            "or_fixed40": (ct.c_uint64, [ct.c_double]),
            "or_born_alloc": (ct.c_uint64, [ct.c_int64, ct.c_int64, d, u32]),
            "or_num_assoc": (ct.c_int64, [ct.c_double, ct.c_int64]),
            "or_born_init": (ct.c_uint32, [P, ct.c_uint32, ct.c_int64, ct.c_int64, u32, d, d,
                                           d, d, d, d, d, d, d, d, d, u32, u8]),
            "or_moments": (None, [ct.c_int64, d, d, d, u32, u32, d, d, d, d, d, d, u8]),
            "or_resample_offset": (ct.c_double, [P, ct.c_uint32]),
            "or_resample_indices": (None, [ct.c_int64, ct.c_int64, d, d, ct.c_double, i64,
                                           u64]),
            "or_resample_weight": (ct.c_double, [ct.c_uint64, ct.c_int64]),
            "or_init_state": (None, [P, ct.c_int64, d, d, d, d, d]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a, dtype):
    """Pointer to a C-contiguous numpy array of exactly `dtype` (None passes NULL)."""
    if a is None:
        return None
    assert a.dtype == dtype and a.flags["C_CONTIGUOUS"], (a.dtype, dtype)
    return a.ctypes.data_as(ct.POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _d(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------------------------
# random numbers
# ------------------------------------------------------------------------------------

def philox(ctr, seed: int) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c, np.uint32), seed, _p(out, np.uint32))
    return out


def uniform(b: int) -> float:
    return lib().or_uniform(int(b))


def box_muller(u1: float, u2: float):
    a, b = ct.c_double(), ct.c_double()
    lib().or_box_muller(u1, u2, ct.byref(a), ct.byref(b))
    return a.value, b.value


def predict_noise(p: Params, cycle: int, n: int) -> np.ndarray:
    out = np.zeros((n, 4), np.float64)
    lib().or_predict_noise(ct.byref(p._c()), cycle, n, _p(out, np.float64))
    return out


# ------------------------------------------------------------------------------------
# a1 predict
# ------------------------------------------------------------------------------------

def cell_key_f64(p: Params, x: float, y: float) -> int:
    return lib().or_cell_key_f64(ct.byref(p._c()), x, y)


def cell_keys_f32(p: Params, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    key = np.zeros(len(x), np.uint32)
    lib().or_cell_keys_f32(p.nx, p.ny, float(np.float32(p.cell_size)), len(x),
                           _p(x, np.float32), _p(y, np.float32), _p(key, np.uint32))
    return key


def predict(p: Params, cycle: int, state: dict, noise=None):
    """state: dict of x, y, vx, vy, w (any float dtype).  Returns (new_state f64, key)."""
    s = {k: _d(state[k]).copy() for k in ("x", "y", "vx", "vy", "w")}
    n = len(s["x"])
    key = np.zeros(n, np.uint32)
    nz = None if noise is None else np.ascontiguousarray(noise, np.float64).reshape(-1)
    lib().or_predict(ct.byref(p._c()), cycle, n, *[_p(s[k], np.float64) for k in
                                                   ("x", "y", "vx", "vy", "w")],
                     _p(nz, np.float64), _p(key, np.uint32))
    return s, key


# ------------------------------------------------------------------------------------
# a2 assign
# ------------------------------------------------------------------------------------

def assign(key: np.ndarray, C: int):
    key = np.ascontiguousarray(key, np.uint32)
    n = len(key)
    perm = np.zeros(n, np.int64)
    start = np.zeros(C, np.uint32)
    end = np.zeros(C, np.uint32)
    rc = lib().or_assign(n, C, _p(key, np.uint32), _p(perm, np.int64), _p(start, np.uint32),
                         _p(end, np.uint32))
    if rc:
        raise ValueError(f"or_assign failed: {rc}")
    return perm, start, end


# ------------------------------------------------------------------------------------
# a3 cell update
# ------------------------------------------------------------------------------------

def dempster(o1, f1, o2, f2):
    o, f = ct.c_double(), ct.c_double()
    conflict = lib().or_dempster(o1, f1, o2, f2, ct.byref(o), ct.byref(f))
    return o.value, f.value, bool(conflict)


CELL_OUT = ("sum_w", "m_pO", "m_pF", "m_O", "m_F", "rho_b", "rho_p", "pign")


def cell_update(p: Params, w_sorted, start, end, m_free_prev, z_occ, z_free):
    C = p.C
    outs = {k: np.zeros(C, np.float64) for k in CELL_OUT}
    w = _d(w_sorted)
    st = lib().or_cell_update(
        ct.byref(p._c()), C, _p(w, np.float64), _p(np.ascontiguousarray(start, np.uint32),
                                                    np.uint32),
        _p(np.ascontiguousarray(end, np.uint32), np.uint32), _p(_d(m_free_prev), np.float64),
        _p(_d(z_occ), np.float64), _p(_d(z_free), np.float64),
        *[_p(outs[k], np.float64) for k in CELL_OUT])
    outs["status"] = int(st)
    return outs


def cell_update_bayes(p: Params, w_sorted, start, end, p_tp, p_fp, det):
    """The particle PHD/MIB cell step of Sec. V (p_A = 0): see or_cell_update_bayes."""
    C = p.C
    outs = {k: np.zeros(C, np.float64) for k in CELL_OUT}
    w = _d(w_sorted)
    st = lib().or_cell_update_bayes(
        ct.byref(p._c()), C, _p(w, np.float64), _p(np.ascontiguousarray(start, np.uint32),
                                                    np.uint32),
        _p(np.ascontiguousarray(end, np.uint32), np.uint32), _p(_d(p_tp), np.float64),
        _p(_d(p_fp), np.float64), _p(_d(det), np.float64),
        *[_p(outs[k], np.float64) for k in CELL_OUT])
    outs["status"] = int(st)
    return outs


# ------------------------------------------------------------------------------------
# a4 persistent update
# ------------------------------------------------------------------------------------

def velocity_likelihood(vx, vy, mux, muy, var):
    return lib().or_velocity_likelihood(vx, vy, mux, muy, var)


def persistent_update(C, w_sorted, vx, vy, start, end, rho_p, p_assoc=None, mu_vx=None,
                      mu_vy=None, var_v=None):
    w = _d(w_sorted).copy()
    mu_A = np.zeros(C, np.float64)
    mu_UA = np.zeros(C, np.float64)
    lib().or_persistent_update(
        C, _p(w, np.float64), _p(_d(vx), np.float64), _p(_d(vy), np.float64),
        _p(np.ascontiguousarray(start, np.uint32), np.uint32),
        _p(np.ascontiguousarray(end, np.uint32), np.uint32), _p(_d(rho_p), np.float64),
        _p(_d(p_assoc), np.float64), _p(_d(mu_vx), np.float64), _p(_d(mu_vy), np.float64),
        _p(_d(var_v), np.float64), _p(mu_A, np.float64), _p(mu_UA, np.float64))
    return w, mu_A, mu_UA


# ------------------------------------------------------------------------------------
# a5 new-born particles
# ------------------------------------------------------------------------------------

def fixed40(m: float) -> int:
    return lib().or_fixed40(m)


def born_alloc(C: int, nb: int, rho_b):
    off = np.zeros(C + 1, np.uint32)
    S = lib().or_born_alloc(C, nb, _p(_d(rho_b), np.float64), _p(off, np.uint32))
    return off, int(S)


def num_assoc(p_a: float, n_c: int) -> int:
    return lib().or_num_assoc(p_a, n_c)


BORN = ("x", "y", "vx", "vy", "w")


def born_init(p: Params, cycle: int, off, rho_b, p_assoc=None, mu_vx=None, mu_vy=None,
              var_v=None, noise=None):
    C, nb = p.C, p.n_born
    b = {k: np.zeros(nb, np.float64) for k in BORN}
    key = np.zeros(nb, np.uint32)
    assoc = np.zeros(nb, np.uint8)
    nz = None if noise is None else np.ascontiguousarray(noise, np.float64).reshape(-1)
    st = lib().or_born_init(
        ct.byref(p._c()), cycle, C, nb, _p(np.ascontiguousarray(off, np.uint32), np.uint32),
        _p(_d(rho_b), np.float64), _p(_d(p_assoc), np.float64), _p(_d(mu_vx), np.float64),
        _p(_d(mu_vy), np.float64), _p(_d(var_v), np.float64), _p(nz, np.float64),
        *[_p(b[k], np.float64) for k in BORN], _p(key, np.uint32), _p(assoc, np.uint8))
    b["key"] = key
    b["assoc"] = assoc
    b["status"] = int(st)
    return b


# ------------------------------------------------------------------------------------
# a6 moments
# ------------------------------------------------------------------------------------

MOM = ("mean_x", "mean_y", "var_x", "var_y", "cov_xy")


def moments(C, w, vx, vy, start, end, rho_p):
    outs = {k: np.zeros(C, np.float64) for k in MOM}
    flag = np.zeros(C, np.uint8)
    lib().or_moments(C, _p(_d(w), np.float64), _p(_d(vx), np.float64), _p(_d(vy), np.float64),
                     _p(np.ascontiguousarray(start, np.uint32), np.uint32),
                     _p(np.ascontiguousarray(end, np.uint32), np.uint32),
                     _p(_d(rho_p), np.float64), *[_p(outs[k], np.float64) for k in MOM],
                     _p(flag, np.uint8))
    outs["flag"] = flag
    return outs


# ------------------------------------------------------------------------------------
# a7 resample
# ------------------------------------------------------------------------------------

def resample_offset(p: Params, cycle: int) -> float:
    return lib().or_resample_offset(ct.byref(p._c()), cycle)


def resample_indices(w_pers, w_born, U: float):
    wp, wb = _d(w_pers), _d(w_born)
    nu, nb = len(wp), len(wb)
    idx = np.zeros(nu, np.int64)
    W = ct.c_uint64()
    lib().or_resample_indices(nu, nb, _p(wp, np.float64), _p(wb, np.float64), U,
                              _p(idx, np.int64), ct.byref(W))
    return idx, int(W.value)


def resample_weight(W_fixed: int, nu: int) -> float:
    return lib().or_resample_weight(W_fixed, nu)


def resample(p: Params, cycle: int, pers: dict, born: dict, U=None):
    """pers / born: dicts of x, y, vx, vy, w.  Returns (next state dict f64, idx, W_fixed)."""
    if U is None:
        U = resample_offset(p, cycle)
    idx, W = resample_indices(pers["w"], born["w"], U)
    nu = len(idx)
    out = {}
    for k in ("x", "y", "vx", "vy"):
        joint = np.concatenate([_d(pers[k]), _d(born[k])])
        out[k] = joint[idx]
    out["w"] = (np.full(nu, resample_weight(W, nu)) if W > 0 else _d(pers["w"]).copy())
    return out, idx, W


def init_state(p: Params, n: int) -> dict:
    s = {k: np.zeros(n, np.float64) for k in ("x", "y", "vx", "vy", "w")}
    lib().or_init_state(ct.byref(p._c()), n, *[_p(s[k], np.float64) for k in
                                                ("x", "y", "vx", "vy", "w")])
    return s


# ------------------------------------------------------------------------------------
# one full cycle, composed from the steps above in the paper's order (Alg. 1-7)
# ------------------------------------------------------------------------------------

def cycle(p: Params, k: int, state: dict, m_F, meas: dict):
    """Runs the whole recursion for cycle k in FP64.  Returns (new state, new m_F, info)
    where info holds every intermediate per-cell and new-born output."""
    C = p.C
    pred, key = predict(p, k, state)
    perm, start, end = assign(key, C)
    srt = {kk: pred[kk][perm] for kk in ("x", "y", "vx", "vy", "w")}
    if "det" in meas:  # the particle PHD/MIB filter of Sec. V
        cu = cell_update_bayes(p, srt["w"], start, end, meas["p_tp"], meas["p_fp"], meas["det"])
    else:
        cu = cell_update(p, srt["w"], start, end, m_F, meas["m_occ"], meas["m_free"])
    opt = {kk: meas.get(kk) for kk in ("p_assoc", "mu_vx", "mu_vy", "var_v")}
    w_post, mu_A, mu_UA = persistent_update(C, srt["w"], srt["vx"], srt["vy"], start, end,
                                            cu["rho_p"], **opt)
    srt["w"] = w_post
    off, S = born_alloc(C, p.n_born, cu["rho_b"])
    born = born_init(p, k, off, cu["rho_b"], **opt)
    mom = moments(C, srt["w"], srt["vx"], srt["vy"], start, end, cu["rho_p"])
    nxt, idx, W = resample(p, k, srt, born)
    info = dict(cu, key=key, perm=perm, start=start, end=end, sorted=srt, mu_A=mu_A,
                mu_UA=mu_UA, born_off=off, S_fixed=S, born=born, moments=mom, idx=idx,
                W_fixed=W)
    return nxt, cu["m_F"], info
