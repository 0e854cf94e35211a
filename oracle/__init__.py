"""FP64 CPU oracle of the REV-scale DDF-MRT lattice Boltzmann model
(Liu & He, arXiv:1611.03329), exposed through ctypes.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package.  The product library under
``paper_1611_03329_amd`` never imports it, and the two share no code: the C
source here is written directly from the paper (Eqs. 4-43, App. A) and applies
the printed matrices densely, one node at a time.

Parity unpinned: none of the functions here is unpinned; see ``tests/test_oracle_*``
for the pin of each one.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_SRC_ENTH = os.path.join(_HERE, "enthalpy_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FACE_NAMES = ("-x", "+x", "-y", "+y", "-z", "+z")
FLOW = {"periodic": 0, "wall": 1, "outlet": 3}
HEAT = {"periodic": 0, "adiabatic": 1, "isothermal": 2, "outflow": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP over nodes)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, _SRC_ENTH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Face(ctypes.Structure):
    _fields_ = [("flow", ctypes.c_int32), ("heat", ctypes.c_int32),
                ("T_wall", ctypes.c_double), ("u_wall", ctypes.c_double * 3)]


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("porosity", ctypes.c_double), ("darcy", ctypes.c_double),
        ("rayleigh", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("reynolds", ctypes.c_double), ("u_char", ctypes.c_double),
        ("mach", ctypes.c_double), ("forchheimer", ctypes.c_double),
        ("sigma", ctypes.c_double), ("J", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("varpi", ctypes.c_double),
        ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_j", ctypes.c_double), ("s_q", ctypes.c_double), ("s_pi", ctypes.c_double),
        ("s_m", ctypes.c_double),
        ("zeta_T", ctypes.c_double), ("zeta_e", ctypes.c_double), ("zeta_nu", ctypes.c_double),
        ("s_nu_set", ctypes.c_double), ("zeta_alpha_set", ctypes.c_double),
        ("gravity_axis", ctypes.c_int32), ("length_axis", ctypes.c_int32),
        ("T_ref", ctypes.c_double), ("delta_T", ctypes.c_double),
        ("accel", ctypes.c_double * 3),
        ("face", _Face * 6),
        ("init_axis", ctypes.c_int32),
        ("init_T_lo", ctypes.c_double), ("init_T_hi", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
        ("init_u", ctypes.c_double * 3),
    ]


class _Derived(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("L", "s_nu", "zeta_alpha", "nu_e", "nu", "alpha_e", "alpha", "K",
                 "F_phi", "gbeta", "l0", "l1")]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.ref_default_params.argtypes = [ctypes.POINTER(_Params)]
        L.ref_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        L.ref_destroy.argtypes = [ctypes.c_void_p]
        L.ref_destroy.restype = None
        L.ref_get_derived.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Derived)]
        L.ref_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ref_time.argtypes = [ctypes.c_void_p]
        L.ref_time.restype = ctypes.c_int64
        L.ref_fields.argtypes = [ctypes.c_void_p, _D, _D, _D, _D, _D]
        L.ref_nusselt.argtypes = [ctypes.c_void_p, _D]
        L.ref_get_state.argtypes = [ctypes.c_void_p, _D, _D]
        L.ref_set_state.argtypes = [ctypes.c_void_p, _D, _D]
        L.ref_set_accel_field.argtypes = [ctypes.c_void_p, _D]
        L.ref_collide_node.argtypes = [ctypes.c_void_p, _D, _D, _D, _D, _D, _D, _D, _D]
        L.ref_velocities.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.ref_weights.argtypes = [ctypes.c_int, ctypes.c_double, _D]
        L.ref_matrix.argtypes = [ctypes.c_int, _D]
        L.ref_matrix_inverse.argtypes = [ctypes.c_int, _D]
        L.ref_feq.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, _D]
        L.ref_meq.argtypes = [ctypes.c_int, ctypes.c_double, _D, ctypes.c_double, _D]
        L.ref_forcing_moments.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, _D]
        L.ref_geq.argtypes = [ctypes.c_double, _D, ctypes.c_double, ctypes.c_double, _D]
        L.ref_neq.argtypes = [ctypes.c_double, _D, ctypes.c_double, ctypes.c_double, _D]
        L.ref_velocity.argtypes = [ctypes.c_int, _D, _D, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, _D]
        L.ref_total_force.argtypes = [_D, _D, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, _D]
        L.ref_threads.argtypes = []
        L.ref_threads.restype = ctypes.c_int
        L.ref_splitmix64.argtypes = [ctypes.c_uint64]
        L.ref_splitmix64.restype = ctypes.c_uint64
        L.ref_noise.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double]
        L.ref_noise.restype = ctypes.c_double
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _vec(x, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n
    return a


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


# ------------------------------------------------------------------ pieces
def velocities(q: int) -> np.ndarray:
    e = (ctypes.c_int * (3 * q))()
    _check(lib().ref_velocities(q, e), "velocities")
    return np.array(e, dtype=np.int64).reshape(3, q)


def weights(q: int, varpi: float = 0.5) -> np.ndarray:
    w = np.zeros(q)
    _check(lib().ref_weights(q, varpi, _ptr(w)), "weights")
    return w


def matrix(q: int) -> np.ndarray:
    m = np.zeros(q * q)
    _check(lib().ref_matrix(q, _ptr(m)), "matrix")
    return m.reshape(q, q)


def matrix_inverse(q: int) -> np.ndarray:
    m = np.zeros(q * q)
    _check(lib().ref_matrix_inverse(q, _ptr(m)), "matrix_inverse")
    return m.reshape(q, q)


def feq(q, rho, u, phi):
    out = np.zeros(q)
    _check(lib().ref_feq(q, rho, _ptr(_vec(u, 3)), phi, _ptr(out)), "feq")
    return out


def meq(q, rho, u, phi):
    out = np.zeros(q)
    _check(lib().ref_meq(q, rho, _ptr(_vec(u, 3)), phi, _ptr(out)), "meq")
    return out


def forcing_moments(q, u, F, phi):
    out = np.zeros(q)
    _check(lib().ref_forcing_moments(q, _ptr(_vec(u, 3)), _ptr(_vec(F, 3)), phi, _ptr(out)),
           "forcing_moments")
    return out


def geq(T, u, sigma=1.0, varpi=0.5):
    out = np.zeros(7)
    _check(lib().ref_geq(T, _ptr(_vec(u, 3)), sigma, varpi, _ptr(out)), "geq")
    return out


def neq(T, u, sigma=1.0, varpi=0.5):
    out = np.zeros(7)
    _check(lib().ref_neq(T, _ptr(_vec(u, 3)), sigma, varpi, _ptr(out)), "neq")
    return out


def velocity(q, f, G, phi, nu, K, F_phi):
    out = np.zeros(3)
    _check(lib().ref_velocity(q, _ptr(_vec(f, q)), _ptr(_vec(G, 3)), phi, nu, K, F_phi,
                              _ptr(out)), "velocity")
    return out


def total_force(u, G, phi, nu, K, F_phi):
    out = np.zeros(3)
    _check(lib().ref_total_force(_ptr(_vec(u, 3)), _ptr(_vec(G, 3)), phi, nu, K, F_phi,
                                 _ptr(out)), "total_force")
    return out


def threads() -> int:
    return int(lib().ref_threads())


def splitmix64(state: int) -> int:
    return int(lib().ref_splitmix64(ctypes.c_uint64(state & 0xFFFFFFFFFFFFFFFF)))


def noise(seed: int, n: int, amp: float) -> float:
    return float(lib().ref_noise(seed, n, amp))


# ------------------------------------------------------------------ lattice
def params_from_workload(wl: dict) -> _Params:
    p = _Params()
    lib().ref_default_params(ctypes.byref(p))
    for key, val in wl.items():
        if key == "faces":
            for k, fc in enumerate(val):
                p.face[k].flow = FLOW[fc["flow"]]
                p.face[k].heat = HEAT[fc["heat"]]
                p.face[k].T_wall = float(fc.get("T_wall", 0.0))
                for a in range(3):
                    p.face[k].u_wall[a] = float(fc.get("u_wall", (0.0, 0.0, 0.0))[a])
        elif key in ("accel", "init_u"):
            arr = getattr(p, key)
            for a in range(3):
                arr[a] = float(val[a])
        elif key in ("name", "steps", "precision", "check_interval", "lattice"):
            continue
        else:
            if not hasattr(p, key):
                raise KeyError(f"unknown workload key {key!r}")
            setattr(p, key, val)
    if "lattice" in wl:
        p.q = int(wl["lattice"])
    return p


class Oracle:
    """One lattice of the oracle.  Arrays are shaped (nz, ny, nx) for fields and
    (q, nz, ny, nx) for populations."""

    def __init__(self, workload: dict):
        self.p = params_from_workload(workload)
        self.q = int(self.p.q)
        self.shape = (int(self.p.nz), int(self.p.ny), int(self.p.nx))
        self.n = self.shape[0] * self.shape[1] * self.shape[2]
        h = ctypes.c_void_p()
        _check(lib().ref_create(ctypes.byref(self.p), ctypes.byref(h)), "create")
        self._h = h

    def close(self):
        if self._h:
            lib().ref_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def time(self) -> int:
        return int(lib().ref_time(self._h))

    def derived(self) -> dict:
        d = _Derived()
        _check(lib().ref_get_derived(self._h, ctypes.byref(d)), "derived")
        return {k: getattr(d, k) for k, _ in _Derived._fields_}

    def step(self, n: int = 1):
        _check(lib().ref_step(self._h, int(n)), "step")

    def fields(self) -> dict:
        out = {k: np.zeros(self.shape) for k in ("rho", "ux", "uy", "uz", "T")}
        _check(lib().ref_fields(self._h, *(_ptr(out[k]) for k in ("rho", "ux", "uy", "uz", "T"))),
               "fields")
        return out

    def nusselt(self) -> np.ndarray:
        nu = np.zeros(6)
        _check(lib().ref_nusselt(self._h, _ptr(nu)), "nusselt")
        return nu

    def get_state(self):
        f = np.zeros((self.q,) + self.shape)
        g = np.zeros((7,) + self.shape)
        _check(lib().ref_get_state(self._h, _ptr(f), _ptr(g)), "get_state")
        return f, g

    def set_state(self, f=None, g=None):
        fa = np.ascontiguousarray(f, dtype=np.float64) if f is not None else None
        ga = np.ascontiguousarray(g, dtype=np.float64) if g is not None else None
        if fa is not None:
            assert fa.shape == (self.q,) + self.shape
        if ga is not None:
            assert ga.shape == (7,) + self.shape
        _check(lib().ref_set_state(self._h, _ptr(fa) if fa is not None else None,
                                   _ptr(ga) if ga is not None else None), "set_state")

    def set_accel_field(self, a):
        if a is None:
            _check(lib().ref_set_accel_field(self._h, None), "set_accel_field")
            return
        arr = np.ascontiguousarray(a, dtype=np.float64)
        assert arr.shape == (3,) + self.shape
        _check(lib().ref_set_accel_field(self._h, _ptr(arr)), "set_accel_field")

    def collide_node(self, f, g):
        fo = np.zeros(self.q)
        go = np.zeros(7)
        rho = np.zeros(1)
        u = np.zeros(3)
        T = np.zeros(1)
        F = np.zeros(3)
        _check(lib().ref_collide_node(self._h, _ptr(_vec(f, self.q)), _ptr(_vec(g, 7)),
                                      _ptr(fo), _ptr(go), _ptr(rho), _ptr(u), _ptr(T), _ptr(F)),
               "collide_node")
        return fo, go, {"rho": rho[0], "u": u, "T": T[0], "F": F}


# ---------------------------------------------------------------- enthalpy model (App. B)
class _EnthParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("varpi", ctypes.c_double), ("porosity", ctypes.c_double),
        ("c_pl", ctypes.c_double), ("c_ps", ctypes.c_double), ("matrix_heat", ctypes.c_double),
        ("latent", ctypes.c_double), ("T_solidus", ctypes.c_double), ("T_liquidus", ctypes.c_double),
        ("alpha_l", ctypes.c_double), ("alpha_s", ctypes.c_double),
        ("zeta_e", ctypes.c_double), ("zeta_nu", ctypes.c_double),
        ("heat", ctypes.c_int32 * 6), ("T_wall", ctypes.c_double * 6),
        ("T_init", ctypes.c_double),
    ]


def _enth_lib():
    L = lib()
    if not getattr(L, "_enth_ready", False):
        L.ref_enthalpy_create.argtypes = [ctypes.POINTER(_EnthParams), ctypes.POINTER(ctypes.c_void_p)]
        L.ref_enthalpy_destroy.argtypes = [ctypes.c_void_p]
        L.ref_enthalpy_destroy.restype = None
        L.ref_enthalpy_time.argtypes = [ctypes.c_void_p]
        L.ref_enthalpy_time.restype = ctypes.c_int64
        L.ref_enthalpy_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.ref_enthalpy_fields.argtypes = [ctypes.c_void_p, _D, _D, _D]
        L.ref_enthalpy_get_state.argtypes = [ctypes.c_void_p, _D]
        L.ref_enthalpy_set_state.argtypes = [ctypes.c_void_p, _D]
        L.ref_enthalpy_phase.argtypes = [ctypes.c_void_p, ctypes.c_double, _D, _D]
        L._enth_ready = True
    return L


def enthalpy_params_from_workload(wl: dict) -> _EnthParams:
    p = _EnthParams()
    p.nx, p.ny, p.nz = wl["nx"], wl["ny"], wl["nz"]
    for k in ("varpi", "porosity", "c_pl", "c_ps", "matrix_heat", "latent", "T_solidus", "T_liquidus",
              "alpha_l", "alpha_s", "zeta_e", "zeta_nu", "T_init"):
        setattr(p, k, float(wl[k]))
    for f, fc in enumerate(wl["faces"]):
        p.heat[f] = HEAT[fc["heat"]]
        p.T_wall[f] = float(fc.get("T_wall", 0.0))
    return p


class EnthalpyOracle:
    """The enthalpy-based D3Q7-MRT model of App. B with u = 0 (Sec. 4.3)."""

    def __init__(self, workload: dict):
        self._lib = _enth_lib()
        self.params = enthalpy_params_from_workload(workload)
        self.shape = (workload["nz"], workload["ny"], workload["nx"])
        self.n = workload["nx"] * workload["ny"] * workload["nz"]
        h = ctypes.c_void_p()
        _check(self._lib.ref_enthalpy_create(ctypes.byref(self.params), ctypes.byref(h)), "ref_enthalpy_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ref_enthalpy_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def time(self) -> int:
        return int(self._lib.ref_enthalpy_time(self._h))

    def step(self, n: int = 1):
        _check(self._lib.ref_enthalpy_step(self._h, int(n)), "ref_enthalpy_step")

    def fields(self) -> dict:
        out = {k: np.empty(self.shape) for k in ("T", "En", "fl")}
        _check(self._lib.ref_enthalpy_fields(self._h, _ptr(out["T"]), _ptr(out["En"]), _ptr(out["fl"])),
               "ref_enthalpy_fields")
        return out

    def get_state(self) -> np.ndarray:
        g = np.empty((7,) + self.shape)
        _check(self._lib.ref_enthalpy_get_state(self._h, _ptr(g)), "ref_enthalpy_get_state")
        return g

    def set_state(self, g):
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert g.shape == (7,) + self.shape
        _check(self._lib.ref_enthalpy_set_state(self._h, _ptr(g)), "ref_enthalpy_set_state")

    def phase(self, En: float):
        T = ctypes.c_double()
        fl = ctypes.c_double()
        _check(self._lib.ref_enthalpy_phase(self._h, float(En), ctypes.byref(T), ctypes.byref(fl)),
               "ref_enthalpy_phase")
        return T.value, fl.value
