"""ctypes binding of ``liblbm.so`` (the C ABI in include/lbm.h).

Argument marshalling only: every step of the time loop, the fields, the
Nusselt numbers, the residual and the totals are computed by the HIP kernels
behind the C ABI.  PyTorch provides device memory and the stream.  There is no
CPU fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime that liblbm.so then shares

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()' "
        "or python paper_1611_03329_amd/build.py)")

_lib = ctypes.CDLL(LIB_PATH)

FP64 = 0
FP32 = 1
FP16_STORAGE = 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16_STORAGE}
ENERGY = {"temperature": 0, "enthalpy": 1}
FLOW = {"periodic": 0, "wall": 1, "outlet": 3}
HEAT = {"periodic": 0, "adiabatic": 1, "isothermal": 2, "outflow": 3}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "device error",
          4: "unstable", 5: "unsupported"}


class LBMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class UnstableError(LBMError):
    pass


class Face(ctypes.Structure):
    _fields_ = [("flow", ctypes.c_int32), ("heat", ctypes.c_int32),
                ("T_wall", ctypes.c_double), ("u_wall", ctypes.c_double * 3)]


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("lattice", ctypes.c_int32), ("precision", ctypes.c_int32),
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
        ("face", Face * 6),
        ("init_axis", ctypes.c_int32),
        ("init_T_lo", ctypes.c_double), ("init_T_hi", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("noise_amp", ctypes.c_double),
        ("check_interval", ctypes.c_int32),
        ("init_u", ctypes.c_double * 3),
        ("energy", ctypes.c_int32),
        ("c_pl", ctypes.c_double), ("c_ps", ctypes.c_double), ("matrix_heat", ctypes.c_double),
        ("latent", ctypes.c_double), ("T_solidus", ctypes.c_double), ("T_liquidus", ctypes.c_double),
        ("alpha_l", ctypes.c_double), ("alpha_s", ctypes.c_double), ("T_init", ctypes.c_double),
    ]


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("group_bytes", ctypes.c_uint64),
                ("xcd_ranges", ctypes.c_int32)]


class Derived(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("L", "s_nu", "zeta_alpha", "nu_e", "nu", "alpha_e", "alpha", "K",
                 "F_phi", "gbeta", "l0", "l1")]


_P = ctypes.POINTER(Params)
_V = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)

_lib.lbm_default_params.argtypes = [_P]
_lib.lbm_default_params.restype = None
_lib.lbm_required_bytes.argtypes = [_P, ctypes.POINTER(ctypes.c_size_t)]
_lib.lbm_create.argtypes = [_P, _V, ctypes.c_size_t, _V, ctypes.POINTER(_V)]
_lib.lbm_destroy.argtypes = [_V]
_lib.lbm_set_stream.argtypes = [_V, _V]
_lib.lbm_step.argtypes = [_V, ctypes.c_int64]
_lib.lbm_time.argtypes = [_V, _I64]
_lib.lbm_derived_params.argtypes = [_V, ctypes.POINTER(Derived)]
_lib.lbm_fields.argtypes = [_V, _V, _V, _V, _V, _V]
_lib.lbm_fields_noalloc.argtypes = [_V, _V, _V, _V, _V, _V]
_lib.lbm_enthalpy_fields.argtypes = [_V, _V, _V, _V]
_lib.lbm_nusselt.argtypes = [_V, _D]
_lib.lbm_nusselt_start.argtypes = [_V]
_lib.lbm_residual.argtypes = [_V, _D, _I64]
_lib.lbm_totals.argtypes = [_V, _D, _D]
_lib.lbm_get_state.argtypes = [_V, _V, _V]
_lib.lbm_set_state.argtypes = [_V, _V, _V]
_lib.lbm_status_string.argtypes = [ctypes.c_int]
_lib.lbm_status_string.restype = ctypes.c_char_p
_lib.lbm_last_error.argtypes = []
_lib.lbm_last_error.restype = ctypes.c_char_p
_lib.lbm_transfer_state.argtypes = [_V, _V]
_lib.lbm_batch_create.argtypes = [_V, ctypes.c_int32, ctypes.POINTER(_V)]
_lib.lbm_batch_destroy.argtypes = [_V]
_lib.lbm_batch_add.argtypes = [_V, _V]
_lib.lbm_batch_remove.argtypes = [_V, _V]
_lib.lbm_batch_size.argtypes = [_V, ctypes.POINTER(ctypes.c_int32)]
_lib.lbm_batch_member.argtypes = [_V, ctypes.c_int32, ctypes.POINTER(_V)]
_lib.lbm_batch_step.argtypes = [_V, ctypes.c_int64]
_lib.lbm_batch_residuals.argtypes = [_V, _D, _I64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]
_lib.lbm_batch_set_launch.argtypes = [_V, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32]
_lib.lbm_batch_autotune.argtypes = [_V, ctypes.POINTER(Launch)]
_lib.lbm_batch_set_graph.argtypes = [_V, ctypes.c_int32]
_lib.lbm_batch_set_span.argtypes = [_V, ctypes.c_int32]
_lib.lbm_batch_set_class_block.argtypes = [_V, ctypes.c_int32, ctypes.c_int32]
_lib.lbm_batch_class_block.argtypes = [_V, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
for _name in ("lbm_required_bytes", "lbm_create", "lbm_destroy", "lbm_set_stream", "lbm_step",
              "lbm_time", "lbm_derived_params", "lbm_fields", "lbm_fields_noalloc", "lbm_nusselt", "lbm_nusselt_start", "lbm_residual",
              "lbm_totals", "lbm_get_state", "lbm_set_state", "lbm_transfer_state", "lbm_enthalpy_fields", "lbm_batch_create", "lbm_batch_destroy",
              "lbm_batch_add", "lbm_batch_remove", "lbm_batch_size", "lbm_batch_member", "lbm_batch_step",
              "lbm_batch_residuals", "lbm_batch_set_launch", "lbm_batch_autotune", "lbm_batch_set_graph",
              "lbm_batch_set_span", "lbm_batch_set_class_block", "lbm_batch_class_block"):
    getattr(_lib, _name).restype = ctypes.c_int


def library() -> ctypes.CDLL:
    return _lib


def _check(status: int):
    if status != 0:
        msg = _lib.lbm_last_error().decode(errors="replace")
        cls = UnstableError if status == 4 else LBMError
        raise cls(status, msg)


_SKIP_KEYS = {"name", "steps", "q"}


def make_params(workload: dict, precision: str | int = "fp64", check_interval: int | None = None) -> Params:
    """Fills the C parameter struct from a plain workload dict (lbm_inputs)."""
    p = Params()
    _lib.lbm_default_params(ctypes.byref(p))
    for key, val in workload.items():
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
        elif key == "precision":
            continue
        elif key == "energy":
            p.energy = ENERGY[val] if isinstance(val, str) else int(val)
        elif key in _SKIP_KEYS:
            continue
        else:
            if not hasattr(p, key):
                raise KeyError(f"unknown workload key {key!r}")
            setattr(p, key, val)
    p.lattice = int(workload.get("lattice", workload.get("q", 19)))
    prec = workload.get("precision", precision) if precision is None else precision
    p.precision = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    if check_interval is not None:
        p.check_interval = int(check_interval)
    return p


def required_bytes(params: Params) -> int:
    n = ctypes.c_size_t()
    _check(_lib.lbm_required_bytes(ctypes.byref(params), ctypes.byref(n)))
    return int(n.value)


def _ptr(t) -> ctypes.c_void_p | None:
    """Address of an FP64 buffer: a contiguous CUDA tensor (device memory) or
    a C-contiguous numpy array (host memory, which the library stages)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.dtype == np.float64 and t.flags["C_CONTIGUOUS"]
        return ctypes.c_void_p(t.ctypes.data)
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One lattice on the current CUDA (HIP) device.  Device memory is a torch
    uint8 tensor owned by this object; all work runs on ``stream``."""

    def __init__(self, workload: dict, precision: str = "fp64", check_interval: int = 0,
                 stream: torch.cuda.Stream | None = None, device=None):
        self.params = make_params(workload, precision, check_interval)
        self.enthalpy = int(self.params.energy) == ENERGY["enthalpy"]
        self.q = 0 if self.enthalpy else int(self.params.lattice)
        self.shape = (int(self.params.nz), int(self.params.ny), int(self.params.nx))
        self.nodes = self.shape[0] * self.shape[1] * self.shape[2]
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.nbytes = required_bytes(self.params)
        self.buf = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.buf.data_ptr()
        self._base = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _check(_lib.lbm_create(ctypes.byref(self.params), ctypes.c_void_p(self._base),
                               ctypes.c_size_t(self.nbytes), ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(h)))
        self._h = h
        self.batch = None

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            if self.batch is not None:
                self.batch.remove(self)
            _check(_lib.lbm_destroy(self._h))
            self._h = None

    def _settle(self):
        """Outputs were written on this lattice's stream: make them safe to use
        on the caller's current stream."""
        if self.stream.cuda_stream != torch.cuda.current_stream(self.device).cuda_stream:
            self.stream.synchronize()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- stepping
    def step(self, n: int = 1):
        _check(_lib.lbm_step(self._h, int(n)))

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        _check(_lib.lbm_time(self._h, ctypes.byref(t)))
        return int(t.value)

    def derived(self) -> dict:
        d = Derived()
        _check(_lib.lbm_derived_params(self._h, ctypes.byref(d)))
        return {k: getattr(d, k) for k, _ in Derived._fields_}

    # -- outputs
    def fields(self, host: bool = False) -> dict:
        """rho, ux, uy, uz, T: FP64 device tensors, or numpy arrays written by
        the library through host pointers (host=True)."""
        keys = ("rho", "ux", "uy", "uz", "T")
        if host:
            out = {k: np.empty(self.shape, dtype=np.float64) for k in keys}
        else:
            out = {k: torch.empty(self.shape, dtype=torch.float64, device=self.device) for k in keys}
        _check(_lib.lbm_fields(self._h, *(_ptr(out[k]) for k in keys)))
        if not host:
            self._settle()
        return out

    def nusselt(self):
        nu = (ctypes.c_double * 6)()
        _check(_lib.lbm_nusselt(self._h, nu))
        return [float(v) for v in nu]

    def nusselt_start(self):
        """Starts the Nusselt reduction of the current state without waiting;
        the next nusselt() collects it."""
        _check(_lib.lbm_nusselt_start(self._h))

    def residual(self):
        r = ctypes.c_double()
        at = ctypes.c_int64()
        _check(_lib.lbm_residual(self._h, ctypes.byref(r), ctypes.byref(at)))
        return float(r.value), int(at.value)

    def totals(self):
        m = ctypes.c_double()
        q = ctypes.c_double()
        _check(_lib.lbm_totals(self._h, ctypes.byref(m), ctypes.byref(q)))
        return float(m.value), float(q.value)

    def get_state(self, host: bool = False):
        """(f, g) pre-collision populations, FP64 device tensors (numpy arrays
        through host pointers with host=True); f is None for an enthalpy
        lattice."""
        if host:
            f = None if self.enthalpy else np.empty((self.q,) + self.shape, dtype=np.float64)
            g = np.empty((7,) + self.shape, dtype=np.float64)
        else:
            f = None if self.enthalpy else torch.empty((self.q,) + self.shape, dtype=torch.float64,
                                                       device=self.device)
            g = torch.empty((7,) + self.shape, dtype=torch.float64, device=self.device)
        _check(_lib.lbm_get_state(self._h, _ptr(f), _ptr(g)))
        if not host:
            self._settle()
        return f, g

    def enthalpy_fields(self, host: bool = False) -> dict:
        """T, En and f_l (Eqs. B7-B9) of an enthalpy lattice (numpy arrays
        through host pointers with host=True)."""
        keys = ("T", "En", "fl")
        if host:
            out = {k: np.empty(self.shape, dtype=np.float64) for k in keys}
        else:
            out = {k: torch.empty(self.shape, dtype=torch.float64, device=self.device) for k in keys}
        _check(_lib.lbm_enthalpy_fields(self._h, *(_ptr(out[k]) for k in keys)))
        if not host:
            self._settle()
        return out

    def transfer_from(self, other: "Lattice"):
        """Takes over the state of ``other`` (same lattice type, shape and rest
        state), converting its storage precision."""
        _check(_lib.lbm_transfer_state(self._h, other._h))

    def set_state(self, f, g):
        """Replaces the state (f must be None for an enthalpy lattice).  numpy
        arrays are passed as host memory (the library stages them); anything
        else is moved to the device first."""
        def arr(a, lead):
            if isinstance(a, np.ndarray):
                a = np.ascontiguousarray(a, dtype=np.float64)
            else:
                a = torch.as_tensor(a, dtype=torch.float64).to(self.device).contiguous()
            assert tuple(a.shape) == (lead,) + self.shape
            return a
        g = arr(g, 7)
        if f is not None:
            f = arr(f, self.q)
        _check(_lib.lbm_set_state(self._h, _ptr(f), _ptr(g)))
        # keep the inputs alive until the copy kernel has run
        self.stream.synchronize()


class Batch:
    """Many lattices advanced by one launch per time step (lbm_batch_* of the C
    ABI).  Members must share lattice type and precision; they move to the
    batch's stream.  ``graph=True`` replays whole check intervals from a HIP
    graph, which needs a stream of its own: one is created when none is given."""

    def __init__(self, check_interval: int, stream: torch.cuda.Stream | None = None, graph: bool = False,
                 block: int | None = None, per_cu: int = 0, group_bytes: int = 0, xcd_ranges: int = 0,
                 span: bool = False, device=None):
        self.device = torch.device("cuda") if device is None else torch.device(device)
        if stream is None:
            stream = torch.cuda.Stream(self.device) if graph else torch.cuda.current_stream(self.device)
        self.stream = stream
        self.check_interval = int(check_interval)
        h = ctypes.c_void_p()
        _check(_lib.lbm_batch_create(ctypes.c_void_p(stream.cuda_stream), self.check_interval, ctypes.byref(h)))
        self._h = h
        self.members: list[Lattice] = []
        if block is not None or per_cu or group_bytes or xcd_ranges:
            self.set_launch(256 if block is None else block, per_cu, group_bytes, xcd_ranges)
        if graph:
            _check(_lib.lbm_batch_set_graph(self._h, 1))
        if span:
            self.set_span(True)

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.lbm_batch_destroy(self._h))
            for m in self.members:
                m.batch = None
            self.members = []
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

    def __len__(self) -> int:
        return len(self.members)

    def add(self, lat: Lattice):
        _check(_lib.lbm_batch_add(self._h, lat._h))
        lat.stream = self.stream
        lat.batch = self
        self.members.append(lat)

    def remove(self, lat: Lattice):
        _check(_lib.lbm_batch_remove(self._h, lat._h))
        lat.batch = None
        self.members.remove(lat)

    def step(self, n: int = 1):
        _check(_lib.lbm_batch_step(self._h, int(n)))

    def set_span(self, on: bool):
        """Residual over the whole check interval (True) or over one step."""
        _check(_lib.lbm_batch_set_span(self._h, int(bool(on))))

    def set_launch(self, block: int, per_cu: int = 0, group_bytes: int = 0, xcd_ranges: int = 0):
        """Threads per tile, resident blocks per compute unit (0: one block per
        tile), the group size limit in bytes (0: no limit) and the number of
        contiguous per-XCD tile ranges (0: hardware order)."""
        _check(_lib.lbm_batch_set_launch(self._h, int(block), int(per_cu), int(group_bytes), int(xcd_ranges)))

    def autotune(self):
        """Times launch shapes over real check intervals; returns the chosen
        (block, per_cu, group_bytes, xcd_ranges)."""
        c = Launch()
        _check(_lib.lbm_batch_autotune(self._h, ctypes.byref(c)))
        return int(c.block), int(c.blocks_per_cu), int(c.group_bytes), int(c.xcd_ranges)

    def set_class_block(self, size_class: int, block: int):
        """Threads per tile for members of 2^size_class .. 2^(size_class+1) - 1
        nodes (0: the batch-wide block)."""
        _check(_lib.lbm_batch_set_class_block(self._h, int(size_class), int(block)))

    def class_blocks(self) -> dict:
        """Threads per tile of every size class whose choice differs from the
        batch-wide block, {size_class: block}."""
        base = ctypes.c_int32()
        out = {}
        for k in range(32):
            _check(_lib.lbm_batch_class_block(self._h, k, ctypes.byref(base)))
            out[k] = int(base.value)
        default = max(set(out.values()), key=list(out.values()).count)
        return {k: v for k, v in out.items() if v != default}

    def residuals(self):
        """(r, at_step, unstable) lists in member order."""
        n = len(self.members)
        r = (ctypes.c_double * max(n, 1))()
        at = (ctypes.c_int64 * max(n, 1))()
        un = (ctypes.c_int32 * max(n, 1))()
        _check(_lib.lbm_batch_residuals(self._h, r, at, un, n))
        return [float(v) for v in r[:n]], [int(v) for v in at[:n]], [bool(v) for v in un[:n]]
