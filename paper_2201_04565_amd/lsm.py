"""Python binding of liblsm.so (argument marshalling only).

Every step of the lattice spring model runs in the library's HIP kernels;
PyTorch only provides the device workspace (a uint8 CUDA tensor) and the
HIP stream the library is bound to.  There is no CPU fallback: if the
library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsm.so")

LSM_OK, LSM_EINVAL, LSM_ENOMEM, LSM_EHIP, LSM_EUNSTABLE, LSM_ESTATE = 0, -1, -2, -3, -4, -5
TRI2D, SC3D = 0, 1
FP64, FP32_KAHAN = 0, 1
PRED_AFFINE, PRED_GRIPS_ONLY = 0, 1
KERNEL_AUTO, KERNEL_GATHER, KERNEL_SWEEP, KERNEL_SWEEP2, KERNEL_SMALL, KERNEL_COMPACT = 0, 1, 2, 3, 4, 5
KERNEL_COMPACT_DIRECT = 6
MAX_PHASES = 8

EXPORTS = (
    "lsm_create", "lsm_destroy", "lsm_build_lattice", "lsm_counts", "lsm_workspace_bytes",
    "lsm_bind", "lsm_apply_strain_increment", "lsm_relax", "lsm_read_state", "lsm_read_broken",
    "lsm_n_broken", "lsm_get_springs", "lsm_get_reference", "lsm_get_positions",
    "lsm_get_velocities", "lsm_set_positions", "lsm_set_velocities", "lsm_eval_forces",
    "lsm_save_state", "lsm_load_state", "lsm_set_timing", "lsm_read_timing", "lsm_step_bytes",
    "lsm_set_launch", "lsm_set_prefetch", "lsm_autotune", "lsm_get_launch", "lsm_last_error",
    "lsm_strerror", "lsm_set_strain_rate", "lsm_relax_trace", "lsm_local_fields",
)


class Config(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nphase", C.c_int32), ("a", C.c_double),
                ("k", C.c_double * 64), ("break_stretch", C.c_double * 64),
                ("k_face", C.c_double), ("k_diag", C.c_double), ("mass", C.c_double * 8),
                ("dt", C.c_double), ("damping", C.c_double), ("precision", C.c_int32),
                ("predictor", C.c_int32), ("void_value", C.c_int32), ("spring_law", C.c_int32),
                ("law_c", C.c_double)]


class Record(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double * 9), ("ke", C.c_double),
                ("pe", C.c_double), ("n_broken", C.c_int64), ("increment", C.c_int32),
                ("step", C.c_int32), ("status", C.c_int32), ("reserved", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("variant", C.c_int32), ("rows_per_wave", C.c_int32), ("prefetch", C.c_int32),
                ("steps_per_launch", C.c_int32), ("us_per_step", C.c_double)]


class Event(C.Structure):
    _fields_ = [("increment", C.c_int32), ("step", C.c_int32), ("spring_id", C.c_int64),
                ("margin", C.c_double)]


EVENT_DTYPE = np.dtype([("inc", np.int32), ("step", np.int32), ("id", np.int64),
                        ("margin", np.float64)])

_lib = None


class LsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def load_library():
    """Loads liblsm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    P = C.POINTER
    L.lsm_create.argtypes = [P(Config), P(vp)]
    L.lsm_destroy.argtypes = [vp]
    L.lsm_destroy.restype = None
    L.lsm_build_lattice.argtypes = [vp, vp, i64, i64, i64]
    L.lsm_counts.argtypes = [vp, P(i64), P(i64)]
    L.lsm_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.lsm_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.lsm_apply_strain_increment.argtypes = [vp, dbl]
    L.lsm_relax.argtypes = [vp, i64]
    L.lsm_read_state.argtypes = [vp, P(Record)]
    L.lsm_set_strain_rate.argtypes = [vp, dbl]
    L.lsm_relax_trace.argtypes = [vp, i64, i64, vp, i64, P(i64)]
    L.lsm_read_broken.argtypes = [vp, i64, i64, vp, P(i64)]
    L.lsm_n_broken.argtypes = [vp, P(i64)]
    L.lsm_get_springs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    for nm in ("lsm_get_reference", "lsm_get_positions", "lsm_get_velocities",
               "lsm_set_positions", "lsm_set_velocities"):
        getattr(L, nm).argtypes = [vp, vp]
    L.lsm_eval_forces.argtypes = [vp, vp, C.c_int]
    L.lsm_local_fields.argtypes = [vp, C.c_int, vp, vp]
    L.lsm_save_state.argtypes = [vp, vp, P(C.c_size_t)]
    L.lsm_load_state.argtypes = [vp, vp, C.c_size_t]
    L.lsm_set_timing.argtypes = [vp, C.c_int]
    L.lsm_read_timing.argtypes = [vp, P(dbl), P(i64)]
    L.lsm_step_bytes.argtypes = [vp, P(i64)]
    L.lsm_set_launch.argtypes = [vp, C.c_int, C.c_int]
    L.lsm_set_prefetch.argtypes = [vp, C.c_int]
    L.lsm_autotune.argtypes = [vp, C.c_int, vp, C.c_int, P(C.c_int)]
    L.lsm_get_launch.argtypes = [vp, P(Tuning)]
    L.lsm_last_error.argtypes = [vp]
    L.lsm_last_error.restype = C.c_char_p
    L.lsm_strerror.argtypes = [C.c_int]
    L.lsm_strerror.restype = C.c_char_p
    _lib = L
    return L


SPRING_LAWS = {"linear": 0, "recover": 1, "cubic": 2}


def make_config(*, lattice, k, s, mass, a=1.0, k_face=1.0, k_diag=1.0, dt=0.01, gamma=0.1,
                precision="fp64", predictor="affine", void_value=-1, spring_law="linear",
                law_c=0.0) -> Config:
    P = len(mass)
    if not 1 <= P <= MAX_PHASES:
        raise ValueError("1..8 phases supported")
    cfg = Config()
    cfg.lattice = lattice
    cfg.nphase = P
    cfg.a = a
    kk = np.asarray(k, dtype=np.float64).reshape(P, P)
    ss = np.asarray(s, dtype=np.float64).reshape(P, P)
    for i in range(64):
        cfg.k[i] = math.nan
        cfg.break_stretch[i] = math.nan
    for i in range(P):
        for j in range(P):
            cfg.k[i * P + j] = kk[i, j]
            cfg.break_stretch[i * P + j] = ss[i, j]
    cfg.k_face, cfg.k_diag = k_face, k_diag
    for i in range(P):
        cfg.mass[i] = mass[i]
    cfg.dt, cfg.damping = dt, gamma
    cfg.precision = {"fp64": FP64, "fp32k": FP32_KAHAN}[precision]
    cfg.predictor = {"affine": PRED_AFFINE, "grips": PRED_GRIPS_ONLY}[predictor]
    cfg.void_value = void_value
    cfg.spring_law = SPRING_LAWS[spring_law]
    cfg.law_c = law_c
    return cfg


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _record_dict(R) -> dict:
    return dict(eps=R.eps, sigma=np.array(R.sigma[:]).reshape(3, 3), ke=R.ke, pe=R.pe,
                n_broken=R.n_broken, inc=R.increment, step=R.step, status=R.status)


class Lattice:
    """A lattice specimen bound to GPU memory and a HIP stream."""

    def __init__(self, image: np.ndarray, *, k, s, mass, a=1.0, k_face=1.0, k_diag=1.0,
                 dt=0.01, gamma=0.1, precision="fp64", predictor="affine", void_value=-1,
                 spring_law="linear", law_c=0.0, device="cuda:0", stream=None):
        import torch

        L = load_library()
        self._L = L
        img = np.ascontiguousarray(image, dtype=np.uint8)
        lattice = TRI2D if img.ndim == 2 else SC3D
        self.dim = 2 if lattice == TRI2D else 3
        cfg = make_config(lattice=lattice, k=k, s=s, mass=mass, a=a, k_face=k_face,
                          k_diag=k_diag, dt=dt, gamma=gamma, precision=precision,
                          predictor=predictor, void_value=void_value, spring_law=spring_law,
                          law_c=law_c)
        self.precision = precision
        h = C.c_void_p()
        self._check(L.lsm_create(C.byref(cfg), C.byref(h)), None)
        self._h = h
        if img.ndim == 2:
            ny, nx = img.shape
            nz = 1
        else:
            nz, ny, nx = img.shape
        self.shape = (nx, ny, nz)
        self._check(L.lsm_build_lattice(h, _ptr(img), nx, ny, nz))
        n, m = C.c_int64(), C.c_int64()
        self._check(L.lsm_counts(h, C.byref(n), C.byref(m)))
        self.n, self.m = n.value, m.value
        nb = C.c_size_t()
        self._check(L.lsm_workspace_bytes(h, C.byref(nb)))
        self.device = torch.device(device)
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._check(L.lsm_bind(h, C.c_void_p(self.workspace.data_ptr()), nb.value,
                               C.c_void_p(self.stream.cuda_stream)))

    @classmethod
    def from_workload(cls, wl: dict, image: np.ndarray, **over):
        kw = dict(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0),
                  k_face=wl.get("k_face", 1.0), k_diag=wl.get("k_diag", 1.0), dt=wl["dt"],
                  gamma=wl["gamma"], precision=wl.get("precision", "fp64"),
                  void_value=wl.get("void_value", -1))
        kw.update(over)
        return cls(image, **kw)

    # ----------------------------------------------------------- plumbing
    def _check(self, rc, h=0):
        if rc == LSM_OK:
            return rc
        hh = self._h if h == 0 else h
        msg = self._L.lsm_last_error(hh).decode() if hh else ""
        raise LsmError(rc, f"{self._L.lsm_strerror(rc).decode()}: {msg}")

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._L.lsm_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ protocol
    def apply_strain_increment(self, d_eps: float):
        self._check(self._L.lsm_apply_strain_increment(self._h, float(d_eps)))

    apply_increment = apply_strain_increment

    def relax(self, nsteps: int):
        self._check(self._L.lsm_relax(self._h, int(nsteps)))

    def read_state(self, allow_unstable=False) -> dict:
        R = Record()
        rc = self._L.lsm_read_state(self._h, C.byref(R))
        if rc != LSM_OK and not (allow_unstable and rc == LSM_EUNSTABLE):
            self._check(rc)
        return _record_dict(R)

    def set_strain_rate(self, rate: float):
        """Constant strain-rate loading (per unit time) from the next step."""
        self._check(self._L.lsm_set_strain_rate(self._h, float(rate)))

    def relax_trace(self, rate, nsteps: int, every: int) -> list:
        """The paper's protocol: grips at a constant strain rate for nsteps,
        a record (strain, stress, energies) after every `every` steps."""
        self.set_strain_rate(rate)
        cap = -(-int(nsteps) // int(every))
        buf = (Record * cap)()
        n = C.c_int64()
        self._check(self._L.lsm_relax_trace(self._h, int(nsteps), int(every), buf, cap, C.byref(n)))
        return [_record_dict(buf[i]) for i in range(n.value)]

    def read_broken(self) -> np.ndarray:
        n = C.c_int64()
        self._check(self._L.lsm_n_broken(self._h, C.byref(n)))
        buf = (Event * max(n.value, 1))()
        got = C.c_int64()
        self._check(self._L.lsm_read_broken(self._h, 0, n.value, buf, C.byref(got)))
        ev = np.zeros(got.value, dtype=EVENT_DTYPE)
        for i in range(got.value):
            e = buf[i]
            ev[i] = (e.increment, e.step, e.spring_id, e.margin)
        return ev

    def n_broken(self) -> int:
        n = C.c_int64()
        self._check(self._L.lsm_n_broken(self._h, C.byref(n)))
        return n.value

    # --------------------------------------------------------------- state
    def springs(self) -> dict:
        m = self.m
        p = np.zeros(m, np.int64)
        q = np.zeros(m, np.int64)
        k = np.zeros(m)
        r0 = np.zeros(m)
        rc = np.zeros(m)
        br = np.zeros(m, np.uint8)
        self._check(self._L.lsm_get_springs(self._h, _ptr(p), _ptr(q), _ptr(k), _ptr(r0),
                                            _ptr(rc), _ptr(br)))
        return dict(p=p, q=q, k=k, r0=r0, rc=rc, broken=br)

    def _getter(self, fn):
        out = np.zeros((self.n, self.dim))
        self._check(fn(self._h, _ptr(out)))
        return out

    @property
    def X0(self):
        return self._getter(self._L.lsm_get_reference)

    @property
    def x(self):
        return self._getter(self._L.lsm_get_positions)

    @x.setter
    def x(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(self.n, self.dim)
        self._check(self._L.lsm_set_positions(self._h, _ptr(val)))

    @property
    def v(self):
        return self._getter(self._L.lsm_get_velocities)

    @v.setter
    def v(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(self.n, self.dim)
        self._check(self._L.lsm_set_velocities(self._h, _ptr(val)))

    def eval_forces(self, commit=False) -> np.ndarray:
        out = np.zeros((self.n, self.dim))
        self._check(self._L.lsm_eval_forces(self._h, _ptr(out), int(bool(commit))))
        return out

    def local_fields(self, radius=0):
        """(stress, strain) per particle, numpy [n, dim, dim] (lsm_local_fields
        into device tensors on the lattice's stream, then copied)."""
        import torch
        d = self.n * self.dim * self.dim
        stress = torch.empty(max(d, 1), dtype=torch.float64, device=self.device)
        strain = torch.empty(max(d, 1), dtype=torch.float64, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        self._check(self._L.lsm_local_fields(self._h, int(radius), C.c_void_p(stress.data_ptr()),
                                             C.c_void_p(strain.data_ptr())))
        self.synchronize()
        shape = (self.n, self.dim, self.dim)
        return stress[:d].cpu().numpy().reshape(shape), strain[:d].cpu().numpy().reshape(shape)

    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._check(self._L.lsm_save_state(self._h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(self._L.lsm_save_state(self._h, buf, C.byref(n)))
        return buf.raw[:n.value]

    def load_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self._L.lsm_load_state(self._h, buf, len(blob)))

    # --------------------------------------------------------- measurement
    def set_timing(self, on: bool):
        self._check(self._L.lsm_set_timing(self._h, int(bool(on))))

    def read_timing(self):
        ms, steps = C.c_double(), C.c_int64()
        self._check(self._L.lsm_read_timing(self._h, C.byref(ms), C.byref(steps)))
        return ms.value, steps.value

    def step_bytes(self) -> int:
        b = C.c_int64()
        self._check(self._L.lsm_step_bytes(self._h, C.byref(b)))
        return b.value

    def set_launch(self, variant="auto", rows_per_wave=0):
        v = {"auto": KERNEL_AUTO, "gather": KERNEL_GATHER, "sweep": KERNEL_SWEEP,
             "sweep2": KERNEL_SWEEP2, "small": KERNEL_SMALL, "compact": KERNEL_COMPACT,
             "compact_direct": KERNEL_COMPACT_DIRECT}[variant]
        self._check(self._L.lsm_set_launch(self._h, v, int(rows_per_wave)))

    def set_prefetch(self, rows_ahead):
        self._check(self._L.lsm_set_prefetch(self._h, int(rows_ahead)))

    def autotune(self, steps_per_trial=100):
        """Times the candidate launches on the lattice at rest and keeps the
        fastest; returns [(variant, rows_per_wave, prefetch, us_per_step)]."""
        buf = (Tuning * 64)()
        n = C.c_int()
        self._check(self._L.lsm_autotune(self._h, int(steps_per_trial), buf, 64, C.byref(n)))
        names = {KERNEL_GATHER: "gather", KERNEL_SWEEP: "sweep", KERNEL_SWEEP2: "sweep2",
                 KERNEL_SMALL: "small", KERNEL_COMPACT: "compact",
                 KERNEL_COMPACT_DIRECT: "compact_direct"}
        return [(names.get(t.variant, "auto"), t.rows_per_wave, t.prefetch, t.us_per_step)
                for t in buf[:n.value]]

    def launch(self):
        t = Tuning()
        self._check(self._L.lsm_get_launch(self._h, C.byref(t)))
        names = {KERNEL_AUTO: "auto", KERNEL_GATHER: "gather", KERNEL_SWEEP: "sweep",
                 KERNEL_SWEEP2: "sweep2", KERNEL_SMALL: "small", KERNEL_COMPACT: "compact",
                 KERNEL_COMPACT_DIRECT: "compact_direct"}
        return dict(variant=names[t.variant], rows_per_wave=t.rows_per_wave, prefetch=t.prefetch,
                    steps_per_launch=t.steps_per_launch)

    def synchronize(self):
        self.stream.synchronize()


class HostModel:
    """Host-only view of a built lattice (no device memory, no GPU calls):
    counts, canonical spring list and reference positions."""

    def __init__(self, image: np.ndarray, *, k, s, mass, a=1.0, k_face=1.0, k_diag=1.0,
                 dt=0.01, gamma=0.1, precision="fp64", predictor="affine", void_value=-1,
                 spring_law="linear", law_c=0.0):
        L = load_library()
        self._L = L
        img = np.ascontiguousarray(image, dtype=np.uint8)
        lattice = TRI2D if img.ndim == 2 else SC3D
        self.dim = 2 if lattice == TRI2D else 3
        cfg = make_config(lattice=lattice, k=k, s=s, mass=mass, a=a, k_face=k_face,
                          k_diag=k_diag, dt=dt, gamma=gamma, precision=precision,
                          predictor=predictor, void_value=void_value, spring_law=spring_law,
                          law_c=law_c)
        h = C.c_void_p()
        rc = L.lsm_create(C.byref(cfg), C.byref(h))
        if rc != LSM_OK:
            raise LsmError(rc, L.lsm_strerror(rc).decode())
        self._h = h
        nz, ny, nx = (1,) + img.shape if img.ndim == 2 else img.shape
        rc = L.lsm_build_lattice(h, _ptr(img), nx, ny, nz)
        if rc != LSM_OK:
            msg = L.lsm_last_error(h).decode()
            L.lsm_destroy(h)
            self._h = None
            raise LsmError(rc, msg)
        n, m = C.c_int64(), C.c_int64()
        L.lsm_counts(h, C.byref(n), C.byref(m))
        self.n, self.m = n.value, m.value

    springs = Lattice.springs
    _check = Lattice._check
    _getter = Lattice._getter
    close = Lattice.close
    __del__ = Lattice.__del__

    @property
    def X0(self):
        return self._getter(self._L.lsm_get_reference)

    def workspace_bytes(self) -> int:
        nb = C.c_size_t()
        self._check(self._L.lsm_workspace_bytes(self._h, C.byref(nb)))
        return nb.value

    def set_launch(self, variant="auto", rows_per_wave=0):
        """Kernel variant whose bytes step_bytes reports (no device call)."""
        v = {"auto": KERNEL_AUTO, "gather": KERNEL_GATHER, "sweep": KERNEL_SWEEP,
             "sweep2": KERNEL_SWEEP2, "small": KERNEL_SMALL, "compact": KERNEL_COMPACT,
             "compact_direct": KERNEL_COMPACT_DIRECT}[variant]
        self._check(self._L.lsm_set_launch(self._h, v, int(rows_per_wave)))

    def step_bytes(self) -> int:
        b = C.c_int64()
        self._check(self._L.lsm_step_bytes(self._h, C.byref(b)))
        return b.value

    def launch_variant(self) -> str:
        """The kernel that would run the interior steps (no device call)."""
        t = Tuning()
        self._check(self._L.lsm_get_launch(self._h, C.byref(t)))
        names = {KERNEL_GATHER: "gather", KERNEL_SWEEP: "sweep", KERNEL_SWEEP2: "sweep2",
                 KERNEL_SMALL: "small", KERNEL_COMPACT: "compact", KERNEL_COMPACT_DIRECT: "compact_direct"}
        return names[t.variant]


BATCH_EXPORTS = (
    "lsm_batch_create", "lsm_batch_destroy", "lsm_batch_last_error", "lsm_batch_counts",
    "lsm_batch_workspace_bytes", "lsm_batch_bind", "lsm_batch_set_launch", "lsm_batch_run",
    "lsm_batch_read", "lsm_batch_set_timing", "lsm_batch_read_timing", "lsm_batch_autotune",
    "lsm_batch_get_launch",
)


class FailRule(C.Structure):
    _fields_ = [("drop_fraction", C.c_double)]


def _load_batch(L):
    if getattr(L, "_batch_ready", False):
        return L
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    P = C.POINTER
    L.lsm_batch_create.argtypes = [P(Config), i64, vp, vp, P(vp)]
    L.lsm_batch_destroy.argtypes = [vp]
    L.lsm_batch_destroy.restype = None
    L.lsm_batch_last_error.argtypes = [vp]
    L.lsm_batch_last_error.restype = C.c_char_p
    L.lsm_batch_counts.argtypes = [vp, P(i64), P(i64)]
    L.lsm_batch_workspace_bytes.argtypes = [vp, P(C.c_size_t)]
    L.lsm_batch_bind.argtypes = [vp, vp, C.c_size_t, vp]
    L.lsm_batch_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.lsm_batch_get_launch.argtypes = [vp, C.POINTER(Tuning)]
    L.lsm_batch_autotune.argtypes = [vp, C.c_int, vp, C.c_int, P(C.c_int)]
    L.lsm_batch_run.argtypes = [vp, dbl, i64, i32, P(FailRule)]
    L.lsm_batch_read.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.lsm_batch_set_timing.argtypes = [vp, C.c_int]
    L.lsm_batch_read_timing.argtypes = [vp, P(dbl), P(i64), P(dbl)]
    L._batch_ready = True
    return L


class Batch:
    """Independent 2D specimens run to failure in shared launches."""

    def __init__(self, images, *, k, s, mass, a=1.0, dt=0.01, gamma=0.1, precision="fp32k",
                 predictor="affine", void_value=-1, device="cuda:0", stream=None):
        import torch

        L = _load_batch(load_library())
        self._L = L
        self._h = None
        imgs = [np.ascontiguousarray(im, dtype=np.uint8) for im in images]
        if not imgs or any(im.ndim != 2 for im in imgs):
            raise ValueError("a batch needs 2D images")
        self._imgs = imgs  # keep alive during creation
        cfg = make_config(lattice=TRI2D, k=k, s=s, mass=mass, a=a, dt=dt, gamma=gamma,
                          precision=precision, predictor=predictor, void_value=void_value)
        n = len(imgs)
        ptrs = (C.c_void_p * n)(*[im.ctypes.data for im in imgs])
        dims = np.array([[im.shape[1], im.shape[0], 1] for im in imgs], dtype=np.int64)
        h = C.c_void_p()
        rc = L.lsm_batch_create(C.byref(cfg), n, ptrs, _ptr(dims), C.byref(h))
        if rc != LSM_OK:
            raise LsmError(rc, L.lsm_strerror(rc).decode())
        self._h = h
        self.n = n
        np_, ms = C.c_int64(), C.c_int64()
        L.lsm_batch_counts(h, C.byref(np_), C.byref(ms))
        self.n_particles, self.n_springs = np_.value, ms.value
        nb = C.c_size_t()
        self._check(L.lsm_batch_workspace_bytes(h, C.byref(nb)))
        self.device = torch.device(device)
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._check(L.lsm_batch_bind(h, C.c_void_p(self.workspace.data_ptr()), nb.value,
                                     C.c_void_p(self.stream.cuda_stream)))
        self.max_inc = None

    @classmethod
    def from_workload(cls, wl: dict, images, **over):
        kw = dict(k=wl["k"], s=wl["s"], mass=wl["mass"], a=wl.get("a", 1.0), dt=wl["dt"],
                  gamma=wl["gamma"], precision=wl.get("precision", "fp32k"),
                  void_value=wl.get("void_value", -1))
        kw.update(over)
        return cls(images, **kw)

    def _check(self, rc):
        if rc == LSM_OK:
            return rc
        msg = self._L.lsm_batch_last_error(self._h).decode() if self._h else ""
        raise LsmError(rc, f"{self._L.lsm_strerror(rc).decode()}: {msg}")

    def close(self):
        if self._h is not None and self._h.value:
            self._L.lsm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_launch(self, rows_per_wave=4, prefetch=1, variant="auto"):
        v = {"auto": KERNEL_AUTO, "sweep": KERNEL_SWEEP, "sweep2": KERNEL_SWEEP2}[variant]
        self._check(self._L.lsm_batch_set_launch(self._h, v, int(rows_per_wave), int(prefetch)))

    def launch(self):
        t = Tuning()
        self._check(self._L.lsm_batch_get_launch(self._h, C.byref(t)))
        names = {KERNEL_SWEEP: "sweep", KERNEL_SWEEP2: "sweep2"}
        return dict(variant=names[t.variant], rows_per_wave=t.rows_per_wave, prefetch=t.prefetch,
                    steps_per_launch=t.steps_per_launch)

    def autotune(self, steps_per_trial=20):
        """Times the candidate launches on this batch before its run and keeps
        the fastest; returns [(variant, rows_per_wave, prefetch, us_per_step)]."""
        buf = (Tuning * 64)()
        n = C.c_int()
        self._check(self._L.lsm_batch_autotune(self._h, int(steps_per_trial), buf, 64, C.byref(n)))
        names = {KERNEL_SWEEP: "sweep", KERNEL_SWEEP2: "sweep2"}
        return [(names[t.variant], t.rows_per_wave, t.prefetch, t.us_per_step) for t in buf[:n.value]]

    def run(self, d_eps, steps_per_inc, max_inc, drop=0.01):
        rule = FailRule(float(drop))
        self._check(self._L.lsm_batch_run(self._h, float(d_eps), int(steps_per_inc),
                                          int(max_inc), C.byref(rule)))
        self.max_inc = int(max_inc)

    def read(self) -> dict:
        mi = self.max_inc
        sxx = np.zeros((self.n, mi))
        ninc = np.zeros(self.n, np.int32)
        mod = np.zeros(self.n)
        st = np.zeros(self.n)
        nb = np.zeros(self.n, np.int64)
        self._check(self._L.lsm_batch_read(self._h, mi, _ptr(sxx), _ptr(ninc), _ptr(mod),
                                           _ptr(st), _ptr(nb)))
        return dict(sigma_xx=sxx, n_inc=ninc, modulus=mod, strength=st, n_broken=nb)

    def set_timing(self, on):
        self._check(self._L.lsm_batch_set_timing(self._h, int(bool(on))))

    def read_timing(self):
        ms, steps, ss = C.c_double(), C.c_int64(), C.c_double()
        self._check(self._L.lsm_batch_read_timing(self._h, C.byref(ms), C.byref(steps),
                                                  C.byref(ss)))
        return ms.value, steps.value, ss.value
