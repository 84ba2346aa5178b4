"""ctypes binding of the FP64 CPU oracle (``oracle/lsm_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark are the only users.  The product package never
imports this module.  Parity unpinned: nothing here; every oracle function is
pinned by a CPU test (see the test files named ``test_oracle_*``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsm_oracle.c")
_LIB = os.environ.get("LSM_ORACLE_LIB") or os.path.join(_HERE, "liblsm_oracle.so")

TRI2D = 0
SC3D = 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: FP64, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Record(C.Structure):
    _fields_ = [("eps", C.c_double), ("sigma", C.c_double * 9), ("ke", C.c_double),
                ("pe", C.c_double), ("n_broken", C.c_int64), ("inc", C.c_int32),
                ("step", C.c_int32), ("status", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        P = C.POINTER
        L.orc_network.restype = vp
        L.orc_network.argtypes = [C.c_int, i64, vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, dbl]
        L.orc_lattice.restype = vp
        L.orc_lattice.argtypes = [C.c_int, vp, i64, i64, i64, dbl, C.c_int, vp, vp, dbl, dbl,
                                  vp, C.c_int]
        L.orc_set_dynamics.argtypes = [vp, dbl, dbl, C.c_int]
        L.orc_set_strain_rate.argtypes = [vp, dbl]
        L.orc_set_spring_law.argtypes = [vp, C.c_int, dbl]
        L.orc_apply_increment.argtypes = [vp, dbl]
        L.orc_relax.argtypes = [vp, i64]
        L.orc_record_state.argtypes = [vp, P(Record)]
        L.orc_run.argtypes = [vp, i32, i64, dbl, vp]
        L.orc_free.argtypes = [vp]
        L.orc_counts.argtypes = [vp, P(i64), P(i64), P(i32)]
        L.orc_omega.argtypes = [vp]
        L.orc_omega.restype = dbl
        for nm in ("orc_get_x", "orc_set_x", "orc_get_v", "orc_set_v", "orc_get_a", "orc_get_X0"):
            getattr(L, nm).argtypes = [vp, vp]
        L.orc_get_particles.argtypes = [vp, vp, vp, vp]
        L.orc_get_springs.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.orc_set_broken.argtypes = [vp, vp]
        L.orc_forces.argtypes = [vp, vp, C.c_int]
        L.orc_potential_energy.argtypes = [vp]
        L.orc_potential_energy.restype = dbl
        L.orc_n_events.argtypes = [vp]
        L.orc_n_events.restype = i64
        L.orc_get_events.argtypes = [vp, vp, vp, vp, vp]
        L.orc_get_clock.argtypes = [vp, P(i32), P(i32), P(dbl)]
        L.orc_run_to_failure.argtypes = [vp, dbl, i64, i32, dbl, vp, vp, vp, P(i32), P(dbl),
                                         P(dbl)]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class Params:
    """Material and integration parameters of a lattice run."""
    k: list            # P x P spring constants, NaN off-diagonal = series rule
    s: list            # P x P critical stretches, NaN off-diagonal = series rule
    mass: list         # per phase
    a: float = 1.0
    k_face: float = 1.0
    k_diag: float = 1.0
    dt: float = 0.01
    gamma: float = 0.1
    predictor: int = 0  # 0 affine, 1 grips only
    void_value: int = -1


EVENT_DTYPE = np.dtype([("inc", np.int32), ("step", np.int32), ("id", np.int64),
                        ("margin", np.float64)])


class Net:
    """A particle-spring network owned by the oracle."""

    def __init__(self, handle):
        if not handle:
            raise ValueError("oracle rejected the network description")
        self._h = C.c_void_p(handle)
        n, m, d = C.c_int64(), C.c_int64(), C.c_int32()
        lib().orc_counts(self._h, C.byref(n), C.byref(m), C.byref(d))
        self.n, self.m, self.dim = n.value, m.value, d.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_free(h)
            self._h = None

    # --- construction -------------------------------------------------
    @classmethod
    def network(cls, dim, X0, mass, c, grip, sp, sq, k, r0, rc, omega=1.0):
        X0 = np.ascontiguousarray(X0, dtype=np.float64)
        n = X0.shape[0]
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        c = np.ascontiguousarray(c, dtype=np.float64)
        grip = np.ascontiguousarray(grip, dtype=np.uint8)
        sp = np.ascontiguousarray(sp, dtype=np.int64)
        sq = np.ascontiguousarray(sq, dtype=np.int64)
        k = np.ascontiguousarray(k, dtype=np.float64)
        r0 = np.ascontiguousarray(r0, dtype=np.float64)
        rc = np.ascontiguousarray(rc, dtype=np.float64)
        h = lib().orc_network(dim, n, _ptr(X0), _ptr(mass), _ptr(c), _ptr(grip), len(sp),
                              _ptr(sp), _ptr(sq), _ptr(k), _ptr(r0), _ptr(rc), float(omega))
        return cls(h)

    @classmethod
    def lattice(cls, img: np.ndarray, prm: Params):
        img = np.ascontiguousarray(img, dtype=np.uint8)
        if img.ndim == 2:
            kind, (ny, nx), nz = TRI2D, img.shape, 1
        else:
            kind, (nz, ny, nx) = SC3D, img.shape
        P = len(prm.mass)
        kpp = np.ascontiguousarray(np.array(prm.k, dtype=np.float64).reshape(P, P))
        spp = np.ascontiguousarray(np.array(prm.s, dtype=np.float64).reshape(P, P))
        mass = np.ascontiguousarray(prm.mass, dtype=np.float64)
        h = lib().orc_lattice(kind, _ptr(img), nx, ny, nz, prm.a, P, _ptr(kpp), _ptr(spp),
                              prm.k_face, prm.k_diag, _ptr(mass), prm.void_value)
        net = cls(h)
        net.set_dynamics(prm.dt, prm.gamma, prm.predictor)
        return net

    # --- dynamics ------------------------------------------------------
    def set_dynamics(self, dt, gamma, predictor=0):
        lib().orc_set_dynamics(self._h, float(dt), float(gamma), int(predictor))

    def set_spring_law(self, law, c=0.0):
        """0 linear (Eq. 1-2), 1 recoverable in compression, 2 cubic with
        coefficient c; see the spring-law comment of the C source."""
        if lib().orc_set_spring_law(self._h, int(law), float(c)) != 0:
            raise ValueError("bad spring law")

    def set_strain_rate(self, rate):
        """Constant strain-rate loading (per unit time) from the next step."""
        lib().orc_set_strain_rate(self._h, float(rate))

    def run_rate(self, rate, nsteps, every):
        """The paper's protocol: grips at a constant strain rate for nsteps,
        a record (strain, stress, energies) every `every` steps."""
        self.set_strain_rate(rate)
        out = []
        done = 0
        while done < nsteps:
            n = min(every, nsteps - done)
            self.relax(n)
            done += n
            out.append(self.record())
        return out

    def apply_increment(self, d_eps):
        rc = lib().orc_apply_increment(self._h, float(d_eps))
        if rc != 0:
            raise RuntimeError(f"oracle increment failed: {rc}")

    def relax(self, nsteps):
        rc = lib().orc_relax(self._h, int(nsteps))
        if rc != 0:
            raise RuntimeError(f"oracle relax failed: {rc}")

    def record(self) -> dict:
        R = Record()
        lib().orc_record_state(self._h, C.byref(R))
        return record_to_dict(R)

    def run(self, n_inc, steps_per_inc, d_eps):
        recs = (Record * n_inc)()
        rc = lib().orc_run(self._h, int(n_inc), int(steps_per_inc), float(d_eps), recs)
        out = [record_to_dict(r) for r in recs]
        return rc, out

    def run_to_failure(self, d_eps, steps, max_inc, drop=0.01) -> dict:
        """Uniaxial test to failure; see orc_run_to_failure."""
        sxx = np.full(max_inc, np.nan)
        eps = np.full(max_inc, np.nan)
        nb = np.zeros(max_inc, dtype=np.int64)
        n = C.c_int32()
        mod, st = C.c_double(), C.c_double()
        rc = lib().orc_run_to_failure(self._h, float(d_eps), int(steps), int(max_inc),
                                      float(drop), _ptr(sxx), _ptr(eps), _ptr(nb), C.byref(n),
                                      C.byref(mod), C.byref(st))
        k = n.value
        return dict(status=rc, n_inc=k, sigma_xx=sxx[:k], eps=eps[:k], n_broken=nb[:k],
                    modulus=mod.value, strength=st.value)

    def forces(self, commit=False) -> np.ndarray:
        F = np.zeros((self.n, self.dim))
        rc = lib().orc_forces(self._h, _ptr(F), int(bool(commit)))
        if rc != 0:
            raise RuntimeError("oracle force evaluation failed")
        return F

    def potential_energy(self) -> float:
        return lib().orc_potential_energy(self._h)

    # --- state ---------------------------------------------------------
    def _get(self, fn):
        out = np.zeros((self.n, self.dim))
        fn(self._h, _ptr(out))
        return out

    @property
    def x(self):
        return self._get(lib().orc_get_x)

    @x.setter
    def x(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(self.n, self.dim)
        lib().orc_set_x(self._h, _ptr(val))

    @property
    def v(self):
        return self._get(lib().orc_get_v)

    @v.setter
    def v(self, val):
        val = np.ascontiguousarray(val, dtype=np.float64).reshape(self.n, self.dim)
        lib().orc_set_v(self._h, _ptr(val))

    @property
    def a(self):
        return self._get(lib().orc_get_a)

    @property
    def X0(self):
        return self._get(lib().orc_get_X0)

    @property
    def omega(self):
        return lib().orc_omega(self._h)

    def particles(self):
        mass = np.zeros(self.n)
        c = np.zeros(self.n)
        grip = np.zeros(self.n, dtype=np.uint8)
        lib().orc_get_particles(self._h, _ptr(mass), _ptr(c), _ptr(grip))
        return mass, c, grip

    def springs(self):
        sp = np.zeros(self.m, dtype=np.int64)
        sq = np.zeros(self.m, dtype=np.int64)
        k = np.zeros(self.m)
        r0 = np.zeros(self.m)
        rc = np.zeros(self.m)
        br = np.zeros(self.m, dtype=np.uint8)
        lib().orc_get_springs(self._h, _ptr(sp), _ptr(sq), _ptr(k), _ptr(r0), _ptr(rc), _ptr(br))
        return dict(p=sp, q=sq, k=k, r0=r0, rc=rc, broken=br)

    def set_broken(self, broken):
        b = np.ascontiguousarray(broken, dtype=np.uint8)
        lib().orc_set_broken(self._h, _ptr(b))

    def events(self) -> np.ndarray:
        ne = lib().orc_n_events(self._h)
        inc = np.zeros(ne, dtype=np.int32)
        step = np.zeros(ne, dtype=np.int32)
        ids = np.zeros(ne, dtype=np.int64)
        mg = np.zeros(ne)
        if ne:
            lib().orc_get_events(self._h, _ptr(inc), _ptr(step), _ptr(ids), _ptr(mg))
        ev = np.zeros(ne, dtype=EVENT_DTYPE)
        ev["inc"], ev["step"], ev["id"], ev["margin"] = inc, step, ids, mg
        return ev

    def clock(self):
        i, s, e = C.c_int32(), C.c_int32(), C.c_double()
        lib().orc_get_clock(self._h, C.byref(i), C.byref(s), C.byref(e))
        return i.value, s.value, e.value


def record_to_dict(R: Record) -> dict:
    return dict(eps=R.eps, sigma=np.array(R.sigma[:]).reshape(3, 3), ke=R.ke, pe=R.pe,
                n_broken=R.n_broken, inc=R.inc, step=R.step, status=R.status)
