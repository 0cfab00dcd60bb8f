"""Plain FP64 CPU oracle of the MUSTA-FORCE step (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It wraps ``mf_oracle.c`` (plain C, built
with gcc into ``liboracle.so`` next to this file) and the exact Riemann solver
in :mod:`oracle.riemann`.  It shares no code with the HIP library.

Arrays are numpy float64, conserved state shaped (4, nz, ny, nx) with x
fastest: components (E, Mx, My, Mz); with the conserved charge (Problem(charge=True))
(5, nz, ny, nx), the fifth component being R.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LIM_NONE, LIM_MINMOD, LIM_SUPERBEE, LIM_MC, LIM_VANLEER, LIM_VANALBADA = range(6)
BC_OUTFLOW, BC_PERIODIC = 0, 1
EOS_IDEAL, EOS_TABLE, EOS_GAMMA = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, no fast-math, OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                        "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int32 * 3), ("bc", C.c_int32 * 3), ("dx", C.c_double * 3), ("xlo", C.c_double * 3),
        ("limiter", C.c_int32), ("k", C.c_int32), ("rk", C.c_int32), ("alpha", C.c_double),
        ("eos", C.c_int32), ("cs2", C.c_double), ("ntab", C.c_int32),
        ("etab", C.POINTER(C.c_double)), ("ptab", C.POINTER(C.c_double)), ("mtab", C.POINTER(C.c_double)),
        ("jet", C.c_int32), ("jet_x0", C.c_double * 3), ("jet_v", C.c_double), ("jet_dedx", C.c_double),
        ("jet_sigma", C.c_double), ("predictor_alpha", C.c_int32), ("unsplit_hancock", C.c_int32),
        ("charge", C.c_int32), ("gamma", C.c_double),
    ]


class Counters(C.Structure):
    _fields_ = [("n_floor", C.c_int64), ("n_bad", C.c_int64), ("n_iter", C.c_int64), ("n_calls", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Stats(C.Structure):
    _fields_ = [("smax", C.c_double), ("cnt", Counters)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        L.ora_pchip_slopes.argtypes = [C.c_int32, _D, _D, _D]
        L.ora_eos_eval.argtypes = [C.POINTER(Params), C.c_int64, _D, _D, _D]
        L.ora_con2prim.argtypes = [C.POINTER(Params), C.c_int64] + [_D] * 11 + [C.POINTER(Counters)]
        L.ora_flux.argtypes = [C.POINTER(Params), C.c_int32, C.c_int64, _D, _D]
        L.ora_limiter.argtypes = [C.c_int32, C.c_int64, _D, _D, _D]
        L.ora_musta.argtypes = [C.POINTER(Params), C.c_int32, C.c_double, C.c_int64, _D, _D, _D]
        L.ora_rhs.argtypes = [C.POINTER(Params), _D, C.c_double, C.c_double, _D, C.POINTER(Counters)]
        L.ora_max_speed.argtypes = [C.POINTER(Params), _D, C.POINTER(Counters)]
        L.ora_max_speed.restype = C.c_double
        L.ora_totals.argtypes = [C.POINTER(Params), _D, _D]
        L.ora_step.argtypes = [C.POINTER(Params), _D, C.c_double, C.c_double, C.c_int32, C.POINTER(Stats)]
        L.ora_step.restype = C.c_int
        L.ora_num_threads.restype = C.c_int
        L.ora_set_num_threads.argtypes = [C.c_int32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class Problem:
    """Grid, scheme and EoS parameters; keeps the table arrays alive."""

    def __init__(self, n=(1, 1, 1), dx=(1.0, 1.0, 1.0), xlo=(0.0, 0.0, 0.0), bc=(0, 0, 0),
                 limiter=LIM_MINMOD, k=2, rk=2, alpha=3.0, cs2=1.0 / 3.0, table=None, jet=None,
                 predictor_alpha=False, unsplit_hancock=False, charge=False, gamma=None):
        """charge: carry the conserved charge R as a fifth component (flux R v_d).
        gamma: the ideal-gas EoS p = (gamma - 1) max(e - n, 0) (needs charge)."""
        self.p = Params()
        self.p.n[:] = [int(v) for v in n]
        self.p.bc[:] = [int(v) for v in bc]
        self.p.dx[:] = [float(v) for v in dx]
        self.p.xlo[:] = [float(v) for v in xlo]
        self.p.limiter, self.p.k, self.p.rk, self.p.alpha = int(limiter), int(k), int(rk), float(alpha)
        self.p.cs2 = float(cs2)
        self.p.eos = EOS_IDEAL
        self._keep = []
        if table is not None:
            e, p = _f64(table[0]), _f64(table[1])
            m = pchip_slopes(e, p)
            self._keep = [e, p, m]
            self.p.eos = EOS_TABLE
            self.p.ntab = len(e)
            self.p.etab, self.p.ptab, self.p.mtab = _p(e), _p(p), _p(m)
        self.p.charge = 1 if charge else 0
        if gamma is not None:
            if not charge:
                raise ValueError("the ideal-gas EoS p(e, n) needs the charge")
            self.p.eos = EOS_GAMMA
            self.p.gamma = float(gamma)
        self.p.predictor_alpha = 1 if predictor_alpha else 0
        self.p.unsplit_hancock = 1 if unsplit_hancock else 0
        self.p.jet = 0
        if jet is not None:
            self.p.jet = 1
            self.p.jet_x0[:] = [float(v) for v in jet["x0"]]
            self.p.jet_v, self.p.jet_dedx, self.p.jet_sigma = float(jet["v"]), float(jet["dedx"]), float(jet["sigma"])

    @classmethod
    def from_workload(cls, w, table=None, jet_x0=None):
        jet = None
        if w.jet is not None:
            jet = dict(x0=jet_x0, v=w.jet["v"], dedx=w.jet["dedx"], sigma=w.jet["sigma"])
        return cls(n=w.n, dx=w.dx, xlo=w.xlo, bc=w.bc, limiter=w.limiter, k=w.k, rk=w.rk,
                   alpha=w.alpha, cs2=w.cs2, table=table, jet=jet,
                   predictor_alpha=w.extra.get("predictor_alpha", False),
                   unsplit_hancock=w.extra.get("unsplit_hancock", False),
                   charge=w.extra.get("charge", False), gamma=w.extra.get("gamma"))

    @property
    def nc(self):
        """Conserved components per cell: 5 with the charge, else 4."""
        return 5 if self.p.charge else 4

    @property
    def ref(self):
        return C.byref(self.p)


def pchip_slopes(x, y) -> np.ndarray:
    x, y = _f64(x), _f64(y)
    m = np.empty_like(x)
    lib().ora_pchip_slopes(len(x), _p(x), _p(y), _p(m))
    return m


def eos(prob: Problem, e):
    e = _f64(e).ravel()
    p, d = np.empty_like(e), np.empty_like(e)
    lib().ora_eos_eval(prob.ref, len(e), _p(e), _p(p), _p(d))
    return p, d


def con2prim(prob: Problem, U):
    """U: (nc, ...) -> (prim (5, ...) = e, p, vx, vy, vz, or (6, ...) with the charge's rest-frame
    density n last; counters dict)."""
    U = _f64(U)
    nc = prob.nc
    shape = U.shape[1:]
    n = int(np.prod(shape)) if shape else 1
    Uf = U.reshape(nc, n)
    comps = [np.ascontiguousarray(Uf[i]) for i in range(nc)]
    out = [np.empty(n) for _ in range(nc + 1)]
    cnt = Counters()
    R = _p(comps[4]) if nc == 5 else None
    nrest = _p(out[5]) if nc == 5 else None
    lib().ora_con2prim(prob.ref, n, *[_p(a) for a in comps[:4]], R, *[_p(a) for a in out[:5]], nrest,
                       C.byref(cnt))
    return np.stack(out).reshape((nc + 1,) + shape), cnt.as_dict()


def flux(prob: Problem, d: int, U):
    U = _f64(U)
    shape = U.shape[1:]
    n = int(np.prod(shape)) if shape else 1
    Uf = np.ascontiguousarray(U.reshape(prob.nc, n))
    F = np.empty_like(Uf)
    lib().ora_flux(prob.ref, d, n, _p(Uf), _p(F))
    return F.reshape(U.shape)


def limiter(kind: int, a, b):
    a, b = np.broadcast_arrays(_f64(a), _f64(b))
    a, b = _f64(a).ravel(), _f64(b).ravel()
    out = np.empty_like(a)
    lib().ora_limiter(kind, len(a), _p(a), _p(b), _p(out))
    return out


def musta(prob: Problem, d: int, lam: float, UL, UR):
    UL, UR = _f64(UL), _f64(UR)
    shape = UL.shape[1:]
    n = int(np.prod(shape)) if shape else 1
    l, r = np.ascontiguousarray(UL.reshape(prob.nc, n)), np.ascontiguousarray(UR.reshape(prob.nc, n))
    F = np.empty_like(l)
    lib().ora_musta(prob.ref, d, lam, n, _p(l), _p(r), _p(F))
    return F.reshape(UL.shape)


def rhs(prob: Problem, U, t: float, dt: float):
    U = _f64(U)
    L = np.empty_like(U)
    cnt = Counters()
    lib().ora_rhs(prob.ref, _p(U), t, dt, _p(L), C.byref(cnt))
    return L, cnt.as_dict()


def max_speed(prob: Problem, U) -> float:
    U = _f64(U)
    return float(lib().ora_max_speed(prob.ref, _p(U), None))


def totals(prob: Problem, U) -> np.ndarray:
    U = _f64(U)
    out = np.empty(prob.nc)
    lib().ora_totals(prob.ref, _p(U), _p(out))
    return out


def step(prob: Problem, U, dt: float, nsteps: int, t0: float = 0.0):
    """Advance a copy of U by nsteps RK steps; returns (U_new, stats dict)."""
    V = _f64(U).copy()
    st = Stats()
    rc = lib().ora_step(prob.ref, _p(V), t0, dt, int(nsteps), C.byref(st))
    if rc != 0:
        raise MemoryError("oracle step could not allocate its work arrays")
    d = st.cnt.as_dict()
    d["smax"] = float(st.smax)
    return V, d


def num_threads() -> int:
    return int(lib().ora_num_threads())


def set_num_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))
