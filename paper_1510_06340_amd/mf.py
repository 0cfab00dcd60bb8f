"""Thin ctypes binding of libmf.so (the C ABI declared in include/mf.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream; state tensors are
passed by raw pointer and must stay alive (the Grid keeps references).
There is no fallback: if libmf.so is missing or the device is unavailable,
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmf.so")

MF_OK, MF_ERR_ARG, MF_ERR_NOMEM, MF_ERR_HIP, MF_ERR_STATE, MF_ERR_UNPHYSICAL, MF_ERR_CFL = 0, -1, -2, -3, -4, -5, -6
MF_BC_OUTFLOW, MF_BC_PERIODIC = 0, 1
MF_F64, MF_F32 = 0, 1
MF_LIM_NONE, MF_LIM_MINMOD, MF_LIM_SUPERBEE, MF_LIM_MC, MF_LIM_VANLEER, MF_LIM_VANALBADA = range(6)
MF_EOS_IDEAL, MF_EOS_TABLE, MF_EOS_GAMMA = 0, 1, 2
MF_C2P_PLAIN, MF_C2P_SEEDED, MF_C2P_CONFORMAL = 0, 1, 2
MF_MLP_HIDDEN, MF_MLP_PARAMS = 64, 4417
MF_MLP_NOALLOC_MAX_N = 16384
MF_FLAG_STRICT = 1
MF_FLAG_PREDICTOR_ALPHA = 2
MF_FLAG_UNSPLIT_HANCOCK = 4
MF_FLAG_CHARGE = 8

EXPORTS = ["mf_grid_init", "mf_set_eos", "mf_set_source_jet", "mf_set_time", "mf_step", "mf_batch_step",
           "mf_con2prim", "mf_con2prim_stats", "mf_totals", "mf_set_tuning", "mf_set_profiling", "mf_get_profile",
           "mf_grid_free", "mf_last_error", "mf_mlp_workspace", "mf_mlp_forward", "mf_mlp_grad", "mf_mlp_grad_noalloc",
           "mf_mlp_adam"]


class GridDesc(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dx", C.c_double * 3), ("origin", C.c_double * 3), ("bc", C.c_int32 * 3),
                ("dtype", C.c_int32), ("limiter", C.c_int32), ("musta_k", C.c_int32), ("rk_order", C.c_int32),
                ("alpha", C.c_double), ("flags", C.c_uint32)]


class Stats(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_int64), ("smax", C.c_double), ("courant", C.c_double),
                ("totals", C.c_double * 4), ("n_floor", C.c_int64), ("n_bad", C.c_int64),
                ("newton_iters", C.c_int64), ("n_fallback", C.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["totals"] = list(self.totals)
        return d


class Surrogate(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("w1", C.POINTER(C.c_float)), ("b1", C.POINTER(C.c_float)),
                ("w2", C.POINTER(C.c_float)), ("b2", C.POINTER(C.c_float)), ("w3", C.POINTER(C.c_float)),
                ("b3", C.c_float), ("in_shift", C.c_float * 2), ("in_scale", C.c_float * 2),
                ("out_shift", C.c_float), ("out_scale", C.c_float),
                ("output", C.c_int32)]


class MFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1510_06340_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.mf_last_error.restype = C.c_char_p
        L.mf_grid_init.argtypes = [C.POINTER(vp), C.POINTER(GridDesc), C.c_int32, C.POINTER(vp), vp]
        L.mf_set_eos.argtypes = [vp, C.c_int32, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.c_int32, C.POINTER(Surrogate)]
        L.mf_set_source_jet.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.c_double, C.c_double, C.c_double]
        L.mf_set_time.argtypes = [vp, C.c_int32, C.c_double, C.c_int64]
        L.mf_step.argtypes = [vp, C.c_double, C.c_int32, C.POINTER(Stats)]
        L.mf_batch_step.argtypes = [vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(Stats)]
        L.mf_con2prim.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_int64, vp, C.c_int32]
        L.mf_totals.argtypes = [vp, C.c_int32, C.POINTER(C.c_double)]
        L.mf_set_tuning.argtypes = [vp, C.POINTER(C.c_int32), C.c_int32]
        L.mf_set_profiling.argtypes = [vp, C.c_int32]
        L.mf_get_profile.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.mf_grid_free.argtypes = [vp]
        L.mf_con2prim_stats.argtypes = [vp, C.POINTER(C.c_int64)]
        L.mf_mlp_workspace.argtypes = [C.c_int64]
        L.mf_mlp_forward.argtypes = [vp, vp, C.c_int64, vp, vp]
        L.mf_mlp_grad.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp, C.c_int64, vp]
        L.mf_mlp_grad_noalloc.argtypes = [vp, vp, vp, C.c_int64, vp, vp, vp]
        L.mf_mlp_adam.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        for name in EXPORTS:
            if name not in ("mf_last_error", "mf_mlp_workspace"):
                getattr(L, name).restype = C.c_int
        L.mf_mlp_workspace.restype = C.c_int64
        _lib = L
    return _lib


def last_error() -> str:
    return lib().mf_last_error().decode()


def _check(rc):
    if rc != MF_OK:
        raise MFError(rc, last_error())


def _ptr(t) -> int:
    return t.data_ptr()


def make_desc(n, dx, origin, bc, dtype=MF_F64, limiter=MF_LIM_MC, k=3, rk=2, alpha=3.0, flags=0) -> GridDesc:
    d = GridDesc()
    d.n[:] = [int(v) for v in n]
    d.dx[:] = [float(v) for v in dx]
    d.origin[:] = [float(v) for v in origin]
    d.bc[:] = [int(v) for v in bc]
    d.dtype, d.limiter, d.musta_k, d.rk_order = int(dtype), int(limiter), int(k), int(rk)
    d.alpha, d.flags = float(alpha), int(flags)
    return d


def desc_from_workload(w, dtype=MF_F64, flags=0) -> GridDesc:
    if w.extra.get("charge"):
        flags |= MF_FLAG_CHARGE
    return make_desc(w.n, w.dx, w.xlo, w.bc, dtype, w.limiter, w.k, w.rk, w.alpha, flags)


class Grid:
    """A handle over one or more events whose state lives in caller-owned device tensors.

    states: list (one per event) of 4 contiguous CUDA tensors (E, Mx, My, Mz),
    each with n[0]*n[1]*n[2] elements of the event's dtype; 5 (R last) for
    descriptors with MF_FLAG_CHARGE.
    """

    def __init__(self, descs, states, stream=None):
        import torch
        if isinstance(descs, GridDesc):
            descs = [descs]
        if len(descs) != len(states):
            raise ValueError("one state (4 tensors) per descriptor")
        self._torch = torch
        self.descs = list(descs)
        self.states = [list(s) for s in states]
        for d, s in zip(self.descs, self.states):
            want = torch.float32 if d.dtype == MF_F32 else torch.float64
            ncell = d.n[0] * d.n[1] * d.n[2]
            if len(s) != (5 if d.flags & MF_FLAG_CHARGE else 4):
                raise ValueError("4 component tensors per event (5 with the charge)")
            for t in s:
                if not t.is_cuda or t.dtype != want or not t.is_contiguous() or t.numel() != ncell:
                    raise ValueError("state tensors must be contiguous CUDA tensors of the event's dtype and size")
        ptrs = [_ptr(t) for s in self.states for t in s]
        arr = (C.c_void_p * len(ptrs))(*ptrs)
        darr = (GridDesc * len(self.descs))(*self.descs)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(lib().mf_grid_init(C.byref(h), darr, len(self.descs), arr, C.c_void_p(stream.cuda_stream)))
        self.h = h

    @property
    def n_events(self):
        return len(self.descs)

    def set_eos_ideal(self, cs2=1.0 / 3.0):
        _check(lib().mf_set_eos(self.h, MF_EOS_IDEAL, float(cs2), None, None, 0, None))

    def set_eos_gamma(self, gamma=5.0 / 3.0):
        """The ideal gas p = (gamma - 1) max(e - n, 0) (needs the charge)."""
        _check(lib().mf_set_eos(self.h, MF_EOS_GAMMA, float(gamma), None, None, 0, None))

    def set_eos_table(self, e, p, surrogate=None):
        """surrogate: None or a SeedNetwork (keeps its arrays alive)."""
        import numpy as np
        e = np.ascontiguousarray(e, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        D = C.POINTER(C.c_double)
        s = surrogate.struct() if surrogate is not None else None
        _check(lib().mf_set_eos(self.h, MF_EOS_TABLE, 0.0, e.ctypes.data_as(D), p.ctypes.data_as(D), len(e),
                                C.byref(s) if s is not None else None))

    def set_jet(self, event, x0, v, dedx, sigma):
        x = (C.c_double * 3)(*[float(q) for q in x0])
        _check(lib().mf_set_source_jet(self.h, int(event), x, float(v), float(dedx), float(sigma)))

    def set_time(self, event, t, steps=0):
        _check(lib().mf_set_time(self.h, int(event), float(t), int(steps)))

    def set_tuning(self, seg=(0, 0, 0), block=256):
        s = (C.c_int32 * 3)(*[int(q) for q in seg])
        _check(lib().mf_set_tuning(self.h, s, int(block)))

    def step(self, dt, nsteps, stats=True):
        """Advance every event; returns a list of per-event stats dicts (or None)."""
        if stats:
            st = (Stats * self.n_events)()
            _check(lib().mf_step(self.h, float(dt), int(nsteps), st))
            return [s.as_dict() for s in st]
        _check(lib().mf_step(self.h, float(dt), int(nsteps), None))
        return None

    def batch_step(self, dts, nsteps, stats=True):
        dt = (C.c_double * self.n_events)(*[float(v) for v in dts])
        if stats:
            st = (Stats * self.n_events)()
            _check(lib().mf_batch_step(self.h, dt, int(nsteps), st))
            return [s.as_dict() for s in st]
        _check(lib().mf_batch_step(self.h, dt, int(nsteps), None))
        return None

    def con2prim(self, U, prim, iters=None, mode=MF_C2P_PLAIN):
        """U: 4 device tensors, prim: 5 device tensors (e, p, vx, vy, vz), iters: int32 tensor or None;
        with the charge U: 5 (R last), prim: 6 (n last)."""
        n = U[0].numel()
        u = (C.c_void_p * len(U))(*[_ptr(t) for t in U])
        p = (C.c_void_p * len(prim))(*[_ptr(t) for t in prim])
        it = C.c_void_p(_ptr(iters)) if iters is not None else None
        _check(lib().mf_con2prim(self.h, u, p, n, it, int(mode)))

    def set_profiling(self, enable=True):
        _check(lib().mf_set_profiling(self.h, 1 if enable else 0))

    def get_profile(self):
        """Per sweep axis (x, y, z): (summed kernel ms, launches) since the last read."""
        ms = (C.c_double * 3)()
        n = (C.c_int64 * 3)()
        _check(lib().mf_get_profile(self.h, ms, n))
        return list(ms), list(n)

    def con2prim_stats(self):
        """Counters of the last con2prim call: (clamped, bad, iterations, seeded guesses outside the bracket)."""
        out = (C.c_int64 * 4)()
        _check(lib().mf_con2prim_stats(self.h, out))
        return list(out)

    def totals(self, event=0):
        """Sums of E, Mx, My, Mz (and R with the charge) times the cell volume."""
        nc = 5 if self.descs[event].flags & MF_FLAG_CHARGE else 4
        out = (C.c_double * nc)()
        _check(lib().mf_totals(self.h, int(event), out))
        return list(out)

    def free(self):
        if getattr(self, "h", None):
            _check(lib().mf_grid_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class SeedNetwork:
    """Host copy of the seed network's FP32 weights and normalisation (for mf_set_eos)."""

    def __init__(self, params, in_shift, in_scale, out_shift, out_scale, output=0):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MF_MLP_PARAMS:
            raise ValueError(f"expected {MF_MLP_PARAMS} parameters")
        H = MF_MLP_HIDDEN
        o = np.cumsum([0, 2 * H, H, H * H, H, H])
        self.params = p
        self.w1, self.b1, self.w2, self.b2, self.w3 = (np.ascontiguousarray(p[o[i]:o[i + 1]]) for i in range(5))
        self.b3 = float(p[-1])
        self.in_shift, self.in_scale = [float(v) for v in in_shift], [float(v) for v in in_scale]
        self.out_shift, self.out_scale = float(out_shift), float(out_scale)
        self.output = int(output)

    def struct(self) -> Surrogate:
        F = C.POINTER(C.c_float)
        s = Surrogate()
        s.hidden = MF_MLP_HIDDEN
        s.w1, s.b1, s.w2, s.b2, s.w3 = (a.ctypes.data_as(F) for a in (self.w1, self.b1, self.w2, self.b2, self.w3))
        s.b3 = self.b3
        s.in_shift[:] = self.in_shift
        s.in_scale[:] = self.in_scale
        s.out_shift, s.out_scale = self.out_shift, self.out_scale
        s.output = self.output
        return s


def mlp_forward(params, X, y, stream=None):
    """y = MLP(X) on the device (torch tensors: params (4417,), X (n, 2), y (n,), float32)."""
    st = stream.cuda_stream if stream is not None else None
    _check(lib().mf_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(y), st))


def mlp_workspace(n) -> int:
    return int(lib().mf_mlp_workspace(int(n)))


def mlp_grad(params, X, t, grad, loss, work, stream=None):
    st = stream.cuda_stream if stream is not None else None
    _check(lib().mf_mlp_grad(_ptr(params), _ptr(X), _ptr(t), X.shape[0], _ptr(grad),
                             _ptr(loss) if loss is not None else None, _ptr(work), work.numel(), st))


def mlp_grad_noalloc(params, X, t, grad, loss, stream=None):
    """mlp_grad with the partial gradients in the library's static device array (no workspace;
    at most MF_MLP_NOALLOC_MAX_N samples; calls that overlap on one GPU race)."""
    st = stream.cuda_stream if stream is not None else None
    _check(lib().mf_mlp_grad_noalloc(_ptr(params), _ptr(X), _ptr(t), X.shape[0], _ptr(grad),
                                     _ptr(loss) if loss is not None else None, st))


def mlp_adam(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    st = stream.cuda_stream if stream is not None else None
    _check(lib().mf_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                             float(beta2), float(eps), st))
