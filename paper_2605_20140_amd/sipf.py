"""ctypes binding of libsipf.so (argument marshalling only; every step runs in HIP kernels).

PyTorch provides the device workspace (a uint8 tensor on the GPU) and the stream.  The
library must be built (``python -m paper_2605_20140_amd.build``); importing this module
without it raises, so nothing can silently fall back to another implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsipf.so")

SIPF_FP64 = 0
SIPF_FP32 = 1

FLAG_FREEZE_W = 0x01
FLAG_FREEZE_V = 0x02
FLAG_FREEZE_M = 0x04
FLAG_NO_NOISE = 0x08
FLAG_LINEAR_MASS = 0x10
FLAG_IMPLICIT_V = 0x20
FLAG_STRICT = 0x40
FLAG_EXP_DIFFUSION = 0x80
FLAG_ALIASED_DIFFUSION = 0x100

ERRORS = {-1: "SIPF_EINVAL", -2: "SIPF_ENOMEM", -3: "SIPF_EHIP", -4: "SIPF_EPOS"}

# exported symbols, as declared in include/sipf.h
EXPORTS = ("sipf_state_bytes", "sipf_init", "sipf_step", "sipf_set_stream", "sipf_step_batch",
           "sipf_step_batch_noalloc", "sipf_fields", "sipf_aux", "sipf_step_timed",
           "sipf_resample", "sipf_destroy", "sipf_last_error")
STAGES = ("zfwd", "yfwd", "xpass", "yinv", "zinv", "particles", "finalize", "binning")


class Params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double), ("N", ctypes.c_int32), ("dim", ctypes.c_int32),
        ("P", ctypes.c_int64), ("dt", ctypes.c_double),
        ("D_u", ctypes.c_double), ("chi", ctypes.c_double), ("D_m", ctypes.c_double),
        ("D_w", ctypes.c_double), ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("sim_id", ctypes.c_uint64), ("step0", ctypes.c_uint64),
        ("precision", ctypes.c_int32), ("deposit_order", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("resort_every", ctypes.c_int32), ("H0", ctypes.c_double),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass_particles", ctypes.c_double), ("mass_grid", ctypes.c_double),
        ("mass_m", ctypes.c_double),
        ("min_v", ctypes.c_double), ("min_m", ctypes.c_double), ("min_w", ctypes.c_double),
        ("max_m", ctypes.c_double), ("max_w", ctypes.c_double),
        ("min_a", ctypes.c_double), ("max_a", ctypes.c_double), ("min_u", ctypes.c_double),
        ("n_nan", ctypes.c_int64), ("n_neg_m", ctypes.c_int64), ("n_neg_w", ctypes.c_int64),
        ("step", ctypes.c_int64),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ResampleInfo(ctypes.Structure):
    _fields_ = [("a0", ctypes.c_double), ("n_det", ctypes.c_int64), ("n_stoch", ctypes.c_int64)]


class SipfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libsipf.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_20140_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
        L.sipf_state_bytes.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]
        L.sipf_init.argtypes = [ctypes.POINTER(Params), vp, ctypes.c_size_t, vp,
                                dp, dp, dp, dp, dp, ctypes.POINTER(vp)]
        L.sipf_step.argtypes = [vp, ctypes.c_int32]
        L.sipf_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32]
        L.sipf_step_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32]
        L.sipf_set_stream.argtypes = [vp, vp]
        L.sipf_fields.argtypes = [vp, dp, dp, dp, dp, dp, ctypes.POINTER(Diag)]
        L.sipf_aux.argtypes = [vp, dp, dp]
        L.sipf_step_timed.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]
        L.sipf_resample.argtypes = [vp, ctypes.POINTER(ResampleInfo)]
        L.sipf_destroy.argtypes = [vp]
        L.sipf_destroy.restype = None
        L.sipf_last_error.restype = ctypes.c_char_p
        for name in ("sipf_state_bytes", "sipf_init", "sipf_step", "sipf_step_batch",
                     "sipf_step_batch_noalloc", "sipf_fields", "sipf_aux", "sipf_step_timed",
                     "sipf_set_stream", "sipf_resample"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise SipfError(rc, lib().sipf_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def make_params(N, P, dt, L=1.0, D_u=1e-3, chi=5e-3, D_m=1e-3, D_w=5e-3, alpha=10.0,
                beta=0.5, gamma=0.5, seed=0, sim_id=0, step0=0, precision=SIPF_FP64,
                deposit_order=2, flags=0, resort_every=0, H0=0.0, dim=0, **_ignored):
    return Params(L=L, N=N, dim=dim, P=P, dt=dt, D_u=D_u, chi=chi, D_m=D_m, D_w=D_w,
                  alpha=alpha, beta=beta, gamma=gamma, seed=seed, sim_id=sim_id, step0=step0,
                  precision=precision, deposit_order=deposit_order, flags=flags,
                  resort_every=resort_every, H0=H0)


def state_bytes(params):
    n = ctypes.c_size_t(0)
    _check(lib().sipf_state_bytes(ctypes.byref(params), ctypes.byref(n)))
    return n.value


class Simulation:
    """One resident simulation: workspace tensor + library handle.

    X0: (P, d) float64 positions; a0: (P,) masses; v0, m0, w0: (N,)*d fields; d = 3, or 2
    when params.dim == 2.
    """

    def __init__(self, params, X0, a0, v0, m0, w0, device="cuda", stream=None):
        import torch
        self.params = params
        N, P = params.N, params.P
        self.d = d = 2 if params.dim == 2 else 3
        nbytes = state_bytes(params)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        if stream is None:
            stream = torch.cuda.current_stream(self.workspace.device)
        self.stream = stream
        X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64).reshape(P, d).T)
        a0 = np.ascontiguousarray(a0, dtype=np.float64)
        v0 = np.ascontiguousarray(v0, dtype=np.float64).reshape(-1)
        m0 = np.ascontiguousarray(m0, dtype=np.float64).reshape(-1)
        w0 = np.ascontiguousarray(w0, dtype=np.float64).reshape(-1)
        assert v0.size == m0.size == w0.size == N ** d and a0.size == P
        h = ctypes.c_void_p()
        _check(lib().sipf_init(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()),
                               nbytes, ctypes.c_void_p(stream.cuda_stream),
                               _dptr(X0), _dptr(a0), _dptr(v0), _dptr(m0), _dptr(w0),
                               ctypes.byref(h)))
        self.handle = h

    def step(self, nsteps=1):
        _check(lib().sipf_step(self.handle, int(nsteps)))

    def fields(self, particles=True):
        N, P, d = self.params.N, self.params.P, self.d
        v = np.empty(N ** d)
        m = np.empty(N ** d)
        w = np.empty(N ** d)
        X = np.empty(d * P) if particles else None
        a = np.empty(P) if particles else None
        d = Diag()
        rc = lib().sipf_fields(self.handle, _dptr(v), _dptr(m), _dptr(w), _dptr(X), _dptr(a),
                               ctypes.byref(d))
        shape = (N,) * self.d
        out = dict(v=v.reshape(shape), m=m.reshape(shape), w=w.reshape(shape),
                   diag=d.as_dict(), rc=rc)
        if particles:
            out["X"] = X.reshape(self.d, P).T.copy()
            out["a"] = a
        if rc not in (0, -4):
            _check(rc)
        return out

    def aux(self):
        N, d = self.params.N, self.d
        G = N ** d
        u = np.empty(G)
        g = np.empty(d * G)
        _check(lib().sipf_aux(self.handle, _dptr(u), _dptr(g)))
        return u.reshape((N,) * d), [g[j * G:(j + 1) * G].reshape((N,) * d) for j in range(d)]

    def set_stream(self, stream):
        """Move the simulation's work to a torch stream (queued work is ordered before)."""
        _check(lib().sipf_set_stream(self.handle, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def step_timed(self, nsteps=1):
        """Run nsteps steps eagerly with HIP events between stages; per-stage total ms."""
        buf = (ctypes.c_float * len(STAGES))()
        _check(lib().sipf_step_timed(self.handle, int(nsteps), buf))
        return dict(zip(STAGES, list(buf)))

    def resample(self):
        """Residual resampling of the particles (synchronous); returns a0, n_det, n_stoch."""
        info = ResampleInfo()
        _check(lib().sipf_resample(self.handle, ctypes.byref(info)))
        return dict(a0=info.a0, n_det=info.n_det, n_stoch=info.n_stoch)

    def close(self):
        if getattr(self, "handle", None):
            lib().sipf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def step_batch(sims, nsteps=1):
    arr = (ctypes.c_void_p * len(sims))(*[s.handle for s in sims])
    _check(lib().sipf_step_batch(arr, len(sims), int(nsteps)))


def step_batch_noalloc(sims, nsteps=1):
    """sipf_step_batch_noalloc: the batched step with its launch table in the library's
    per-GPU device array (no device allocation, no graph instantiation)."""
    arr = (ctypes.c_void_p * len(sims))(*[s.handle for s in sims])
    _check(lib().sipf_step_batch_noalloc(arr, len(sims), int(nsteps)))
