"""Python binding of libmgmc.so (the MI355X MGMC sampler).

Argument marshalling only: every step of the sampler runs in the HIP library.
The functions carry the names of the C ABI in ``include/mgmc.h``; torch is
used for device memory and streams.  If the library has not been built the
import of this module fails loudly -- there is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgmc.so")

MGMC_OK, MGMC_EINVAL, MGMC_ENOMEM, MGMC_EDEVICE, MGMC_ENOTSPD, MGMC_EUNSUPPORTED, MGMC_ESTATE = range(7)
MGMC_FP64, MGMC_FP32 = 0, 1
MGMC_OPT_TILED_SWEEPS, MGMC_OPT_SWEEP_VARIANT, MGMC_OPT_CHAINS_PER_BLOCK = 1, 2, 3
MGMC_OPT_COARSE_FUSED, MGMC_OPT_LOWRANK_MFMA, MGMC_OPT_MARCH3D, MGMC_OPT_RESTRICT3D = 4, 5, 6, 7
MGMC_OP_FD, MGMC_OP_FEM_Q1, MGMC_OP_SSL13 = 0, 1, 2
MGMC_SAMPLER_MGMC, MGMC_SAMPLER_GIBBS, MGMC_SAMPLER_CHOLESKY = 0, 1, 2
_OPS = {"fd": MGMC_OP_FD, "fem": MGMC_OP_FEM_Q1, "ssl13": MGMC_OP_SSL13}
_SAMPLERS = {"mgmc": MGMC_SAMPLER_MGMC, "gibbs": MGMC_SAMPLER_GIBBS, "cholesky": MGMC_SAMPLER_CHOLESKY}

EXPORTED = [
    "mgmc_setup", "mgmc_sample", "mgmc_posterior_sample", "mgmc_levels", "mgmc_level_sites",
    "mgmc_set_graph", "mgmc_set_option", "mgmc_set_profiling", "mgmc_profile_read", "mgmc_destroy",
    "mgmc_last_error", "mgmc_time_updates", "mgmc_batch_create", "mgmc_batch_sample",
    "mgmc_batch_destroy", "mgmc_set_level_option", "mgmc_pnet_param_count", "mgmc_pnet_create", "mgmc_pnet_set_params",
    "mgmc_pnet_get_params", "mgmc_pnet_weights", "mgmc_pnet_loss_grad", "mgmc_pnet_train_step",
    "mgmc_pnet_destroy", "mgmc_sample_noalloc",
]

_dp = ctypes.POINTER(ctypes.c_double)


class mgmc_problem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int32), ("n", ctypes.c_int32), ("levels", ctypes.c_int32),
        ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("kappa2", ctypes.c_double),
        ("scale", ctypes.c_double), ("face_coef", _dp), ("prolong_w", _dp),
        ("precision", ctypes.c_int32), ("nchains", ctypes.c_int32),
        ("chain_offset", ctypes.c_int64), ("seed", ctypes.c_uint64),
        ("op", ctypes.c_int32), ("cycle_gamma", ctypes.c_int32), ("omega", ctypes.c_double),
        ("nu0", ctypes.c_int32), ("sampler", ctypes.c_int32),
    ]


class mgmc_obs(ctypes.Structure):
    _fields_ = [
        ("beta", ctypes.c_int32), ("ptr", ctypes.POINTER(ctypes.c_int64)),
        ("idx", ctypes.POINTER(ctypes.c_int32)), ("val", _dp), ("gamma", _dp),
    ]


class MGMCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mgmc status {status}: {message}")
        self.status = status


_lib = None


def load_library():
    """Load libmgmc.so; raise if it is missing (build it with python -m paper_2407_12149_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: the HIP library must be built "
                          "(python -m paper_2407_12149_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    lib.mgmc_setup.restype = ctypes.c_int
    lib.mgmc_setup.argtypes = [ctypes.POINTER(mgmc_problem), ctypes.POINTER(mgmc_obs), vp,
                               ctypes.POINTER(vp)]
    lib.mgmc_sample.restype = ctypes.c_int
    lib.mgmc_sample.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp]
    lib.mgmc_sample_noalloc.restype = ctypes.c_int
    lib.mgmc_sample_noalloc.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp]
    lib.mgmc_posterior_sample.restype = ctypes.c_int
    lib.mgmc_posterior_sample.argtypes = [vp, _dp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp]
    lib.mgmc_levels.restype = ctypes.c_int32
    lib.mgmc_levels.argtypes = [vp]
    lib.mgmc_level_sites.restype = ctypes.c_int64
    lib.mgmc_level_sites.argtypes = [vp, ctypes.c_int32]
    lib.mgmc_set_graph.restype = ctypes.c_int
    lib.mgmc_set_graph.argtypes = [vp, ctypes.c_int32]
    lib.mgmc_set_option.restype = ctypes.c_int
    lib.mgmc_set_option.argtypes = [vp, ctypes.c_int32, ctypes.c_int64]
    lib.mgmc_set_level_option.restype = ctypes.c_int
    lib.mgmc_set_level_option.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64]
    lib.mgmc_set_profiling.restype = ctypes.c_int
    lib.mgmc_set_profiling.argtypes = [vp, ctypes.c_int32]
    lib.mgmc_profile_read.restype = ctypes.c_int
    lib.mgmc_profile_read.argtypes = [vp, _dp, ctypes.POINTER(ctypes.c_int64)]
    lib.mgmc_time_updates.restype = ctypes.c_int
    lib.mgmc_time_updates.argtypes = [vp, ctypes.c_int32, _dp]
    lib.mgmc_batch_create.restype = ctypes.c_int
    lib.mgmc_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, vp,
                                      ctypes.POINTER(vp)]
    lib.mgmc_batch_sample.restype = ctypes.c_int
    lib.mgmc_batch_sample.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(vp),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp)]
    lib.mgmc_batch_destroy.restype = ctypes.c_int
    lib.mgmc_batch_destroy.argtypes = [vp]
    lib.mgmc_destroy.restype = ctypes.c_int
    lib.mgmc_destroy.argtypes = [vp]
    _fp = ctypes.POINTER(ctypes.c_float)
    lib.mgmc_pnet_param_count.restype = ctypes.c_int64
    lib.mgmc_pnet_param_count.argtypes = []
    lib.mgmc_pnet_create.restype = ctypes.c_int
    lib.mgmc_pnet_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp,
                                     ctypes.POINTER(vp)]
    lib.mgmc_pnet_set_params.restype = ctypes.c_int
    lib.mgmc_pnet_set_params.argtypes = [vp, _fp]
    lib.mgmc_pnet_get_params.restype = ctypes.c_int
    lib.mgmc_pnet_get_params.argtypes = [vp, _fp]
    lib.mgmc_pnet_weights.restype = ctypes.c_int
    lib.mgmc_pnet_weights.argtypes = [vp, vp, ctypes.c_int32, vp]
    lib.mgmc_pnet_loss_grad.restype = ctypes.c_int
    lib.mgmc_pnet_loss_grad.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                        _dp, _fp]
    lib.mgmc_pnet_train_step.restype = ctypes.c_int
    lib.mgmc_pnet_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.c_float, _dp]
    lib.mgmc_pnet_destroy.restype = ctypes.c_int
    lib.mgmc_pnet_destroy.argtypes = [vp]
    lib.mgmc_last_error.restype = ctypes.c_char_p
    lib.mgmc_last_error.argtypes = []
    _lib = lib
    return lib


def _check(status):
    if status != MGMC_OK:
        raise MGMCError(status, load_library().mgmc_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def mgmc_setup(problem, obs=None, stream=None):
    """problem: dict with dim, n, levels, kappa2 and optional scale, face_coef,
    prolong_w, nu1, nu2, precision ('fp64'|'fp32'), nchains, chain_offset, seed,
    op ('fd'|'fem'|'ssl13'), cycle_gamma, omega, nu0, sampler
    ('mgmc'|'gibbs'|'cholesky').  obs: (ptr, idx, val, gamma) numpy arrays or
    None.  Returns an opaque handle."""
    lib = load_library()
    keep = []

    def arr(a, dtype):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=dtype)
        keep.append(a)
        return a

    face = arr(problem.get("face_coef"), np.float64)
    pw = arr(problem.get("prolong_w"), np.float64)
    prec = problem.get("precision", "fp64")
    p = mgmc_problem(
        dim=int(problem["dim"]), n=int(problem["n"]), levels=int(problem["levels"]),
        nu1=int(problem.get("nu1", 1)), nu2=int(problem.get("nu2", 1)),
        kappa2=float(problem["kappa2"]), scale=float(problem.get("scale", 0.0) or 0.0),
        face_coef=None if face is None else face.ctypes.data_as(_dp),
        prolong_w=None if pw is None else pw.ctypes.data_as(_dp),
        precision=MGMC_FP32 if prec in ("fp32", MGMC_FP32) else MGMC_FP64,
        nchains=int(problem.get("nchains", 1)), chain_offset=int(problem.get("chain_offset", 0)),
        seed=int(problem.get("seed", 0)),
        op=_OPS.get(problem.get("op", "fd"), problem.get("op", 0)),
        cycle_gamma=int(problem.get("cycle_gamma", 1)), omega=float(problem.get("omega", 1.0)),
        nu0=int(problem.get("nu0", 0)),
        sampler=_SAMPLERS.get(problem.get("sampler", "mgmc"), problem.get("sampler", 0)))
    o = None
    if obs is not None:
        ptr, idx, val, gamma = obs
        ptr, idx = arr(ptr, np.int64), arr(idx, np.int32)
        val, gamma = arr(val, np.float64), arr(gamma, np.float64)
        o = mgmc_obs(beta=len(ptr) - 1, ptr=ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                     idx=idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     val=val.ctypes.data_as(_dp), gamma=gamma.ctypes.data_as(_dp))
    handle = ctypes.c_void_p()
    _check(lib.mgmc_setup(ctypes.byref(p), None if o is None else ctypes.byref(o),
                          _stream_handle(stream), ctypes.byref(handle)))
    return handle


def mgmc_sample(ctx, m0, nsamples, theta, rhs=None, F=None, qoi=None):
    _check(load_library().mgmc_sample(ctx, int(m0), int(nsamples), _ptr(theta), _ptr(rhs),
                                      _ptr(F), _ptr(qoi)))


def mgmc_sample_noalloc(ctx, m0, nsamples, theta, rhs=None, F=None, qoi=None):
    _check(load_library().mgmc_sample_noalloc(ctx, int(m0), int(nsamples), _ptr(theta), _ptr(rhs),
                                              _ptr(F), _ptr(qoi)))


def mgmc_posterior_sample(ctx, y, m0, nsamples, theta, F=None, qoi=None):
    y = np.ascontiguousarray(y, dtype=np.float64)
    _check(load_library().mgmc_posterior_sample(ctx, y.ctypes.data_as(_dp), int(m0),
                                                int(nsamples), _ptr(theta), _ptr(F), _ptr(qoi)))


def mgmc_levels(ctx):
    return int(load_library().mgmc_levels(ctx))


def mgmc_level_sites(ctx, level):
    return int(load_library().mgmc_level_sites(ctx, int(level)))


def mgmc_set_graph(ctx, enabled):
    _check(load_library().mgmc_set_graph(ctx, 1 if enabled else 0))


def mgmc_set_option(ctx, option, value):
    _check(load_library().mgmc_set_option(ctx, int(option), int(value)))


def mgmc_set_level_option(ctx, level, option, value):
    _check(load_library().mgmc_set_level_option(ctx, int(level), int(option), int(value)))


def mgmc_set_profiling(ctx, enabled):
    _check(load_library().mgmc_set_profiling(ctx, 1 if enabled else 0))


def mgmc_profile_read(ctx):
    """(summed kernel milliseconds, launches) of the finest-level sweeps."""
    ms = ctypes.c_double()
    cnt = ctypes.c_int64()
    _check(load_library().mgmc_profile_read(ctx, ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


def mgmc_time_updates(ctx, nupdates):
    ms = ctypes.c_double()
    _check(load_library().mgmc_time_updates(ctx, int(nupdates), ctypes.byref(ms)))
    return ms.value


def mgmc_batch_create(ctxs, updates_per_launch, stream):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    handle = ctypes.c_void_p()
    _check(load_library().mgmc_batch_create(arr, len(ctxs), int(updates_per_launch),
                                            _stream_handle(stream), ctypes.byref(handle)))
    return handle


def mgmc_batch_sample(batch, m0, nsamples, thetas, Fs=None, qois=None):
    k = len(thetas)

    def ptrs(ts):
        if ts is None:
            return None
        return (ctypes.c_void_p * k)(*[None if t is None else t.data_ptr() for t in ts])

    _check(load_library().mgmc_batch_sample(batch, int(m0), int(nsamples), ptrs(thetas),
                                            ptrs(Fs), ptrs(qois)))


def mgmc_batch_destroy(batch):
    _check(load_library().mgmc_batch_destroy(batch))


def mgmc_destroy(ctx):
    _check(load_library().mgmc_destroy(ctx))


def mgmc_last_error():
    return load_library().mgmc_last_error().decode()


def mgmc_pnet_param_count():
    return int(load_library().mgmc_pnet_param_count())


def mgmc_pnet_create(n, max_batch, max_errors, stream=None):
    handle = ctypes.c_void_p()
    _check(load_library().mgmc_pnet_create(int(n), int(max_batch), int(max_errors),
                                           _stream_handle(stream), ctypes.byref(handle)))
    return handle


def mgmc_pnet_set_params(net, params):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(load_library().mgmc_pnet_set_params(net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))


def mgmc_pnet_get_params(net):
    a = np.zeros(mgmc_pnet_param_count(), dtype=np.float32)
    _check(load_library().mgmc_pnet_get_params(net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return a


def mgmc_pnet_weights(net, faces, batch, w):
    _check(load_library().mgmc_pnet_weights(net, _ptr(faces), int(batch), _ptr(w)))


def mgmc_pnet_loss_grad(net, faces, errors, batch, nerrors, kappa2, want_grad=True):
    """(loss, grad or None); faces and errors are device tensors."""
    loss = ctypes.c_double()
    grad = np.zeros(mgmc_pnet_param_count(), dtype=np.float32) if want_grad else None
    _check(load_library().mgmc_pnet_loss_grad(
        net, _ptr(faces), _ptr(errors), int(batch), int(nerrors), float(kappa2), ctypes.byref(loss),
        None if grad is None else grad.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return loss.value, grad


def mgmc_pnet_train_step(net, faces, errors, batch, nerrors, kappa2, lr, want_loss=True):
    loss = ctypes.c_double()
    _check(load_library().mgmc_pnet_train_step(net, _ptr(faces), _ptr(errors), int(batch),
                                               int(nerrors), float(kappa2), float(lr),
                                               ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def mgmc_pnet_destroy(net):
    _check(load_library().mgmc_pnet_destroy(net))


class PNet:
    """Learned prolongation network on its own torch stream (fine grid n)."""

    def __init__(self, n, max_batch=1, max_errors=1, params=None, device="cuda"):
        import torch
        self.n = n
        self.nc = (n - 1) // 2
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.handle = mgmc_pnet_create(n, max_batch, max_errors, self.stream)
        if params is not None:
            self.set_params(params)

    def _wait(self):
        import torch
        self.stream.wait_stream(torch.cuda.current_stream(self.device))

    def set_params(self, params):
        mgmc_pnet_set_params(self.handle, params)

    def params(self):
        return mgmc_pnet_get_params(self.handle)

    def weights(self, faces):
        """faces: device FP64 [batch][2 (n+1) n] -> device FP64 [batch][nc*nc][9]."""
        import torch
        faces = faces.reshape(-1, 2 * (self.n + 1) * self.n).contiguous()
        w = torch.empty((faces.shape[0], self.nc * self.nc, 9), dtype=torch.float64,
                        device=self.device)
        self._wait()
        mgmc_pnet_weights(self.handle, faces, faces.shape[0], w)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        faces.record_stream(self.stream)
        w.record_stream(self.stream)
        return w

    def loss_grad(self, faces, errors, kappa2, want_grad=True):
        faces = faces.reshape(-1, 2 * (self.n + 1) * self.n).contiguous()
        b = faces.shape[0]
        errors = errors.reshape(b, -1, self.n * self.n).contiguous()
        self._wait()
        return mgmc_pnet_loss_grad(self.handle, faces, errors, b, errors.shape[1], kappa2, want_grad)

    def train_step(self, faces, errors, kappa2, lr, want_loss=True):
        faces = faces.reshape(-1, 2 * (self.n + 1) * self.n).contiguous()
        b = faces.shape[0]
        errors = errors.reshape(b, -1, self.n * self.n).contiguous()
        self._wait()
        out = mgmc_pnet_train_step(self.handle, faces, errors, b, errors.shape[1], kappa2, lr,
                                   want_loss)
        if not want_loss:
            faces.record_stream(self.stream)
            errors.record_stream(self.stream)
        return out

    def close(self):
        if getattr(self, "handle", None) is not None:
            mgmc_pnet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Sampler:
    """Owner of one context plus the chain states (torch tensors on the GPU)."""

    def __init__(self, problem, obs=None, stream=None, device="cuda"):
        import torch
        self.torch = torch
        self.problem = dict(problem)
        self.dtype = torch.float32 if problem.get("precision", "fp64") == "fp32" else torch.float64
        self.nchains = int(problem.get("nchains", 1))
        self.N = int(problem["n"]) ** int(problem["dim"])
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.ctx = mgmc_setup(problem, obs, self.stream)
        self.device = device
        self.theta = torch.zeros(self.nchains, self.N, dtype=self.dtype, device=device)

    def _run(self, call, nsamples, F, want_qoi):
        torch = self.torch
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        qoi = None
        with torch.cuda.stream(self.stream):
            if F is not None and want_qoi:
                qoi = torch.zeros(nsamples, self.nchains, dtype=torch.float64, device=self.device)
            call(F if qoi is not None else None, qoi)
        cur.wait_stream(self.stream)
        return qoi

    def sample(self, m0, nsamples, rhs=None, F=None, want_qoi=True):
        """Updates m0..m0+nsamples-1 of every chain in place on self.theta;
        returns the [nsamples, nchains] FP64 QoI series if F is given."""
        return self._run(lambda Fp, q: mgmc_sample(self.ctx, m0, nsamples, self.theta, rhs, Fp, q),
                         nsamples, F, want_qoi)

    def posterior_sample(self, y, m0, nsamples, F=None, want_qoi=True):
        return self._run(
            lambda Fp, q: mgmc_posterior_sample(self.ctx, y, m0, nsamples, self.theta, Fp, q),
            nsamples, F, want_qoi)

    def synchronize(self):
        self.stream.synchronize()

    def set_graph(self, enabled):
        mgmc_set_graph(self.ctx, enabled)

    def set_option(self, option, value):
        mgmc_set_option(self.ctx, option, value)

    def set_level_option(self, level, option, value):
        mgmc_set_level_option(self.ctx, level, option, value)

    def set_profiling(self, enabled):
        mgmc_set_profiling(self.ctx, enabled)

    def profile_read(self):
        return mgmc_profile_read(self.ctx)

    def time_updates(self, nupdates):
        return mgmc_time_updates(self.ctx, nupdates)

    def close(self):
        if self.ctx is not None:
            mgmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several samplers (any sizes) updated together: each step of all their
    chains is one launch of a HIP graph with one branch per sampler."""

    def __init__(self, samplers, updates_per_launch=10, stream=None):
        import torch
        self.torch = torch
        self.samplers = list(samplers)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.handle = mgmc_batch_create([s.ctx for s in self.samplers], updates_per_launch,
                                        self.stream)

    def sample(self, m0, nsamples, Fs=None):
        """Advance every sampler's chains; returns one QoI series per sampler
        (None where no F is given)."""
        torch = self.torch
        cur = torch.cuda.current_stream()
        self.stream.wait_stream(cur)
        for s in self.samplers:
            self.stream.wait_stream(s.stream)
        qois = None
        with torch.cuda.stream(self.stream):
            if Fs is not None:
                qois = [None if F is None else
                        torch.zeros(nsamples, s.nchains, dtype=torch.float64, device=s.device)
                        for s, F in zip(self.samplers, Fs)]
            mgmc_batch_sample(self.handle, m0, nsamples, [s.theta for s in self.samplers],
                              Fs, qois)
        cur.wait_stream(self.stream)
        return qois

    def close(self):
        if self.handle is not None:
            mgmc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
