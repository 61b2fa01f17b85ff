"""Python access to the plain FP64 CPU oracle of Multigrid Monte Carlo.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it to check and time the HIP library.  The product
path never imports this package.

The oracle follows Alg. 1 (V-cycle) with the low-rank Gibbs smoother of
Alg. 3 (omega = 1) and an exact Cholesky coarsest sample, see
``mgmc_oracle.h`` for the conventions.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None

OP_FD, OP_FEM_Q1, OP_SSL13 = 0, 1, 2
SAMPLER_MGMC, SAMPLER_GIBBS = 0, 1


class OraOptions(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n", ctypes.c_int), ("levels", ctypes.c_int),
        ("kappa2", ctypes.c_double), ("scale", ctypes.c_double),
        ("face_coef", ctypes.POINTER(ctypes.c_double)), ("prolong_w", ctypes.POINTER(ctypes.c_double)),
        ("nu1", ctypes.c_int), ("nu2", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("op", ctypes.c_int), ("gamma", ctypes.c_int), ("omega", ctypes.c_double),
        ("nu0", ctypes.c_int), ("sampler", ctypes.c_int),
    ]

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_i64_p = ctypes.POINTER(ctypes.c_int64)
_c_i32_p = ctypes.POINTER(ctypes.c_int32)
_c_u32_p = ctypes.POINTER(ctypes.c_uint32)


def load():
    """Load liboracle.so, compiling it with gcc first if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    lib.ora_philox4x32_10.argtypes = [_c_u32_p, _c_u32_p, _c_u32_p]
    lib.ora_normal_pair.argtypes = [_c_u32_p, _c_u32_p, _c_double_p]
    lib.ora_create_ex.restype = ctypes.c_void_p
    lib.ora_create_ex.argtypes = [ctypes.POINTER(OraOptions)]
    lib.ora_set_noise_log.argtypes = [ctypes.c_void_p, _c_u32_p, ctypes.c_int64]
    lib.ora_noise_log_len.restype = ctypes.c_int64
    lib.ora_noise_log_len.argtypes = [ctypes.c_void_p]
    lib.ora_create.restype = ctypes.c_void_p
    lib.ora_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, _c_double_p, _c_double_p, ctypes.c_int,
                               ctypes.c_int, ctypes.c_uint64]
    lib.ora_destroy.argtypes = [ctypes.c_void_p]
    lib.ora_last_error.restype = ctypes.c_char_p
    lib.ora_set_obs.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_i64_p, _c_i32_p, _c_double_p,
                                _c_double_p]
    lib.ora_set_rhs.argtypes = [ctypes.c_void_p, _c_double_p]
    lib.ora_set_posterior_rhs.argtypes = [ctypes.c_void_p, _c_double_p]
    lib.ora_set_noise.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]
    lib.ora_set_restriction_scale.argtypes = [ctypes.c_void_p, ctypes.c_double]
    lib.ora_noise_drawn.restype = ctypes.c_int64
    lib.ora_noise_drawn.argtypes = [ctypes.c_void_p]
    lib.ora_cycle.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, _c_double_p]
    lib.ora_chain.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                              _c_double_p, _c_double_p, _c_double_p, _c_double_p]
    lib.ora_smooth.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int64, ctypes.c_int64, _c_double_p, _c_double_p]
    lib.ora_levels.argtypes = [ctypes.c_void_p]
    lib.ora_level_n.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.ora_level_sites.restype = ctypes.c_int64
    lib.ora_level_sites.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.ora_beta.argtypes = [ctypes.c_void_p]
    lib.ora_dense.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_double_p]
    _LIB = lib
    return lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(_c_double_p)


def philox4x32_10(ctr, key):
    lib = load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib.ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normal_pair(ctr, key):
    lib = load()
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_double * 2)()
    lib.ora_normal_pair(c, k, o)
    return float(o[0]), float(o[1])


NOISE_PHILOX, NOISE_ZERO, NOISE_IMPULSE = 0, 1, 2


class Oracle:
    """One problem hierarchy of the oracle (prior, or posterior after set_obs)."""

    def __init__(self, dim, n, levels, kappa2, scale=0.0, face_coef=None, prolong_w=None,
                 nu1=1, nu2=1, seed=0, op=OP_FD, gamma=1, omega=1.0, nu0=0, sampler=SAMPLER_MGMC):
        lib = load()
        self._keep = []
        fc = None if face_coef is None else np.ascontiguousarray(face_coef, dtype=np.float64)
        pw = None if prolong_w is None else np.ascontiguousarray(prolong_w, dtype=np.float64)
        self._keep += [fc, pw]
        opts = OraOptions(dim=dim, n=n, levels=levels, kappa2=kappa2, scale=scale,
                          face_coef=_dp(fc), prolong_w=_dp(pw), nu1=nu1, nu2=nu2, seed=seed,
                          op=op, gamma=gamma, omega=omega, nu0=nu0, sampler=sampler)
        h = lib.ora_create_ex(ctypes.byref(opts))
        if not h:
            raise ValueError("oracle: " + lib.ora_last_error().decode())
        self.h = h
        self.lib = lib
        self.dim, self.n, self.levels = dim, n, levels
        self.N = int(lib.ora_level_sites(h, levels - 1))
        self.beta = 0

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.ora_destroy(self.h)
            self.h = None

    def set_obs(self, ptr, idx, val, gamma):
        ptr = np.ascontiguousarray(ptr, dtype=np.int64)
        idx = np.ascontiguousarray(idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        gamma = np.ascontiguousarray(gamma, dtype=np.float64)
        beta = len(ptr) - 1
        rc = self.lib.ora_set_obs(self.h, beta, ptr.ctypes.data_as(_c_i64_p),
                                  idx.ctypes.data_as(_c_i32_p), _dp(val), _dp(gamma))
        if rc != 0:
            raise ValueError("oracle: " + self.lib.ora_last_error().decode())
        self.beta = beta

    def set_rhs(self, f):
        f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        self.lib.ora_set_rhs(self.h, _dp(f))

    def set_posterior_rhs(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        if self.lib.ora_set_posterior_rhs(self.h, _dp(y)) != 0:
            raise ValueError("oracle: " + self.lib.ora_last_error().decode())

    def set_noise(self, mode, impulse=0):
        self.lib.ora_set_noise(self.h, mode, impulse)

    def set_restriction_scale(self, scale):
        """Planted-mistake hook (tests only): f_{l-1} = scale * P^T r."""
        self.lib.ora_set_restriction_scale(self.h, scale)

    def noise_drawn(self):
        return int(self.lib.ora_noise_drawn(self.h))

    def log_noise(self, fn, cap=1 << 20):
        """Run fn() with draw logging on; returns an [draws, 7] uint32 array of
        (key0, key1, counter0..3, slot) in draw order."""
        buf = np.zeros((cap, 7), dtype=np.uint32)
        self.lib.ora_set_noise_log(self.h, buf.ctypes.data_as(_c_u32_p), cap)
        try:
            fn()
            k = int(self.lib.ora_noise_log_len(self.h))
        finally:
            self.lib.ora_set_noise_log(self.h, None, 0)
        if k > cap:
            raise ValueError("noise log overflow")
        return buf[:k].copy()

    def cycle(self, theta, chain=0, m=0):
        t = np.ascontiguousarray(theta, dtype=np.float64).copy()
        self.lib.ora_cycle(self.h, chain, m, _dp(t))
        return t

    def chain(self, theta0, m0, nsamples, chain=0, F=None, traj=False):
        t = np.ascontiguousarray(theta0, dtype=np.float64).copy()
        Fa = None if F is None else np.ascontiguousarray(F, dtype=np.float64)
        q = np.zeros(nsamples) if F is not None else None
        tr = np.zeros((nsamples, self.N)) if traj else None
        rc = self.lib.ora_chain(self.h, chain, m0, nsamples, _dp(t), _dp(Fa), _dp(q), _dp(tr))
        if rc != 0:
            raise RuntimeError("oracle: " + self.lib.ora_last_error().decode())
        return t, q, tr

    def smooth(self, level, direction, theta, f=None, sigma=0, chain=0, m=0):
        t = np.ascontiguousarray(theta, dtype=np.float64).copy()
        fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
        if self.lib.ora_smooth(self.h, level, direction, sigma, chain, m, _dp(t), _dp(fa)) != 0:
            raise ValueError("oracle: " + self.lib.ora_last_error().decode())
        return t

    def level_n(self, level):
        return int(self.lib.ora_level_n(self.h, level))

    def level_sites(self, level):
        return int(self.lib.ora_level_sites(self.h, level))

    def dense(self, level, what):
        N = self.level_sites(level)
        shape = {0: (N, N), 1: (N, self.level_sites(level - 1)) if level > 0 else (0, 0),
                 2: (N, self.beta), 3: (N, self.beta), 4: (N, self.beta), 5: (N, N),
                 6: (N, N), 7: (N,), 8: (N,)}[what]
        out = np.zeros(shape)
        if self.lib.ora_dense(self.h, level, what, _dp(out)) != 0:
            raise ValueError("oracle: dense accessor failed")
        return out
