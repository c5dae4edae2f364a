"""ctypes loader of the CPU FP64 oracle (liborc.so).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it to produce reference results.  The GPU library never
imports it.  The oracle is built from oracle/*.cpp by build() (g++, -O2, no
fast-math, no FMA contraction on the default x86-64 target).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile liborc.so in place."""
    srcs = [os.path.join(_HERE, "orc.cpp")]
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", _LIB + ".tmp"] + srcs
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [("gamma", C.c_double), ("courant", C.c_double), ("dt_base", C.c_double),
                ("dt_fixed", C.c_double), ("grace", C.c_double), ("p_floor", C.c_double),
                ("kmax", C.c_int32), ("nslots", C.c_int32), ("nguard", C.c_int32),
                ("limiter", C.c_int32), ("prec", C.c_int32), ("dt_mode", C.c_int32),
                ("periodic", C.c_int32 * 3), ("box_lo", C.c_double * 3),
                ("box_hi", C.c_double * 3), ("eta", C.c_double), ("gamma_ad", C.c_double),
                ("rho_ion", C.c_double), ("torder", C.c_int32)]


class _Desc(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("size", C.c_double * 3), ("n", C.c_int32),
                ("level", C.c_int32), ("flags", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        L.orc_create.argtypes = [C.POINTER(_Cfg), C.POINTER(_Desc), C.c_int32, C.POINTER(C.c_void_p)]
        L.orc_init.argtypes = [C.c_void_p, dp, C.c_size_t, C.c_double]
        L.orc_advance_to.argtypes = [C.c_void_p, C.c_double]
        L.orc_read_state.argtypes = [C.c_void_p, dp, C.c_size_t, dp]
        L.orc_read_schedule.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_int32), C.c_size_t]
        L.orc_stats.argtypes = [C.c_void_p, dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_last_error.restype = C.c_char_p
        L.orc_set_order.argtypes = [C.c_void_p, C.c_int32, C.c_uint64, C.c_int32]
        L.orc_layout.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        L.orc_nbors.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_size_t]
        L.orc_padded.argtypes = [C.c_void_p, C.c_int32, dp, C.c_size_t]
        L.orc_slot.argtypes = [C.c_void_p, C.c_int32, C.c_int32, dp, C.c_size_t,
                               C.POINTER(C.c_int64), dp]
        L.orc_advance_limited.argtypes = [C.c_void_p, C.c_double, C.c_int64]
        L.orc_times.argtypes = [C.c_void_p, C.POINTER(C.c_int64), dp]
        L.orc_hlld_flux.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, dp]
        L.orc_jvp_fixed.argtypes = [C.c_void_p, dp, dp, C.c_int32, C.c_double, dp, dp]
        L.orc_count_flops.argtypes = [C.c_void_p, dp, C.c_double, dp]
        L.orc_extrapolated.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise OracleError(rc, lib().orc_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_cfg(cfg) -> _Cfg:
    c = _Cfg()
    for f in ("gamma", "courant", "dt_base", "dt_fixed", "grace", "p_floor", "kmax", "nslots",
              "nguard", "limiter", "prec", "dt_mode", "eta", "gamma_ad", "rho_ion", "torder"):
        setattr(c, f, getattr(cfg, f))
    for d in range(3):
        c.periodic[d] = int(cfg.periodic[d])
        c.box_lo[d] = cfg.box_lo[d]
        c.box_hi[d] = cfg.box_hi[d]
    return c


def make_descs(patches):
    arr = (_Desc * len(patches))()
    for i, p in enumerate(patches):
        for d in range(3):
            arr[i].origin[d] = p.origin[d]
            arr[i].size[d] = p.size
        arr[i].n = p.n
        arr[i].level = p.level
        arr[i].flags = 1 if p.frozen else 0
    return arr


class OracleSet:
    """A patch set advanced by the CPU oracle (FP64)."""

    def __init__(self, cfg, patches):
        self.cfg, self.patches = cfg, list(patches)
        self._c = make_cfg(cfg)
        self._d = make_descs(self.patches)
        h = C.c_void_p()
        _check(lib().orc_create(C.byref(self._c), self._d, len(self.patches), C.byref(h)))
        self.h = h
        self.nvals = int(sum(5 * p.n ** 3 + 3 * p.n * p.n * (p.n + 1) for p in self.patches))

    @classmethod
    def from_problem(cls, prob, **over):
        import dataclasses
        cfg = dataclasses.replace(prob.cfg, **over) if over else prob.cfg
        s = cls(cfg, prob.patches)
        s.init(prob.U0)
        return s

    def close(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    __del__ = close

    def init(self, U, t0=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64)
        _check(lib().orc_init(self.h, _dp(U), U.size, t0))

    def advance_to(self, t):
        _check(lib().orc_advance_to(self.h, float(t)))

    def advance_limited(self, t, max_updates):
        _check(lib().orc_advance_limited(self.h, float(t), int(max_updates)))

    def times(self):
        n = len(self.patches)
        tk = np.zeros(n, dtype=np.int64)
        t = np.zeros(n)
        _check(lib().orc_times(self.h, tk.ctypes.data_as(C.POINTER(C.c_int64)), _dp(t)))
        return tk, t

    def extrapolated(self):
        c = C.c_int64()
        _check(lib().orc_extrapolated(self.h, C.byref(c)))
        return c.value

    def read_state(self):
        U = np.empty(self.nvals)
        t = C.c_double()
        _check(lib().orc_read_state(self.h, _dp(U), U.size, C.byref(t)))
        return U

    def read_schedule(self, klog_cap=0):
        n = len(self.patches)
        steps = np.zeros(n, dtype=np.int64)
        kh = np.zeros(n, dtype=np.uint64)
        kl = np.zeros(n * max(klog_cap, 1), dtype=np.int32)
        _check(lib().orc_read_schedule(self.h, steps.ctypes.data_as(C.POINTER(C.c_int64)),
                                       kh.ctypes.data_as(C.POINTER(C.c_uint64)),
                                       kl.ctypes.data_as(C.POINTER(C.c_int32)) if klog_cap else None,
                                       klog_cap))
        if klog_cap:
            return steps, kh, kl.reshape(n, klog_cap)
        return steps, kh

    def stats(self):
        out = np.zeros(16)
        _check(lib().orc_stats(self.h, _dp(out)))
        return out

    def set_order(self, order=0, seed=1, nthreads=1):
        _check(lib().orc_set_order(self.h, order, seed, nthreads))

    def nbors(self):
        n = len(self.patches)
        cnt = np.zeros(n, dtype=np.int32)
        _check(lib().orc_nbors(self.h, cnt.ctypes.data_as(C.POINTER(C.c_int32)), None, 0))
        ids = np.zeros(int(cnt.sum()), dtype=np.int32)
        _check(lib().orc_nbors(self.h, cnt.ctypes.data_as(C.POINTER(C.c_int32)),
                               ids.ctypes.data_as(C.POINTER(C.c_int32)), ids.size))
        out, o = [], 0
        for c in cnt:
            out.append(ids[o:o + c].tolist())
            o += c
        return out

    def padded(self, p):
        n = self.patches[p].n
        N = n + 2 * self.cfg.nguard
        size = 5 * N ** 3 + 3 * N * N * (N + 1)
        out = np.empty(size)
        _check(lib().orc_padded(self.h, p, _dp(out), size))
        return out

    def slot(self, q, rel=0):
        n = self.patches[q].n
        out = np.empty(5 * n ** 3 + 3 * n * n * (n + 1))
        tk = C.c_int64()
        t = C.c_double()
        _check(lib().orc_slot(self.h, q, rel, _dp(out), out.size, C.byref(tk), C.byref(t)))
        return out, tk.value, t.value

    def jvp_fixed(self, U0, dU0, nsteps, dt):
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        dU0 = np.ascontiguousarray(dU0, dtype=np.float64)
        UT = np.empty_like(U0)
        dUT = np.empty_like(U0)
        _check(lib().orc_jvp_fixed(self.h, _dp(U0), _dp(dU0), nsteps, dt, _dp(UT), _dp(dUT)))
        return UT, dUT

    def count_flops(self, U0, t_end):
        """(floating-point operations, cell updates, operations of the
        Courant rate) of the method from U0 to t_end (+, -, *, / and sqrt
        count one each)."""
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        out = np.zeros(3)
        _check(lib().orc_count_flops(self.h, _dp(U0), float(t_end), _dp(out)))
        return out[0], out[1], out[2]


def hlld_flux(wl, wr, bn, gamma=5.0 / 3.0, eps=1e-12):
    """(mass, mn, mt1, mt2, energy, bt1, bt2) fluxes and, last, the upwind
    speed that orients the edge EMFs."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(8)
    _check(lib().orc_hlld_flux(_dp(wl), _dp(wr), float(bn), gamma, eps, _dp(f)))
    return f


def run(prob, t_end=None, order=0, nthreads=1, seed=1, **over):
    """Advance a Problem with the oracle; returns (state, steps, khash, stats)."""
    s = OracleSet.from_problem(prob, **over)
    s.set_order(order, seed, nthreads)
    s.advance_to(prob.t_end if t_end is None else t_end)
    U = s.read_state()
    steps, kh = s.read_schedule()
    st = s.stats()
    s.close()
    return U, steps, kh, st
