"""Thin ctypes binding of libdsp.so (include/dsp.h): argument marshalling only.

Every function keeps the C name (dsp_create, dsp_init, dsp_advance_to, ...);
`PatchSet` wraps a handle.  Every step of the patch update runs in the HIP
kernels of libdsp.so; if the library is missing or cannot be loaded the
import of this module's functions raises.  PyTorch only provides the HIP
stream the set runs on and the device tensors of the fixed-step entries.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsp.so")
_lib = None

DSP_OK, DSP_EINVAL, DSP_ENOMEM, DSP_EHIP, DSP_EKMAX, DSP_EALIGN, DSP_ENONFINITE, DSP_ENEGATIVE, DSP_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
DSP_F32, DSP_F64 = 1, 2
DSP_DT_LOCAL, DSP_DT_GLOBAL_QUANT, DSP_DT_GLOBAL_EXACT, DSP_DT_FIXED = 0, 1, 2, 3

# every entry point declared in include/dsp.h
EXPORTS = ["dsp_create", "dsp_init", "dsp_init_device", "dsp_advance_to", "dsp_advance_to_plain", "dsp_read_state",
           "dsp_read_schedule", "dsp_stats", "dsp_kernel_time", "dsp_kernel_stats", "dsp_fixed_steps_fwd",
           "dsp_fixed_steps_adj", "dsp_save_snapshot", "dsp_load_snapshot", "dsp_hlld_faces",
           "dsp_hlld_faces_noalloc", "dsp_set_dispatch", "dsp_get_dispatch", "dsp_autotune", "dsp_set_output",
           "dsp_destroy",
           "dsp_last_error"]
DSP_DISPATCH_ROUNDS, DSP_DISPATCH_QUEUE = 0, 1


class dsp_config(C.Structure):
    _fields_ = [("gamma", C.c_double), ("courant", C.c_double), ("dt_base", C.c_double),
                ("dt_fixed", C.c_double), ("grace", C.c_double), ("p_floor", C.c_double),
                ("kmax", C.c_int32), ("nslots", C.c_int32), ("nguard", C.c_int32),
                ("limiter", C.c_int32), ("prec", C.c_int32), ("dt_mode", C.c_int32),
                ("periodic", C.c_int32 * 3), ("box_lo", C.c_double * 3), ("box_hi", C.c_double * 3),
                ("eta", C.c_double), ("gamma_ad", C.c_double), ("rho_ion", C.c_double), ("torder", C.c_int32)]


class dsp_patch_desc(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("size", C.c_double * 3), ("n", C.c_int32),
                ("level", C.c_int32), ("flags", C.c_int32)]


class DspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdsp error {code}: {msg}")
        self.code = code


def load():
    """Load libdsp.so (built in place by csrc/build.py if it is absent)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch ships its own libamdhip64.so.7; when it
    # is imported first, the dynamic loader binds libdsp.so to that copy (same
    # soname) instead of loading a second runtime from /opt/rocm.
    try:
        import torch  # noqa: F401
    except Exception:  # pragma: no cover - torch absent: system runtime
        pass
    if not os.path.exists(LIB_PATH):
        from .csrc import build as _b
        _b.build()
    L = C.CDLL(LIB_PATH)
    vp, dp, sz = C.c_void_p, C.POINTER(C.c_double), C.c_size_t
    L.dsp_create.argtypes = [C.POINTER(dsp_config), C.POINTER(dsp_patch_desc), C.c_int32, vp, vp,
                             C.POINTER(vp)]
    L.dsp_init.argtypes = [vp, dp, sz, C.c_double]
    L.dsp_init_device.argtypes = [vp, vp, C.c_double]
    L.dsp_advance_to.argtypes = [vp, C.c_double]
    L.dsp_advance_to_plain.argtypes = [vp, C.c_double]
    L.dsp_read_state.argtypes = [vp, dp, sz, dp]
    L.dsp_read_schedule.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_int32), sz]
    L.dsp_stats.argtypes = [vp, dp]
    L.dsp_kernel_time.argtypes = [vp, dp, C.POINTER(C.c_int64)]
    L.dsp_kernel_stats.argtypes = [vp, dp]
    L.dsp_fixed_steps_fwd.argtypes = [vp, vp, vp, C.c_int32, vp]
    L.dsp_fixed_steps_adj.argtypes = [vp, vp, vp, vp, C.c_int32, C.c_int32]
    L.dsp_save_snapshot.argtypes = [vp, C.c_char_p]
    L.dsp_load_snapshot.argtypes = [vp, C.c_char_p]
    L.dsp_hlld_faces.argtypes = [C.c_int32, dp, dp, dp, C.c_int64, C.c_double, dp]
    L.dsp_hlld_faces_noalloc.argtypes = [C.c_int32, dp, dp, dp, C.c_int64, C.c_double, dp]
    L.dsp_set_dispatch.argtypes = [vp, C.c_int32, C.c_int32]
    L.dsp_get_dispatch.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    L.dsp_autotune.argtypes = [vp, C.c_double, C.c_char_p, dp]
    L.dsp_set_output.argtypes = [vp, C.c_double, vp, C.c_int32]
    L.dsp_destroy.argtypes = [vp]
    L.dsp_destroy.restype = None
    L.dsp_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise DspError(rc, load().dsp_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(cfg) -> dsp_config:
    c = dsp_config()
    for f in ("gamma", "courant", "dt_base", "dt_fixed", "grace", "p_floor", "kmax", "nslots",
              "nguard", "limiter", "prec", "dt_mode", "eta", "gamma_ad", "rho_ion", "torder"):
        setattr(c, f, getattr(cfg, f))
    for d in range(3):
        c.periodic[d] = int(cfg.periodic[d])
        c.box_lo[d] = cfg.box_lo[d]
        c.box_hi[d] = cfg.box_hi[d]
    return c


def make_descs(patches):
    arr = (dsp_patch_desc * len(patches))()
    for i, p in enumerate(patches):
        for d in range(3):
            arr[i].origin[d] = p.origin[d]
            arr[i].size[d] = p.size
        arr[i].n = p.n
        arr[i].level = p.level
        arr[i].flags = 1 if p.frozen else 0
    return arr


def _torch_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - no torch / no GPU
        pass
    return None


# --- functions with the C names ------------------------------------------------

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class dsp_allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def torch_allocator():
    """A dsp_allocator over torch's caching allocator (current device and
    stream).  The returned object must outlive every set created with it."""
    import torch

    def alloc(ctx, nbytes):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:  # out of memory: dsp_create reports DSP_ENOMEM
            return None

    def free(ctx, ptr):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC_FN(alloc), _FREE_FN(free)
    st = dsp_allocator(None, a, f)
    st._keep = (a, f)  # the callbacks live as long as the structure
    return st


def dsp_create(cfg, patches, stream=None, allocator=None):
    c = make_config(cfg)
    d = make_descs(patches)
    h = C.c_void_p()
    _check(load().dsp_create(C.byref(c), d, len(patches), stream,
                             C.byref(allocator) if allocator is not None else None, C.byref(h)))
    return h


def dsp_init(h, U, t0=0.0):
    U = np.ascontiguousarray(U, dtype=np.float64)
    _check(load().dsp_init(h, _dp(U), U.size, float(t0)))


def dsp_init_device(h, U_dev, t0=0.0):
    _check(load().dsp_init_device(h, C.c_void_p(U_dev), float(t0)))


def dsp_advance_to(h, t_end):
    _check(load().dsp_advance_to(h, float(t_end)))


def dsp_advance_to_plain(h, t_end):
    _check(load().dsp_advance_to_plain(h, float(t_end)))


def dsp_read_state(h, nvals):
    U = np.empty(nvals)
    t = C.c_double()
    _check(load().dsp_read_state(h, _dp(U), U.size, C.byref(t)))
    return U, t.value


def dsp_read_schedule(h, npatch, klog_cap=0):
    steps = np.zeros(npatch, dtype=np.int64)
    kh = np.zeros(npatch, dtype=np.uint64)
    kl = np.zeros(npatch * max(klog_cap, 1), dtype=np.int32)
    _check(load().dsp_read_schedule(h, steps.ctypes.data_as(C.POINTER(C.c_int64)),
                                    kh.ctypes.data_as(C.POINTER(C.c_uint64)),
                                    kl.ctypes.data_as(C.POINTER(C.c_int32)) if klog_cap else None,
                                    klog_cap))
    return (steps, kh, kl.reshape(npatch, klog_cap)) if klog_cap else (steps, kh)


def dsp_stats(h):
    out = np.zeros(16)
    _check(load().dsp_stats(h, _dp(out)))
    return out


def dsp_kernel_time(h):
    ms = C.c_double()
    n = C.c_int64()
    _check(load().dsp_kernel_time(h, C.byref(ms), C.byref(n)))
    return ms.value, n.value


def dsp_kernel_stats(h):
    out = np.zeros(4)
    _check(load().dsp_kernel_stats(h, _dp(out)))
    return out


def dsp_fixed_steps_fwd(h, U0_dev, UT_dev, nsteps, ckpt_dev=None):
    _check(load().dsp_fixed_steps_fwd(h, C.c_void_p(U0_dev), C.c_void_p(UT_dev), int(nsteps),
                                      C.c_void_p(ckpt_dev) if ckpt_dev else None))


def dsp_fixed_steps_adj(h, ckpt_dev, lamT_dev, lam0_dev, nsteps, seg=8):
    _check(load().dsp_fixed_steps_adj(h, C.c_void_p(ckpt_dev), C.c_void_p(lamT_dev),
                                      C.c_void_p(lam0_dev), int(nsteps), int(seg)))


def dsp_save_snapshot(h, path):
    _check(load().dsp_save_snapshot(h, str(path).encode()))


def dsp_load_snapshot(h, path):
    _check(load().dsp_load_snapshot(h, str(path).encode()))


def dsp_hlld_faces(prec, wl, wr, bn, gamma=5.0 / 3.0, noalloc=False):
    """Fluxes [nface, 8] of faces with states wl, wr [nface, 7] and normal
    field bn [nface] (see include/dsp.h); noalloc: the entry point that
    stages in the library's fixed device array instead of allocating."""
    wl = np.ascontiguousarray(wl, dtype=np.float64).reshape(-1, 7)
    wr = np.ascontiguousarray(wr, dtype=np.float64).reshape(-1, 7)
    bn = np.ascontiguousarray(bn, dtype=np.float64).reshape(-1)
    if not (wl.shape[0] == wr.shape[0] == bn.shape[0]):
        raise ValueError("wl, wr and bn must describe the same number of faces")
    out = np.empty((bn.shape[0], 8))
    fn = load().dsp_hlld_faces_noalloc if noalloc else load().dsp_hlld_faces
    _check(fn(int(prec), _dp(wl), _dp(wr), _dp(bn), bn.shape[0], float(gamma), _dp(out)))
    return out


def dsp_set_dispatch(h, mode, workers=0):
    _check(load().dsp_set_dispatch(h, int(mode), int(workers)))


def dsp_get_dispatch(h):
    """(mode, queue available, workers)"""
    m, a, w = C.c_int32(), C.c_int32(), C.c_int32()
    _check(load().dsp_get_dispatch(h, C.byref(m), C.byref(a), C.byref(w)))
    return m.value, bool(a.value), w.value


def dsp_autotune(h, t_probe, cache_path=None):
    """Times the dispatch candidates (ms per candidate, -1 where not one)."""
    out = np.zeros(4)
    _check(load().dsp_autotune(h, float(t_probe), str(cache_path).encode() if cache_path else None, _dp(out)))
    return out


def dsp_set_output(h, out_dt, frames_ptr, nframes):
    _check(load().dsp_set_output(h, float(out_dt), frames_ptr, int(nframes)))


def dsp_destroy(h):
    if h:
        load().dsp_destroy(h)


class PatchSet:
    """A patch set on the GPU (owns a dsp_set handle)."""

    def __init__(self, cfg, patches, stream="torch", allocator=None):
        """allocator: None (hipMalloc), or "torch" (torch's caching allocator,
        so the set's device memory shows in torch's memory statistics)."""
        self.cfg, self.patches = cfg, list(patches)
        self.nvals = int(sum(5 * p.n ** 3 + 3 * p.n * p.n * (p.n + 1) for p in self.patches))
        s = _torch_stream() if stream == "torch" else stream
        self._alloc = torch_allocator() if allocator == "torch" else allocator
        self.h = dsp_create(cfg, self.patches, s, self._alloc)

    @classmethod
    def from_problem(cls, prob, allocator=None, **over):
        import dataclasses
        cfg = dataclasses.replace(prob.cfg, **over) if over else prob.cfg
        s = cls(cfg, prob.patches, allocator=allocator)
        s.init(prob.U0)
        return s

    def close(self):
        if getattr(self, "h", None):
            dsp_destroy(self.h)
            self.h = None

    __del__ = close

    def init(self, U, t0=0.0):
        dsp_init(self.h, U, t0)

    def init_device(self, U_dev, t0=0.0):
        dsp_init_device(self.h, U_dev, t0)

    def advance_to(self, t):
        dsp_advance_to(self.h, t)

    def advance_to_plain(self, t):
        dsp_advance_to_plain(self.h, t)

    def read_state(self):
        return dsp_read_state(self.h, self.nvals)[0]

    def read_schedule(self, klog_cap=0):
        return dsp_read_schedule(self.h, len(self.patches), klog_cap)

    def stats(self):
        return dsp_stats(self.h)

    def kernel_time(self):
        return dsp_kernel_time(self.h)

    def kernel_stats(self):
        return dsp_kernel_stats(self.h)

    def save(self, path):
        dsp_save_snapshot(self.h, path)

    def set_dispatch(self, mode, workers=0):
        dsp_set_dispatch(self.h, mode, workers)

    def dispatch(self):
        return dsp_get_dispatch(self.h)

    def autotune(self, t_probe, cache_path=None):
        return dsp_autotune(self.h, t_probe, cache_path)

    def load(self, path):
        dsp_load_snapshot(self.h, path)

    def set_output(self, out_dt, nframes):
        """Output cadence: returns the device tensor [nframes, values] (the
        set's precision, host layout) that each patch fills with its slice at
        every multiple of out_dt; nframes = 0 turns it off."""
        import torch
        if nframes <= 0:
            dsp_set_output(self.h, out_dt, None, 0)
            self._frames = None
            return None
        frames = torch.full((nframes, self.nvals), float("nan"), dtype=self._dtype(), device="cuda")
        dsp_set_output(self.h, out_dt, frames.data_ptr(), nframes)
        self._frames = frames  # kept alive while the cadence is set
        return frames

    # ---- fixed-dt steps and their adjoint (device tensors in the host layout)

    def _dtype(self):
        import torch
        return torch.float32 if self.cfg.prec == 1 else torch.float64

    def fixed_steps_fwd(self, U0, nsteps, checkpoints=True):
        """nsteps fixed steps from the device tensor U0 (host layout, the set's
        precision).  Returns (UT, ckpt): ckpt holds the state every 8 steps
        (None if checkpoints is False)."""
        import torch
        U0 = U0.contiguous()
        if U0.dtype != self._dtype() or U0.numel() != self.nvals or not U0.is_cuda:
            raise ValueError("U0 must be a device tensor of the set's precision and size")
        UT = torch.empty_like(U0)
        ckpt = torch.empty((nsteps // 8 + 1, self.nvals), dtype=U0.dtype, device=U0.device) if checkpoints else None
        dsp_fixed_steps_fwd(self.h, U0.data_ptr(), UT.data_ptr(), nsteps,
                            ckpt.data_ptr() if ckpt is not None else None)
        return UT, ckpt

    def fixed_steps_adj(self, ckpt, lamT, nsteps):
        """dJ/dU0 from dJ/dUT (device tensors) through nsteps fixed steps,
        recomputing forward states from the checkpoints."""
        import torch
        lamT = lamT.contiguous().to(self._dtype())
        lam0 = torch.empty_like(lamT)
        dsp_fixed_steps_adj(self.h, ckpt.data_ptr(), lamT.data_ptr(), lam0.data_ptr(), nsteps, 8)
        return lam0


def fixed_steps(pset, U0, nsteps):
    """Differentiable nsteps fixed-dt steps of the patch set: UT = F(U0), with
    the gradient from the hand-written adjoint (checkpoints every 8 steps)."""
    import torch

    class _FixedSteps(torch.autograd.Function):
        @staticmethod
        def forward(ctx, u0):
            UT, ckpt = pset.fixed_steps_fwd(u0.detach(), nsteps, checkpoints=True)
            ctx.save_for_backward(ckpt)
            return UT

        @staticmethod
        def backward(ctx, gUT):
            (ckpt,) = ctx.saved_tensors
            return pset.fixed_steps_adj(ckpt, gUT, nsteps)

    return _FixedSteps.apply(U0)
