"""ctypes binding of the C ABI in include/swe_nh.h (same names, argument
marshalling only).  PyTorch provides device memory and the current HIP
stream; every step of the method runs in the HIP kernels of libswe_nh.so.

There is no fallback: importing this module on a machine where the HIP
library has not been built raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libswe_nh.so")

OK, EINVAL, ENOCONV, EDRY, ENAN, EHIP, ENOMEM = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOCONV", -3: "EDRY", -4: "ENAN", -5: "EHIP",
                -6: "ENOMEM"}


class swe_nh_body(C.Structure):
    _fields_ = [("kind", C.c_int32), ("law", C.c_int32), ("amp", C.c_double), ("len", C.c_double),
                ("x0", C.c_double), ("y0", C.c_double), ("dir", C.c_double),
                ("q", C.c_double * 5)]


class swe_nh_config(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("batch", C.c_int32),
                ("offsets", C.POINTER(C.c_int64)), ("dx", C.c_double), ("dy", C.c_double),
                ("g", C.c_double), ("rho", C.c_double), ("cfl", C.c_double),
                ("dt_fixed", C.c_double), ("crit", C.c_int32), ("k_nh", C.c_double),
                ("enlarge", C.c_int32), ("first_global", C.c_int32), ("precision", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("warm", C.c_int32),
                ("tile1d", C.c_int32), ("step1d_form", C.c_int32), ("tensor2d", C.c_int32),
                ("depth_static", C.c_void_p),
                ("bodies", C.POINTER(swe_nh_body))]


class swe_nh_dg1d_config(C.Structure):
    _fields_ = [("n", C.c_int32), ("dx", C.c_double), ("dt", C.c_double), ("g", C.c_double),
                ("rho", C.c_double), ("d_static", C.c_double), ("body", swe_nh_body),
                ("adaptive", C.c_int32), ("crit", C.c_int32), ("enlarge", C.c_int32),
                ("first_global", C.c_int32), ("k_nh", C.c_double),
                ("marked", C.POINTER(C.c_int32))]


class swe_nh_stats(C.Structure):
    _fields_ = [("n_active", C.c_int64), ("iters", C.c_int32), ("status", C.c_int32),
                ("rel_res", C.c_double), ("dt", C.c_double), ("t", C.c_double),
                ("steps", C.c_int64), ("iters_total", C.c_int64)]


class SweNhError(RuntimeError):
    def __init__(self, code, where, msg=""):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} {msg}".strip())
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.swe_nh_workspace_bytes.restype = C.c_size_t
    lib.swe_nh_workspace_bytes.argtypes = [C.POINTER(swe_nh_config)]
    lib.swe_nh_init.argtypes = [C.POINTER(swe_nh_config), vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.swe_nh_destroy.argtypes = [vp]
    lib.swe_nh_destroy.restype = None
    lib.swe_nh_last_error.argtypes = [vp]
    lib.swe_nh_last_error.restype = C.c_char_p
    lib.swe_nh_set_time.argtypes = [vp, C.POINTER(dbl)]
    lib.swe_nh_get_time.argtypes = [vp, C.POINTER(dbl)]
    lib.swe_nh_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, i32]
    lib.swe_nh_sync_stats.argtypes = [vp, C.POINTER(swe_nh_stats)]
    lib.swe_nh_step_t.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(swe_nh_stats)]
    lib.swe_nh_predict.argtypes = [vp, vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl), vp, vp, vp,
                                   vp]
    lib.swe_nh_mask.argtypes = [vp, vp, vp, vp, vp, C.POINTER(dbl), i32, vp, C.POINTER(i64)]
    lib.swe_nh_solve_pressure.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl),
                                          vp, C.POINTER(i32), C.POINTER(dbl)]
    lib.swe_nh_correct.argtypes = [vp, vp, vp, vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl), vp,
                                   vp, vp]
    lib.swe_nh_time_stage.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp, C.POINTER(dbl)]
    lib.swe_nh_cnn_param_count.restype = C.c_size_t
    lib.swe_nh_cnn_param_count.argtypes = []
    lib.swe_nh_cnn_workspace_bytes.restype = C.c_size_t
    lib.swe_nh_cnn_workspace_bytes.argtypes = [i32, i32, i32]
    lib.swe_nh_cnn_forward.argtypes = [vp, vp, i32, i32, i32, vp, vp, C.c_size_t, vp]
    lib.swe_nh_cnn_forward_noalloc.argtypes = [vp, vp, i32, i32, i32, vp, vp]
    lib.swe_nh_cnn_backward.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, C.c_size_t, vp]
    lib.swe_nh_cnn_mse.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, C.c_size_t, vp]
    lib.swe_nh_cnn_bce.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, C.c_size_t, vp]
    lib.swe_nh_cnn_adam.argtypes = [vp, vp, vp, vp, i64, i32, C.c_float, C.c_float, C.c_float,
                                    C.c_float, vp]
    lib.swe_nh_features.argtypes = [vp, vp, vp, vp, vp, C.POINTER(dbl), C.POINTER(dbl), vp]
    lib.swe_nh_set_warm_start_net.argtypes = [vp, vp, C.POINTER(dbl), dbl]
    lib.swe_nh_dg1d_run.argtypes = [C.POINTER(swe_nh_dg1d_config), dbl, i32, vp, vp, vp, vp, vp,
                                    vp]
    lib.swe_nh_dg1d_run_batch.argtypes = [C.POINTER(swe_nh_dg1d_config), i32, dbl, i32, vp, vp, vp,
                                          vp, vp, vp]
    for name in ("swe_nh_cnn_forward", "swe_nh_cnn_forward_noalloc", "swe_nh_cnn_backward",
                 "swe_nh_cnn_mse", "swe_nh_cnn_bce", "swe_nh_cnn_adam",
                 "swe_nh_features", "swe_nh_set_warm_start_net", "swe_nh_time_stage", "swe_nh_init", "swe_nh_set_time", "swe_nh_get_time", "swe_nh_step",
                 "swe_nh_sync_stats", "swe_nh_predict", "swe_nh_mask", "swe_nh_solve_pressure",
                 "swe_nh_correct", "swe_nh_dg1d_run", "swe_nh_dg1d_run_batch"):
        getattr(lib, name).restype = C.c_int
    return lib


LIB = _load()
EXPORTED = ["swe_nh_workspace_bytes", "swe_nh_init", "swe_nh_destroy", "swe_nh_last_error",
            "swe_nh_set_time", "swe_nh_get_time", "swe_nh_step", "swe_nh_step_t",
            "swe_nh_sync_stats",
            "swe_nh_predict", "swe_nh_mask", "swe_nh_solve_pressure", "swe_nh_correct",
            "swe_nh_time_stage", "swe_nh_cnn_param_count", "swe_nh_cnn_workspace_bytes",
            "swe_nh_cnn_forward", "swe_nh_cnn_forward_noalloc", "swe_nh_cnn_backward",
            "swe_nh_cnn_mse", "swe_nh_cnn_bce", "swe_nh_cnn_adam", "swe_nh_features",
            "swe_nh_set_warm_start_net",
            "swe_nh_dg1d_run", "swe_nh_dg1d_run_batch"]
NOALLOC_MAX_PIXELS = 131072
DG_MAX_ELEMS = 1024
DG_MAX_ENLARGE = 64
DG_MAX_BATCH = 65536


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("arguments must be contiguous device tensors")
    return C.c_void_p(t.data_ptr())


def _darr(vals):
    a = (C.c_double * len(vals))(*[float(v) for v in vals])
    return a


def body_struct(body) -> swe_nh_body:
    b = swe_nh_body()
    b.kind, b.law = int(body.kind), int(body.law)
    b.amp, b.len, b.x0, b.y0, b.dir = body.amp, body.length, body.x0, body.y0, body.dir
    for i in range(5):
        b.q[i] = float(body.q[i])
    return b


class Context:
    """owns a swe_nh_ctx, its workspace tensor and the tensors its config points to"""

    def __init__(self, *, dim, nx, ny=1, dx, dy=0.0, depth_static: torch.Tensor,
                 bodies: Sequence, offsets: Optional[Sequence[int]] = None, g=9.81, rho=1000.0,
                 cfl=0.5, dt_fixed=0.0, crit=6, k_nh=1e-3, enlarge=1, first_global=1,
                 precision=0, tol=1e-12, max_iter=8, warm=1, tile1d=0, step1d_form=0, tensor2d=0,
                 device="cuda"):
        self.device = torch.device(device)
        self.depth = depth_static.to(self.device, torch.float64).contiguous()
        self._bodies = (swe_nh_body * len(bodies))(*[body_struct(b) for b in bodies])
        cfg = swe_nh_config()
        cfg.dim, cfg.nx, cfg.ny = dim, nx, ny
        cfg.batch = len(bodies) if dim == 1 else 1
        if offsets is not None:
            self._offsets = (C.c_int64 * len(offsets))(*[int(o) for o in offsets])
            cfg.offsets = self._offsets
        else:
            self._offsets = None
            cfg.offsets = None
        cfg.dx, cfg.dy, cfg.g, cfg.rho = dx, dy, g, rho
        cfg.cfl, cfg.dt_fixed = cfl, dt_fixed
        cfg.crit, cfg.k_nh, cfg.enlarge, cfg.first_global = crit, k_nh, enlarge, first_global
        cfg.precision, cfg.tol, cfg.max_iter, cfg.warm = precision, tol, max_iter, warm
        cfg.tile1d = tile1d
        cfg.step1d_form = step1d_form
        cfg.tensor2d = tensor2d
        cfg.depth_static = C.c_void_p(self.depth.data_ptr())
        cfg.bodies = self._bodies
        self.cfg = cfg
        self.nch = cfg.batch
        nbytes = LIB.swe_nh_workspace_bytes(C.byref(cfg))
        if nbytes == 0:
            raise SweNhError(EINVAL, "swe_nh_workspace_bytes", "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        stream = torch.cuda.current_stream(self.device).cuda_stream
        ctx = C.c_void_p()
        rc = LIB.swe_nh_init(C.byref(cfg), C.c_void_p(aligned), C.c_size_t(nbytes),
                             C.c_void_p(stream), C.byref(ctx))
        if rc != OK:
            raise SweNhError(rc, "swe_nh_init")
        self.ctx = ctx

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx and LIB is not None:
            try:
                LIB.swe_nh_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    def _check(self, rc, where):
        if rc != OK:
            raise SweNhError(rc, where, LIB.swe_nh_last_error(self.ctx).decode())

    # ---- time ----
    def set_time(self, t):
        t = [t] * self.nch if np.isscalar(t) else list(t)
        self._check(LIB.swe_nh_set_time(self.ctx, _darr(t)), "swe_nh_set_time")

    def get_time(self):
        out = (C.c_double * self.nch)()
        self._check(LIB.swe_nh_get_time(self.ctx, out), "swe_nh_get_time")
        return np.array(out[:])

    # ---- whole step ----
    def step(self, h, hu, hv, hw, p, mask=None, nsteps=1):
        self._check(LIB.swe_nh_step(self.ctx, _ptr(h), _ptr(hu), _ptr(hv), _ptr(hw), _ptr(p),
                                    _ptr(mask), int(nsteps)), "swe_nh_step")

    def step_t(self, h, hu, hv, hw, p, t_dev, stats=True):
        """swe_nh_step_t: one step with the time in the device tensor t_dev;
        returns the statistics (synchronising) or None"""
        st = swe_nh_stats() if stats else None
        self._check(LIB.swe_nh_step_t(self.ctx, _ptr(h), _ptr(hu), _ptr(hv), _ptr(hw), _ptr(p),
                                      _ptr(t_dev), C.byref(st) if st is not None else None),
                    "swe_nh_step_t")
        return {k: getattr(st, k) for k, _ in swe_nh_stats._fields_} if st is not None else None

    def sync_stats(self):
        st = swe_nh_stats()
        self._check(LIB.swe_nh_sync_stats(self.ctx, C.byref(st)), "swe_nh_sync_stats")
        return {k: getattr(st, k) for k, _ in swe_nh_stats._fields_}

    def time_stage(self, stage, nreps, h, hu, hv, hw, p):
        us = C.c_double()
        self._check(LIB.swe_nh_time_stage(self.ctx, int(stage), int(nreps), _ptr(h), _ptr(hu),
                                          _ptr(hv), _ptr(hw), _ptr(p), C.byref(us)),
                    "swe_nh_time_stage")
        return us.value

    def features(self, ht, mt, nt, mask, t1, scales, out):
        self._check(LIB.swe_nh_features(self.ctx, _ptr(ht), _ptr(mt), _ptr(nt), _ptr(mask),
                                        self._times(t1), _darr(scales), _ptr(out)),
                    "swe_nh_features")

    def set_warm_start_net(self, params, scales, p_scale):
        self._net = params  # the library keeps the pointer
        self._check(LIB.swe_nh_set_warm_start_net(self.ctx, _ptr(params), _darr(scales),
                                                  float(p_scale)), "swe_nh_set_warm_start_net")

    # ---- stages ----
    def _times(self, t):
        return _darr([t] * self.nch if np.isscalar(t) else list(t))

    def predict(self, h, hu, hv, hw, t, dt, ht, mt, nt, kt):
        self._check(LIB.swe_nh_predict(self.ctx, _ptr(h), _ptr(hu), _ptr(hv), _ptr(hw),
                                       self._times(t), self._times(dt), _ptr(ht), _ptr(mt),
                                       _ptr(nt), _ptr(kt)), "swe_nh_predict")

    def mask(self, ht, mt, nt, kt, t1, first_step, mask_out):
        na = C.c_int64()
        self._check(LIB.swe_nh_mask(self.ctx, _ptr(ht), _ptr(mt), _ptr(nt), _ptr(kt),
                                    self._times(t1), int(first_step), _ptr(mask_out),
                                    C.byref(na)), "swe_nh_mask")
        return na.value

    def solve_pressure(self, ht, mt, nt, kt, mask, t, dt, p):
        it, rr = C.c_int32(), C.c_double()
        self._check(LIB.swe_nh_solve_pressure(self.ctx, _ptr(ht), _ptr(mt), _ptr(nt), _ptr(kt),
                                              _ptr(mask), self._times(t), self._times(dt),
                                              _ptr(p), C.byref(it), C.byref(rr)),
                    "swe_nh_solve_pressure")
        return it.value, rr.value

    def correct(self, ht, mt, nt, kt, mask, p, t, dt, m_out, n_out, k_out):
        self._check(LIB.swe_nh_correct(self.ctx, _ptr(ht), _ptr(mt), _ptr(nt), _ptr(kt),
                                       _ptr(mask), _ptr(p), self._times(t), self._times(dt),
                                       _ptr(m_out), _ptr(n_out), _ptr(k_out)), "swe_nh_correct")


def context_1d(case_or_ensemble, **kw) -> Context:
    """Context for one 1D case (swe_inputs.Case1D) or an ensemble of channels"""
    if hasattr(case_or_ensemble, "channels"):
        ens = case_or_ensemble
        ds = torch.from_numpy(ens.packed("ds"))
        return Context(dim=1, nx=int(ens.offsets[-1]), dx=ens.channels[0].dx, depth_static=ds,
                       bodies=[c.body for c in ens.channels], offsets=list(ens.offsets), **kw)
    c = case_or_ensemble
    return Context(dim=1, nx=c.n, dx=c.dx, depth_static=torch.from_numpy(np.asarray(c.ds)),
                   bodies=[c.body], **kw)


def context_2d(case, **kw) -> Context:
    return Context(dim=2, nx=case.nx, ny=case.ny, dx=case.dx, dy=case.dy,
                   depth_static=torch.from_numpy(np.asarray(case.ds)), bodies=[case.body], **kw)


def cnn_forward_noalloc(params, x, n, h, w, out):
    """swe_nh_cnn_forward_noalloc on the current stream; returns the status code"""
    stream = torch.cuda.current_stream(out.device).cuda_stream
    return int(LIB.swe_nh_cnn_forward_noalloc(_ptr(params), _ptr(x), int(n), int(h), int(w),
                                              _ptr(out), C.c_void_p(stream)))


def dg1d_config(n, dx, dt, d_static, body, g=9.81, rho=1000.0, crit=None, k_nh=1e-3, enlarge=0,
                first_global=False, marked=None, nsteps=None):
    """a swe_nh_dg1d_config: crit None is the global model, else the adaptive
    model with that criterion (marked: optional device int32 tensor of at
    least nsteps per-step counts)"""
    cfg = swe_nh_dg1d_config()
    cfg.n, cfg.dx, cfg.dt, cfg.g, cfg.rho, cfg.d_static = int(n), dx, dt, g, rho, d_static
    cfg.body = body_struct(body)
    if crit is not None:
        cfg.adaptive, cfg.crit, cfg.enlarge = 1, int(crit), int(enlarge)
        cfg.first_global, cfg.k_nh = int(bool(first_global)), float(k_nh)
        if marked is not None:
            if marked.dtype != torch.int32 or nsteps is None or marked.numel() < int(nsteps):
                raise ValueError("marked must be a device int32 tensor of at least nsteps")
            cfg.marked = C.cast(_ptr(marked), C.POINTER(C.c_int32))
    return cfg


def dg1d_run(n, dx, dt, d_static, body, t0, nsteps, h, hu, hw, p, status, g=9.81, rho=1000.0,
             crit=None, k_nh=1e-3, enlarge=0, first_global=False, marked=None):
    """swe_nh_dg1d_run on the current stream: h, hu, hw, p device [n, 2]
    (FP64), status a device int32 scratch word; crit None: the global model,
    else the adaptive model with that criterion (marked: optional device
    int32 [nsteps] of per-step counts); returns the status code"""
    cfg = dg1d_config(n, dx, dt, d_static, body, g, rho, crit, k_nh, enlarge, first_global,
                      marked, nsteps)
    stream = torch.cuda.current_stream(h.device).cuda_stream
    return int(LIB.swe_nh_dg1d_run(C.byref(cfg), float(t0), int(nsteps), _ptr(h), _ptr(hu),
                                   _ptr(hw), _ptr(p), _ptr(status), C.c_void_p(stream)))


def dg1d_run_batch(cfgs, t0, nsteps, h, hu, hw, p, status):
    """swe_nh_dg1d_run_batch on the current stream: cfgs a list of
    swe_nh_dg1d_config (dg1d_config), h, hu, hw, p device FP64 tensors of all
    channels' node values packed in channel order ([sum n, 2]); returns the
    status code"""
    arr = (swe_nh_dg1d_config * len(cfgs))(*cfgs)
    tot = sum(int(c.n) for c in cfgs)
    for t in (h, hu, hw, p):
        if t.dtype != torch.float64 or t.numel() < 2 * tot:
            raise ValueError("node arrays must be FP64 device tensors of 2 x total elements")
    stream = torch.cuda.current_stream(h.device).cuda_stream
    return int(LIB.swe_nh_dg1d_run_batch(arr, len(cfgs), float(t0), int(nsteps), _ptr(h),
                                         _ptr(hu), _ptr(hw), _ptr(p), _ptr(status),
                                         C.c_void_p(stream)))


class Net:
    """the warm-start network's kernels on caller-owned device buffers"""

    def __init__(self, n, h, w, device="cuda"):
        self.n, self.h, self.w = n, h, w
        nb = LIB.swe_nh_cnn_workspace_bytes(n, h, w)
        if nb == 0:
            raise SweNhError(EINVAL, "swe_nh_cnn_workspace_bytes", f"shape {n}x{h}x{w}")
        self.ws = torch.empty(nb + 256, dtype=torch.uint8, device=device)
        self.wsp = (self.ws.data_ptr() + 255) // 256 * 256
        self.nbytes = nb
        self.stream = torch.cuda.current_stream(torch.device(device)).cuda_stream

    @staticmethod
    def param_count():
        return int(LIB.swe_nh_cnn_param_count())

    def _ok(self, rc, where):
        if rc != OK:
            raise SweNhError(rc, where)

    def forward(self, params, x, out):
        self._ok(LIB.swe_nh_cnn_forward(_ptr(params), _ptr(x), self.n, self.h, self.w, _ptr(out),
                                        C.c_void_p(self.wsp), C.c_size_t(self.nbytes),
                                        C.c_void_p(self.stream)), "swe_nh_cnn_forward")

    def backward(self, params, x, dout, grad):
        self._ok(LIB.swe_nh_cnn_backward(_ptr(params), _ptr(x), _ptr(dout), self.n, self.h,
                                         self.w, _ptr(grad), C.c_void_p(self.wsp),
                                         C.c_size_t(self.nbytes), C.c_void_p(self.stream)),
                 "swe_nh_cnn_backward")

    def mse(self, out, target, weight, dout, loss):
        self._ok(LIB.swe_nh_cnn_mse(_ptr(out), _ptr(target), _ptr(weight), self.n, self.h, self.w,
                                    _ptr(dout), _ptr(loss), C.c_void_p(self.wsp),
                                    C.c_size_t(self.nbytes), C.c_void_p(self.stream)),
                 "swe_nh_cnn_mse")

    def bce(self, out, target, weight, dout, loss):
        self._ok(LIB.swe_nh_cnn_bce(_ptr(out), _ptr(target), _ptr(weight), self.n, self.h, self.w,
                                    _ptr(dout), _ptr(loss), C.c_void_p(self.wsp),
                                    C.c_size_t(self.nbytes), C.c_void_p(self.stream)),
                 "swe_nh_cnn_bce")

    def adam(self, params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._ok(LIB.swe_nh_cnn_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                     int(params.numel()), int(step), float(lr), float(beta1),
                                     float(beta2), float(eps), C.c_void_p(self.stream)),
                 "swe_nh_cnn_adam")
