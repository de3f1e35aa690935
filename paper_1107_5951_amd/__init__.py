"""MI355X fast-multipole gravity forward model: Python binding of libgrav.

The functions mirror the C ABI of ``include/grav.h`` (``grav_plan``,
``grav_eval``, ``grav_adjoint`` ...) and only marshal arguments: rho, g and
the residuals are torch tensors on the HIP device, passed by data pointer
together with the current HIP stream.  :class:`GravFMM` wraps evaluation
and its hand-written adjoint as a ``torch.autograd.Function``.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import GRAV_FP64, GRAV_MIXED, GravError, check, load

__all__ = [
    "GRAV_FP64", "GRAV_MIXED", "GravError", "PlanSpec", "Plan", "GravFMM", "grav_plan",
    "grav_eval", "grav_adjoint", "grav_operator", "grav_harmonics", "grav_plan_bytes",
    "grav_plan_info", "load",
]


@dataclass
class PlanSpec:
    """Fields of ``grav_plan_desc``; points is an ``[n, 3]`` float64 array or
    None.  sources (``[n, 3]``) replaces the cells' quadrature points by
    explicit point sources inside the mesh box; source_volumes (``[n]``)
    makes the density values per-source densities (mass = value * volume),
    without it they are masses."""
    n: Sequence[int]
    h: float
    origin: Sequence[float] = (0.0, 0.0, 0.0)
    quad_order: int = 1
    points: Optional[np.ndarray] = None
    voxel_centres: bool = False
    components: int = 3
    p: int = 8
    leaf_size: int = 64
    precision: int = GRAV_FP64
    batch: int = 1
    G: float = 1.0
    device: int = 0
    sources: Optional[np.ndarray] = None
    source_volumes: Optional[np.ndarray] = None

    def to_desc(self):
        lib = load()
        d = _lib.GravDesc()
        lib.grav_desc_init(ctypes.byref(d))
        d.nx, d.ny, d.nz = (int(v) for v in self.n)
        for a in range(3):
            d.origin[a] = float(self.origin[a])
        d.h = float(self.h)
        d.quad_order = int(self.quad_order)
        keep = None
        if self.points is not None and len(self.points):
            keep = np.ascontiguousarray(self.points, dtype=np.float64).reshape(-1, 3)
            d.n_points = keep.shape[0]
            d.points = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.voxel_centres = 1 if self.voxel_centres else 0
        d.components = int(self.components)
        d.p = int(self.p)
        d.leaf_size = int(self.leaf_size)
        d.precision = int(self.precision)
        d.batch = int(self.batch)
        d.G = float(self.G)
        d.device = int(self.device)
        keep = [keep]
        if self.sources is not None and len(self.sources):
            src = np.ascontiguousarray(self.sources, dtype=np.float64).reshape(-1, 3)
            d.n_sources = src.shape[0]
            d.sources = src.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            keep.append(src)
            if self.source_volumes is not None:
                vol = np.ascontiguousarray(self.source_volumes, dtype=np.float64).reshape(-1)
                if vol.shape[0] != src.shape[0]:
                    raise ValueError("source_volumes must have one entry per source")
                d.source_volumes = vol.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                keep.append(vol)
        return d, keep


def _stream_ptr(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Plan:
    """Owner of a ``grav_plan_t``; destroyed with the object."""

    def __init__(self, spec: PlanSpec):
        lib = load()
        desc, keep = spec.to_desc()
        h = ctypes.c_void_p()
        check(lib.grav_plan(ctypes.byref(desc), ctypes.byref(h)), "grav_plan")
        del keep  # grav_plan copied the points
        self._h = h
        self.spec = spec
        n_t, lev, lc, nl = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        check(lib.grav_plan_info(h, ctypes.byref(n_t), ctypes.byref(lev), ctypes.byref(lc),
                                 ctypes.byref(nl)), "grav_plan_info")
        self.n_targets = n_t.value
        self.levels = lev.value
        self.leaf_cells = lc.value
        self.n_target_leaves = nl.value

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            load().grav_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def out_shape(self):
        return (self.spec.batch, self.n_targets, self.spec.components)

    @property
    def rho_shape(self):
        if self.spec.sources is not None and len(self.spec.sources):
            return (self.spec.batch, int(np.asarray(self.spec.sources).reshape(-1, 3).shape[0]))
        n = self.spec.n
        return (self.spec.batch, int(n[2]), int(n[1]), int(n[0]))

    def bytes(self):
        r, c = ctypes.c_size_t(), ctypes.c_size_t()
        check(load().grav_plan_bytes(self.handle, ctypes.byref(r), ctypes.byref(c)), "grav_plan_bytes")
        return r.value, c.value

    def work(self):
        """(M2L box pairs, P2P point pairs, source points), per density model."""
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        check(load().grav_plan_work(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "grav_plan_work")
        return a.value, b.value, c.value

    def check(self) -> str:
        """Host validation of the plan's index tables ('ok' or the first violation)."""
        buf = ctypes.create_string_buffer(512)
        load().grav_plan_check(self.handle, buf, 512)
        return buf.value.decode()

    def eval(self, rho, out=None, stream=None):
        """g = A rho for a float64 device tensor rho [B, nz, ny, nx] (or [nz, ny, nx])."""
        import torch
        squeeze = rho.dim() == 3
        r = rho.reshape(self.rho_shape)
        if r.dtype != torch.float64 or not r.is_cuda or not r.is_contiguous():
            raise ValueError("rho must be a contiguous float64 HIP tensor of shape %s" % (self.rho_shape,))
        if out is None:
            out = torch.empty(self.out_shape, dtype=torch.float64, device=r.device)
        grav_eval(self, r, out, stream)
        return out[0] if squeeze else out

    def direct(self, rho, out=None, stream=None):
        """g by direct summation over all quadrature points (grav_direct), same layout as eval."""
        import torch
        squeeze = rho.dim() == 3
        r = rho.reshape(self.rho_shape)
        if r.dtype != torch.float64 or not r.is_cuda or not r.is_contiguous():
            raise ValueError("rho must be a contiguous float64 HIP tensor of shape %s" % (self.rho_shape,))
        if out is None:
            out = torch.empty(self.out_shape, dtype=torch.float64, device=r.device)
        grav_direct(self, r, out, stream)
        return out[0] if squeeze else out

    def analytic(self, rho, out=None, stream=None):
        """gz by the closed-form summation method (grav_analytic): exact for a
        cell-wise constant density; plans with components=1 only.  Output
        [B, M, 1] (or [M, 1]), like eval."""
        import torch
        squeeze = rho.dim() == 3
        r = rho.reshape(self.rho_shape)
        if r.dtype != torch.float64 or not r.is_cuda or not r.is_contiguous():
            raise ValueError("rho must be a contiguous float64 HIP tensor of shape %s" % (self.rho_shape,))
        if out is None:
            out = torch.empty(self.out_shape, dtype=torch.float64, device=r.device)
        grav_analytic(self, r, out, stream)
        return out[0] if squeeze else out

    def adjoint(self, resid, out=None, stream=None):
        """drho = A^T resid for a float64 device tensor resid [B, M, C] (or [M, C])."""
        import torch
        squeeze = resid.dim() == 2
        r = resid.reshape(self.out_shape)
        if r.dtype != torch.float64 or not r.is_cuda or not r.is_contiguous():
            raise ValueError("resid must be a contiguous float64 HIP tensor of shape %s" % (self.out_shape,))
        if out is None:
            out = torch.empty(self.rho_shape, dtype=torch.float64, device=r.device)
        grav_adjoint(self, r, out, stream)
        return out[0] if squeeze else out

    def set_profiling(self, on: bool = True) -> None:
        check(load().grav_set_profiling(self.handle, 1 if on else 0), "grav_set_profiling")

    def stage_times(self):
        n = 16
        names = (ctypes.c_char_p * n)()
        ms = (ctypes.c_double * n)()
        cnt = ctypes.c_int32()
        check(load().grav_stage_times(self.handle, names, ms, n, ctypes.byref(cnt)), "grav_stage_times")
        return [(names[i].decode(), ms[i]) for i in range(cnt.value)]


def grav_plan(spec: PlanSpec) -> Plan:
    return Plan(spec)


def grav_plan_bytes(plan: Plan):
    return plan.bytes()


def grav_plan_info(plan: Plan):
    return plan.n_targets, plan.levels, plan.leaf_cells, plan.n_target_leaves


def grav_eval(plan: Plan, rho, g_out, stream=None) -> None:
    check(load().grav_eval(plan.handle, ctypes.c_void_p(rho.data_ptr()),
                           ctypes.c_void_p(g_out.data_ptr()), _stream_ptr(stream)), "grav_eval")


def grav_direct(plan: Plan, rho, g_out, stream=None) -> None:
    check(load().grav_direct(plan.handle, ctypes.c_void_p(rho.data_ptr()),
                             ctypes.c_void_p(g_out.data_ptr()), _stream_ptr(stream)), "grav_direct")


def grav_direct_noalloc(plan: Plan, rho, g_out, stream=None) -> None:
    check(load().grav_direct_noalloc(plan.handle, ctypes.c_void_p(rho.data_ptr()),
                                     ctypes.c_void_p(g_out.data_ptr()), _stream_ptr(stream)),
          "grav_direct_noalloc")


def grav_analytic(plan: Plan, rho, gz_out, stream=None) -> None:
    check(load().grav_analytic(plan.handle, ctypes.c_void_p(rho.data_ptr()),
                               ctypes.c_void_p(gz_out.data_ptr()), _stream_ptr(stream)), "grav_analytic")


def grav_adjoint(plan: Plan, resid, drho_out, stream=None) -> None:
    check(load().grav_adjoint(plan.handle, ctypes.c_void_p(resid.data_ptr()),
                              ctypes.c_void_p(drho_out.data_ptr()), _stream_ptr(stream)), "grav_adjoint")


def grav_operator(p: int, kind: int, which: int = 0, d=(0, 0, 0)) -> np.ndarray:
    """Operator matrix (p^2 x p^2, FP64) used by the plans; see include/grav.h."""
    out = np.zeros((p * p, p * p), dtype=np.float64)
    check(load().grav_operator(p, kind, which, int(d[0]), int(d[1]), int(d[2]),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "grav_operator")
    return out


def grav_harmonics(p: int, kind: int, x: float, y: float, z: float) -> np.ndarray:
    out = np.zeros(p * p, dtype=np.float64)
    check(load().grav_harmonics(p, kind, x, y, z, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
          "grav_harmonics")
    return out


class GravFMM:
    """``torch.autograd.Function`` over a plan: forward = grav_eval, backward = grav_adjoint."""

    @staticmethod
    def apply(rho, plan: Plan):
        return _fn().apply(rho, plan)


_FN = None


def _fn():
    global _FN
    if _FN is None:
        import torch

        class _GravFMMFn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, rho, plan):
                ctx.plan = plan
                return plan.eval(rho.contiguous())

            @staticmethod
            def backward(ctx, grad):
                return ctx.plan.adjoint(grad.contiguous()), None

        _FN = _GravFMMFn
    return _FN
