"""FP64 CPU oracle for the voxel gravity forward model -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and the two share no code: the only common module is ``workloads``,
which draws seeded inputs and holds none of the method's arithmetic.

Contents
--------
``direct.c``   plain direct summation of Eq. (1) (Sec. 1.1) under the cell
               quadrature of Sec. 2.1, and its exact transpose (C, OpenMP).
``prism.py``   closed-form vertical attraction of a uniform rectangular prism
               (the analytic solution the paper's Sec. 3 uses), and the error
               norms of Eqs. (15)-(17) with the quadrature of Appendix A.

Conventions (shared with the GPU library by specification, not by code):
``rho`` is ``[batch][nz][ny][nx]`` with x fastest; cell (i, j, k) has centre
``origin + (i + 1/2, j + 1/2, k + 1/2) * h``; targets are ``[m][3]``; outputs
are ``[batch][m][comps]`` with comps 1 = (gz), 3 = (gx, gy, gz),
4 = (phi, gx, gy, gz); g = -grad(phi) and phi = G * sum(m / r).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "direct.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``direct.c`` into ``_liboracle.so`` (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            dp = ctypes.POINTER(ctypes.c_double)
            lib.oracle_forward.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                           ctypes.c_int, ctypes.c_int, dp, ctypes.c_int64, dp,
                                           ctypes.c_int, ctypes.c_double, dp]
            lib.oracle_adjoint.argtypes = lib.oracle_forward.argtypes
            lib.oracle_adjoint_cells.argtypes = lib.oracle_forward.argtypes[:-1] + [
                ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), dp]
            lib.oracle_points.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int64, dp,
                                          ctypes.c_int, ctypes.c_double, dp]
            lib.oracle_num_threads.argtypes = []
            lib.oracle_set_threads.argtypes = [ctypes.c_int]
            for f in (lib.oracle_forward, lib.oracle_adjoint, lib.oracle_adjoint_cells,
                      lib.oracle_points, lib.oracle_num_threads, lib.oracle_set_threads):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    """OpenMP threads the oracle uses (``OMP_NUM_THREADS`` or all cores)."""
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> int:
    """Use n OpenMP threads from now on (n >= 1); returns the count in effect."""
    return int(_load().oracle_set_threads(int(n)))


def forward(rho, origin, h, q, targets, comps=3, G=1.0) -> np.ndarray:
    """Direct sum of Eq. (1) under the q-point-per-axis cell quadrature.

    rho: ``[nz, ny, nx]`` or ``[batch, nz, ny, nx]``; origin: lower corner of
    cell (0, 0, 0); h: cell edge (scalar or (hx, hy, hz)); q: 1 or 2;
    targets: ``[m, 3]``.  Returns ``[m, comps]`` (or ``[batch, m, comps]``).
    """
    rho = _f64(rho)
    squeeze = rho.ndim == 3
    if squeeze:
        rho = rho[None]
    batch, nz, ny, nx = rho.shape
    tg = _f64(targets).reshape(-1, 3)
    m = tg.shape[0]
    org = _f64(origin).reshape(3)
    hh = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)))
    out = np.zeros((batch, m, comps), dtype=np.float64)
    rc = _load().oracle_forward(nx, ny, nz, _ptr(org), _ptr(hh), int(q), batch, _ptr(rho),
                                m, _ptr(tg), int(comps), float(G), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_forward failed with code %d" % rc)
    return out[0] if squeeze else out


def adjoint(resid, origin, h, q, shape, targets, comps=3, G=1.0) -> np.ndarray:
    """Exact transpose of :func:`forward` with respect to rho.

    resid: ``[m, comps]`` or ``[batch, m, comps]``; shape: (nz, ny, nx).
    Returns ``[nz, ny, nx]`` (or ``[batch, nz, ny, nx]``).
    """
    resid = _f64(resid)
    squeeze = resid.ndim == 2
    if squeeze:
        resid = resid[None]
    batch, m, c = resid.shape
    if c != comps:
        raise ValueError("resid has %d components, expected %d" % (c, comps))
    nz, ny, nx = shape
    tg = _f64(targets).reshape(-1, 3)
    if tg.shape[0] != m:
        raise ValueError("resid and targets disagree on the number of targets")
    org = _f64(origin).reshape(3)
    hh = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)))
    drho = np.zeros((batch, nz, ny, nx), dtype=np.float64)
    rc = _load().oracle_adjoint(nx, ny, nz, _ptr(org), _ptr(hh), int(q), batch, _ptr(resid),
                                m, _ptr(tg), int(comps), float(G), _ptr(drho))
    if rc != 0:
        raise ValueError("oracle_adjoint failed with code %d" % rc)
    return drho[0] if squeeze else drho


def adjoint_cells(resid, origin, h, q, shape, targets, cells, comps=3, G=1.0) -> np.ndarray:
    """:func:`adjoint` evaluated only at the flat cell indices ``cells``.

    Returns ``[len(cells)]`` (or ``[batch, len(cells)]`` for batched resid).
    """
    resid = _f64(resid)
    squeeze = resid.ndim == 2
    if squeeze:
        resid = resid[None]
    batch, m, c = resid.shape
    if c != comps:
        raise ValueError("resid has %d components, expected %d" % (c, comps))
    nz, ny, nx = shape
    tg = _f64(targets).reshape(-1, 3)
    if tg.shape[0] != m:
        raise ValueError("resid and targets disagree on the number of targets")
    cl = np.ascontiguousarray(cells, dtype=np.int64).reshape(-1)
    org = _f64(origin).reshape(3)
    hh = _f64(np.broadcast_to(np.asarray(h, dtype=np.float64), (3,)))
    out = np.zeros((batch, cl.size), dtype=np.float64)
    rc = _load().oracle_adjoint_cells(nx, ny, nz, _ptr(org), _ptr(hh), int(q), batch, _ptr(resid),
                                      m, _ptr(tg), int(comps), float(G), cl.size,
                                      cl.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_adjoint_cells failed with code %d" % rc)
    return out[0] if squeeze else out


def points(src, mass, targets, comps=4, G=1.0) -> np.ndarray:
    """Direct sum over explicit point masses: ``[m, comps]``."""
    src = _f64(src).reshape(-1, 3)
    mass = _f64(mass).reshape(-1)
    tg = _f64(targets).reshape(-1, 3)
    out = np.zeros((tg.shape[0], comps), dtype=np.float64)
    rc = _load().oracle_points(src.shape[0], _ptr(src), _ptr(mass), tg.shape[0], _ptr(tg),
                               int(comps), float(G), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_points failed with code %d" % rc)
    return out


def rel_l2(approx, exact) -> float:
    """Relative L2 error over all entries: ||approx - exact|| / ||exact||."""
    a = np.asarray(approx, dtype=np.float64)
    e = np.asarray(exact, dtype=np.float64)
    den = np.linalg.norm(e.ravel())
    return float(np.linalg.norm((a - e).ravel()) / (den if den > 0 else 1.0))
