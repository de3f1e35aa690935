"""Closed-form attraction of a uniform prism and the paper's error norms.

TEST INFRASTRUCTURE (part of the oracle; see ``oracle/__init__.py``).

* :func:`prism_gz` -- vertical attraction of a uniform rectangular prism.
  Sec. 3 of May & Knepley computes its exact solution with the closed form of
  Li & Chouteau (1998).  This is the textbook antiderivative written out from
  the mathematics, with the sign of Eq. (1):
  ``gz(P) = G rho * integral over the prism of (P_z - z') / |P - x'|^3 dV'``,
  i.e. gz > 0 above a positive anomaly.  With u = x' - P_x, v = y' - P_y,
  w = z' - P_z and r = |(u, v, w)|, the function
  ``F = u ln(v + r) + v ln(u + r) - w arctan(u v / (w r))``
  satisfies d3F/(du dv dw) = -w / r^3, so ``gz = G rho [[[F]]]`` evaluated
  between the lower and upper corners (sign (-1)^(i+j+k), index 1 = lower).
  Plain ``arctan`` is used, not a two-argument arctangent: the branch must
  follow the sign of ``w``.
* :func:`sum_an` -- the closed-form summation method SUM-AN of Sec. 2.1: gz
  at each point as the sum over all cells of a cell-wise constant density of
  :func:`prism_gz` of the cell, written out cell by cell.
* :func:`field_norms` -- Appendix A: integrals of |gz| and gz^2 over the model
  domain with a 4-point Gauss-Legendre rule per axis on an m x m x m
  subdivision of each of the Mbar^3 cells (Table A1), plus max |gz| over the
  same quadrature points (the table's third column).
* :func:`discrete_errors` -- Eqs. (15)-(17) approximated with a one-point rule
  per cell (Sec. 3.1): E1 = sum h^3 |d|, E2 = (sum h^3 d^2)^(1/2),
  Einf = max |d|.
* :func:`convergence_rate` -- least-squares slope of log E against log h
  (the rates of Tables 1 and 3).
"""
from __future__ import annotations

import numpy as np


def _F(u, v, w):
    r = np.sqrt(u * u + v * v + w * w)
    with np.errstate(divide="ignore", invalid="ignore"):
        t1 = np.where(u == 0.0, 0.0, u * np.log(np.where(v + r > 0, v + r, 1.0)))
        t2 = np.where(v == 0.0, 0.0, v * np.log(np.where(u + r > 0, u + r, 1.0)))
        wr = w * r
        t3 = np.where(w == 0.0, 0.0, w * np.arctan(u * v / np.where(wr == 0.0, 1.0, wr)))
    return t1 + t2 - t3


def prism_gz(points, box, rho=1.0, G=1.0) -> np.ndarray:
    """gz at ``points [..., 3]`` of the prism ``box = ((x1, x2), (y1, y2), (z1, z2))``."""
    p = np.asarray(points, dtype=np.float64)
    (x1, x2), (y1, y2), (z1, z2) = box
    px, py, pz = p[..., 0], p[..., 1], p[..., 2]
    acc = np.zeros(px.shape, dtype=np.float64)
    for i, xa in ((1, x1), (2, x2)):
        for j, yb in ((1, y1), (2, y2)):
            for k, zc in ((1, z1), (2, z2)):
                sign = -1.0 if (i + j + k) % 2 else 1.0
                acc += sign * _F(xa - px, yb - py, zc - pz)
    return G * rho * acc


def sum_an(rho, origin, h, points, G=1.0) -> np.ndarray:
    """SUM-AN (Sec. 2.1): gz at ``points [M, 3]`` of the density ``rho
    [nz, ny, nx]`` (constant per cell, cell (i, j, k) = the box from
    origin + (i, j, k) h to origin + (i + 1, j + 1, k + 1) h), as the sum over
    cells of the closed-form prism attraction."""
    r = np.asarray(rho, dtype=np.float64)
    nz, ny, nx = r.shape
    o = np.asarray(origin, dtype=np.float64)
    out = np.zeros(np.asarray(points).shape[0], dtype=np.float64)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if r[k, j, i] == 0.0:
                    continue
                box = ((o[0] + i * h, o[0] + (i + 1) * h), (o[1] + j * h, o[1] + (j + 1) * h),
                       (o[2] + k * h, o[2] + (k + 1) * h))
                out += prism_gz(points, box, r[k, j, i], G)
    return out


def gauss_legendre(n: int):
    """n-point Gauss-Legendre abscissae and weights on [-1, 1]."""
    return np.polynomial.legendre.leggauss(n)


def field_norms(box, domain, nbar, m, rho=1.0, G=1.0, order=4):
    """(integral |gz|, sqrt(integral gz^2), max |gz|) over ``domain``.

    ``domain = ((x0, x1), (y0, y1), (z0, z1))`` is split into nbar cells per
    axis, each cell into m sub-cells per axis, each sub-cell integrated with
    an ``order``-point Gauss-Legendre rule per axis (Appendix A).
    """
    xi, wi = gauss_legendre(order)
    axes = []
    for lo, hi in domain:
        ns = nbar * m
        hs = (hi - lo) / ns
        centres = lo + (np.arange(ns) + 0.5) * hs
        pts = (centres[:, None] + 0.5 * hs * xi[None, :]).ravel()
        wts = np.broadcast_to(0.5 * hs * wi[None, :], (ns, order)).ravel()
        axes.append((pts, wts))
    (X, WX), (Y, WY), (Z, WZ) = axes
    XX, YY = np.meshgrid(X, Y, indexing="ij")
    WXY = np.outer(WX, WY)
    l1 = 0.0
    l2 = 0.0
    linf = 0.0
    for z, wz in zip(Z, WZ):
        pts = np.stack([XX, YY, np.full_like(XX, z)], axis=-1)
        gz = prism_gz(pts, box, rho=rho, G=G)
        a = np.abs(gz)
        l1 += wz * float(np.sum(WXY * a))
        l2 += wz * float(np.sum(WXY * a * a))
        linf = max(linf, float(a.max()))
    return l1, float(np.sqrt(l2)), linf


def discrete_errors(exact, approx, h):
    """(E1, E2, Einf) of Eqs. (15)-(17) with a one-point rule per cell of edge h."""
    d = np.abs(np.asarray(exact, dtype=np.float64) - np.asarray(approx, dtype=np.float64))
    vol = float(h) ** 3
    return float(vol * d.sum()), float(np.sqrt(vol * (d * d).sum())), float(d.max())


def convergence_rate(hs, errs) -> float:
    """Least-squares slope of log(err) against log(h)."""
    lh = np.log(np.asarray(hs, dtype=np.float64))
    le = np.log(np.asarray(errs, dtype=np.float64))
    return float(np.polyfit(lh, le, 1)[0])
