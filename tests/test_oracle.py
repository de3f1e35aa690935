"""Pins of the FP64 direct-sum oracle to things other than itself.

Each test fixes the oracle against a value the paper prints, a closed form, a
physical invariant, or an independent brute-force computation, so that a
plausible mistake (dropped term, wrong sign, swapped axis, misplaced Gauss
point, wrong weight) fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import prism

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --------------------------------------------------------------------------
# Closed-form prism: Appendix A, Table A1 (fixes magnitudes, geometry, G) and
# brute-force quadrature of the defining integral (fixes the sign).
# --------------------------------------------------------------------------
@pytest.mark.parametrize("row", [0, 2])
def test_prism_closed_form_reproduces_table_a1(row):
    tab = _golden("table_a1_quadrature.json")
    r = tab["rows"][row]
    l1, l2, linf = prism.field_norms(W.PAPER_CUBE, W.PAPER_DOMAIN, r["Mbar"], r["m"],
                                     rho=tab["rho"], G=tab["G"])
    assert l1 == pytest.approx(r["l1"], rel=2e-12)
    assert l2 == pytest.approx(r["l2"], rel=2e-12)
    assert linf == pytest.approx(r["linf"], rel=2e-12)


def _gauss_box_integral(box, pt, n=24, sub=4):
    """Brute-force tensor Gauss quadrature of (P_z - z')/|P - x'|^3 over box."""
    xi, wi = np.polynomial.legendre.leggauss(n)
    axes = []
    for lo, hi in box:
        edges = np.linspace(lo, hi, sub + 1)
        pts = ((edges[:-1] + edges[1:])[:, None] / 2 + (edges[1:] - edges[:-1])[:, None] / 2 * xi).ravel()
        wts = (((edges[1:] - edges[:-1]) / 2)[:, None] * wi).ravel()
        axes.append((pts, wts))
    (X, WX), (Y, WY), (Z, WZ) = axes
    dz = pt[2] - Z[:, None, None]
    dy = pt[1] - Y[None, :, None]
    dx = pt[0] - X[None, None, :]
    r3 = (dx * dx + dy * dy + dz * dz) ** 1.5
    return float(np.einsum("k,j,i,kji->", WZ, WY, WX, dz / r3))


@pytest.mark.parametrize("pt", [(310.0, 290.0, 150.0), (0.0, 600.0, -450.0),
                                (300.0, 300.0, -40.0), (420.0, 180.0, -260.0)])
def test_prism_closed_form_matches_brute_force(pt):
    exact = prism.prism_gz(np.array(pt), W.PAPER_CUBE, rho=1.0, G=1.0)
    brute = _gauss_box_integral(W.PAPER_CUBE, np.array(pt))
    assert exact == pytest.approx(brute, rel=1e-10)


def test_prism_sign_points_away_from_mass():
    above = prism.prism_gz(np.array([300.0, 300.0, 0.0]), W.PAPER_CUBE)
    below = prism.prism_gz(np.array([300.0, 300.0, -300.0]), W.PAPER_CUBE)
    assert above > 0 and below < 0
    assert above == pytest.approx(-below, rel=1e-12)


# --------------------------------------------------------------------------
# Table 1: SUM-G1 / SUM-G2 convergence rates on the paper's model.
# --------------------------------------------------------------------------
def _crop(grid, rho):
    """Drop all-zero cells around the anomaly (they contribute exactly zero)."""
    nz = np.nonzero(rho)
    k0, j0, i0 = (int(a.min()) for a in nz)
    k1, j1, i1 = (int(a.max()) + 1 for a in nz)
    org = (grid.origin[0] + i0 * grid.h, grid.origin[1] + j0 * grid.h, grid.origin[2] + k0 * grid.h)
    return rho[k0:k1, j0:j1, i0:i1], org


@pytest.mark.slow
@pytest.mark.parametrize("q,name", [(1, "SUM-G1"), (2, "SUM-G2")])
def test_sum_rates_reproduce_table1(q, name):
    tab = _golden("table1_sum_rates.json")
    hs, errs = [], []
    for nbar in tab["Mbar"]:
        grid, rho = W.paper_model(nbar)
        sub, org = _crop(grid, rho)
        tg = grid.centres()
        gz = oracle.forward(sub, org, grid.h, q, tg, comps=1, G=W.G_SI)[:, 0]
        ex = prism.prism_gz(tg, W.PAPER_CUBE, rho=W.PAPER_RHO, G=W.G_SI)
        hs.append(grid.h)
        errs.append(prism.discrete_errors(ex, gz, grid.h))
    errs = np.array(errs)
    for col, key in enumerate(("E1", "E2", "Einf")):
        rate = prism.convergence_rate(hs, errs[:, col])
        assert round(rate, 2) == pytest.approx(tab[name][key], abs=1e-9), (key, rate)


# --------------------------------------------------------------------------
# Independent brute force: explicit point list built here from the Gauss rule,
# summed in extended precision.
# --------------------------------------------------------------------------
def _explicit_points(rho, origin, h, q):
    nz, ny, nx = rho.shape
    if q == 1:
        offs, wts = np.array([0.0]), np.array([1.0])
    else:
        offs, wts = np.array([-1.0, 1.0]) / (2 * np.sqrt(3.0)), np.array([0.5, 0.5])
    pts, ms = [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for a, wa in zip(offs, wts):
                    for b, wb in zip(offs, wts):
                        for c, wc in zip(offs, wts):
                            pts.append((origin[0] + (i + 0.5 + c) * h,
                                        origin[1] + (j + 0.5 + b) * h,
                                        origin[2] + (k + 0.5 + a) * h))
                            ms.append(rho[k, j, i] * h ** 3 * wa * wb * wc)
    return np.array(pts), np.array(ms)


@pytest.mark.parametrize("q", [1, 2])
def test_oracle_matches_longdouble_brute_force(q):
    rng = np.random.default_rng(11)
    rho = rng.normal(size=(3, 4, 5))
    origin, h = (0.1, -0.2, 0.3), 0.25
    tg = np.concatenate([rng.uniform(-1, 2, size=(12, 3)),
                         [[0.1 + 0.625, -0.2 + 0.375, 0.3 + 0.125]]])  # a cell centre
    pts, ms = _explicit_points(rho, origin, h, q)
    P = pts.astype(np.longdouble)
    M = ms.astype(np.longdouble)
    ref = np.zeros((tg.shape[0], 4), dtype=np.longdouble)
    for j, t in enumerate(tg.astype(np.longdouble)):
        d = t[None, :] - P
        r2 = (d * d).sum(axis=1)
        keep = r2 != 0
        r = np.sqrt(r2[keep])
        ref[j, 0] = (M[keep] / r).sum()
        ref[j, 1:] = (M[keep, None] * d[keep] / (r ** 3)[:, None]).sum(axis=0)
    got = oracle.forward(rho, origin, h, q, tg, comps=4, G=1.0)
    np.testing.assert_allclose(got, ref.astype(np.float64), rtol=1e-13, atol=1e-15)
    # and the explicit-point entry agrees with the lattice entry
    pts_out = oracle.points(pts, ms, tg, comps=4)
    np.testing.assert_allclose(pts_out, got, rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# Physics: sphere exterior field, Newton's third law, g = -grad(phi).
# --------------------------------------------------------------------------
def test_voxel_sphere_exterior_field():
    n, R = 32, 0.3
    grid = W.Grid.unit(n)
    c = np.array([0.5, 0.5, 0.5])
    rho = W.sphere_density(grid, c, R)
    mass = rho.sum() * grid.h ** 3
    dirs = np.array([[0, 0, 1], [1, 0, 0], [1, 1, 1], [0.3, -0.8, 0.5]], dtype=float)
    dirs /= np.linalg.norm(dirs, axis=1)[:, None]
    devs = []
    for rr in (3 * R, 6 * R):
        tg = c + rr * dirs
        g = oracle.forward(rho, grid.origin, grid.h, 1, tg, comps=3)
        radial = (g * dirs).sum(axis=1)
        tang = np.linalg.norm(g - radial[:, None] * dirs, axis=1)
        assert np.all(radial > 0)  # g points away from the mass (Eq. 1)
        dev = np.abs(radial * rr * rr / mass - 1.0)
        assert np.all(dev < 2e-3)
        assert np.all(tang < 2e-3 * radial)
        devs.append(dev.max())
    # cubic symmetry removes degrees 1-3: the deviation falls off like r^-4
    assert devs[1] < devs[0] / 8


def test_newton_third_law_invariant():
    rng = np.random.default_rng(5)
    grid = W.Grid.unit(8)
    rho = rng.normal(size=grid.shape)
    tg = grid.centres()
    g = oracle.forward(rho, grid.origin, grid.h, 1, tg, comps=3)
    m = rho.ravel() * grid.h ** 3
    total = (m[:, None] * g).sum(axis=0)
    scale = (np.abs(m)[:, None] * np.abs(g)).sum()
    assert np.all(np.abs(total) < 1e-13 * scale)


def test_gradient_of_potential():
    rng = np.random.default_rng(9)
    grid = W.Grid.unit(6)
    rho = rng.normal(size=grid.shape)
    tg = rng.uniform(-0.5, 1.5, size=(6, 3))
    tg[:, 2] = np.abs(tg[:, 2]) + 1.2  # away from the sources
    out = oracle.forward(rho, grid.origin, grid.h, 2, tg, comps=4)
    eps = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fp = oracle.forward(rho, grid.origin, grid.h, 2, tg + e, comps=4)[:, 0]
        fm = oracle.forward(rho, grid.origin, grid.h, 2, tg - e, comps=4)[:, 0]
        np.testing.assert_allclose(out[:, 1 + a], -(fp - fm) / (2 * eps), rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("q", [1, 2])
def test_prism_convergence_in_h(q):
    """The cell quadrature converges to the closed form at stations above the
    body.  Both rules are O(h^4) there: the h^2 term of the midpoint rule is
    proportional to the integral of the kernel's Laplacian, which vanishes
    because the kernel is harmonic away from the station."""
    box = ((0.25, 0.75), (0.25, 0.75), (0.25, 0.75))
    st = W.stations(6, z=1.1)
    exact = prism.prism_gz(st, box)
    errs = []
    for n in (8, 16, 32):
        grid = W.Grid.unit(n)
        rho = W.box_density(grid, box)
        gz = oracle.forward(rho, grid.origin, grid.h, q, st, comps=1)[:, 0]
        errs.append(np.abs(gz - exact).max() / np.abs(exact).max())
    assert errs[2] < 1e-6
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


# --------------------------------------------------------------------------
# The transpose: dot-product identity for every output mode.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("q,comps", [(1, 1), (2, 3), (1, 4)])
def test_adjoint_dot_product(q, comps):
    rng = np.random.default_rng(3)
    grid = W.Grid.unit(5)
    rho = rng.normal(size=(2,) + grid.shape)
    tg = np.concatenate([grid.centres()[::7], W.stations(4, 1.1)])
    r = rng.normal(size=(2, tg.shape[0], comps))
    Ax = oracle.forward(rho, grid.origin, grid.h, q, tg, comps=comps)
    ATr = oracle.adjoint(r, grid.origin, grid.h, q, grid.shape, tg, comps=comps)
    lhs = (Ax * r).sum()
    rhs = (rho * ATr).sum()
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(r)


@pytest.mark.parametrize("q,comps", [(1, 1), (2, 4)])
def test_adjoint_cells_equals_full_adjoint_at_those_cells(q, comps):
    """The sampled transpose decodes each flat cell index (x fastest, then y,
    then z) on a mesh whose three axes differ, so an axis mix-up or an
    origin/offset slip changes the value; the full transpose it is compared
    with is pinned by the dot-product identity above."""
    rng = np.random.default_rng(8)
    grid = W.Grid(7, 5, 4, (0.3, -0.1, 0.2), 0.15)
    tg = np.concatenate([grid.centres()[::5], rng.uniform(-0.5, 1.5, size=(30, 3))])
    r = rng.normal(size=(2, tg.shape[0], comps))
    full = oracle.adjoint(r, grid.origin, grid.h, q, grid.shape, tg, comps=comps).reshape(2, -1)
    cells = np.array([0, grid.ncell - 1, 6, 7, 34, 35, 71, 3, 3, 139, 100, 57])
    got = oracle.adjoint_cells(r, grid.origin, grid.h, q, grid.shape, tg, cells, comps=comps)
    np.testing.assert_allclose(got, full[:, cells], rtol=1e-14, atol=1e-15 * np.abs(full).max())
    one = oracle.adjoint_cells(r[1], grid.origin, grid.h, q, grid.shape, tg, cells, comps=comps)
    np.testing.assert_allclose(one, full[1, cells], rtol=1e-14, atol=1e-15 * np.abs(full).max())


# ---------------------------------------------------------------- SUM-AN
def _st(n=5, z=1.1):
    return W.stations(n, z)


def test_sum_an_of_uniform_block_is_the_block_closed_form():
    """Summing the closed form over the cells of a uniform, non-cubic block
    gives the closed form of the whole block (interior faces cancel): pins
    the cell indexing, its axis order and the corner signs of sum_an."""
    h = 0.125
    rho = np.zeros((4, 5, 6))
    rho[1:3, 1:5, 2:5] = 2.5  # z in [1, 3), y in [1, 5), x in [2, 5) (cells)
    origin = np.array([0.1, -0.2, 0.3])
    pts = np.concatenate([_st(4, 1.1), [[0.4, 0.3, 0.45], [0.9, -0.5, 0.0]]])
    got = prism.sum_an(rho, origin, h, pts)
    box = ((origin[0] + 2 * h, origin[0] + 5 * h), (origin[1] + 1 * h, origin[1] + 5 * h),
           (origin[2] + 1 * h, origin[2] + 3 * h))
    ref = prism.prism_gz(pts, box, 2.5)
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14)


def test_sum_an_single_cell_matches_brute_force_quadrature():
    """One off-centre cell against a 24-point-per-axis Gauss-Legendre
    integral of (P_z - z') / |P - x'|^3 (Eq. (1)) far enough away that the
    quadrature converges to rounding."""
    h = 0.2
    rho = np.zeros((2, 2, 3))
    rho[1, 0, 2] = 1.7
    origin = np.array([0.0, 0.0, 0.0])
    pts = np.array([[0.1, 0.9, 1.5], [1.3, -0.4, -0.8], [0.5, 0.1, 0.7]])
    got = prism.sum_an(rho, origin, h, pts)
    xi, wi = prism.gauss_legendre(24)
    lo = origin + np.array([2, 0, 1]) * h
    q = lo[None, :] + 0.5 * h * (xi[:, None] + 1.0)
    X, Y, Z = np.meshgrid(q[:, 0], q[:, 1], q[:, 2], indexing="ij")
    Wt = np.einsum("i,j,k->ijk", wi, wi, wi) * (0.5 * h) ** 3
    ref = []
    for p in pts:
        d = np.sqrt((p[0] - X) ** 2 + (p[1] - Y) ** 2 + (p[2] - Z) ** 2)
        ref.append(1.7 * np.sum(Wt * (p[2] - Z) / d ** 3))
    np.testing.assert_allclose(got, ref, rtol=1e-9)


def test_sum_an_is_linear_in_rho():
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(3, 3, 3)), rng.normal(size=(3, 3, 3))
    pts = _st(3, 0.9)
    lhs = prism.sum_an(2.0 * a - b, (0, 0, 0), 0.3, pts)
    rhs = 2.0 * prism.sum_an(a, (0, 0, 0), 0.3, pts) - prism.sum_an(b, (0, 0, 0), 0.3, pts)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-14)
