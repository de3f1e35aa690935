"""Explicit point sources (scattered points with volumes, the extension named
in Sec. 4 of the paper): the FMM with sources given as points instead of the
cells' quadrature points.

* sources at the cell centres with masses rho h^3 reproduce the voxel path
  (1-point rule) to rounding: the same pairs, the same expansion basis;
* scattered sources with volumes against the oracle's direct sum over point
  masses (Eq. (1) as an N-body sum, Eq. (11)) at the accuracy bars;
* the adjoint: the dot-product identity, and the transpose of the direct
  sum, which by the antisymmetry of the kernel is minus the field of the
  residuals placed at the targets, evaluated at the sources.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1107_5951_amd")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _targets(rng, n_st=20, n_in=300, lo=-0.1, hi=1.1):
    st = W.stations(n_st, 1.1)
    return np.concatenate([st, rng.uniform(lo, hi, size=(n_in, 3))])


def test_sources_at_cell_centres_equal_the_voxel_path():
    rng = np.random.default_rng(11)
    n = (12, 10, 9)
    h = 1 / 12
    rho = np.random.default_rng(3).normal(size=(2, n[2], n[1], n[0]))
    cz, cy, cx = np.meshgrid(*[(np.arange(k) + 0.5) * h for k in (n[2], n[1], n[0])], indexing="ij")
    src = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1)
    tg = rng.uniform(-0.2, 1.2, size=(400, 3))
    base = dict(n=n, h=h, points=tg, components=4, p=12, leaf_size=27, batch=2)
    vox = G.Plan(G.PlanSpec(**base))
    pts = G.Plan(G.PlanSpec(**base, sources=src))
    assert pts.check() == "ok"
    r = torch.as_tensor(rho, device="cuda")
    g_vox = vox.eval(r).cpu().numpy()
    g_pts = pts.eval(torch.as_tensor(rho.reshape(2, -1) * h ** 3, device="cuda")).cpu().numpy()
    d = oracle.rel_l2(g_pts, g_vox)
    _say("explicit sources at the centres vs the voxel path (FP64 p=12): %.3e" % d)
    assert d <= 1e-12
    # the same with densities and volumes h^3
    vol = G.Plan(G.PlanSpec(**base, sources=src, source_volumes=np.full(src.shape[0], h ** 3)))
    d2 = oracle.rel_l2(vol.eval(torch.as_tensor(rho.reshape(2, -1), device="cuda")).cpu().numpy(), g_vox)
    assert d2 <= 1e-12


@pytest.mark.parametrize("prec,p,bar", [(0, 14, 1e-6), (1, 10, 1e-4)])
def test_scattered_sources_match_oracle(prec, p, bar):
    rng = np.random.default_rng(5)
    N = 20000
    src = rng.uniform(0.0, 1.0, size=(N, 3)) ** np.array([1.0, 1.0, 1.5])  # denser near z = 0
    vol = rng.uniform(0.5, 1.5, size=N) / N  # volumes of a partition of the unit cube, roughly
    dens = np.stack([np.sin(3 * src[:, 0]) + src[:, 2], np.cos(2 * src[:, 1]) - 0.5])
    tg = _targets(rng, 24, 500)
    plan = G.Plan(G.PlanSpec(n=(32, 32, 32), h=1 / 32, points=tg, components=4, p=p, leaf_size=64, batch=2,
                             precision=prec, sources=src, source_volumes=vol))
    assert plan.check() == "ok"
    m2l, p2p, ns = plan.work()
    assert ns == N and p2p > 0 and m2l > 0
    g = plan.eval(torch.as_tensor(dens, device="cuda")).cpu().numpy()
    worst = 0.0
    for b in range(2):
        ref = oracle.points(src, dens[b] * vol, tg, comps=4)
        worst = max(worst, oracle.rel_l2(g[b], ref))
    _say("scattered sources prec=%d p=%d: rel err %.3e (bar %g)" % (prec, p, worst, bar))
    assert worst <= bar


def test_sources_adjoint_transpose():
    rng = np.random.default_rng(8)
    N = 6000
    src = rng.uniform(0.0, 1.0, size=(N, 3))
    vol = rng.uniform(0.5, 1.5, size=N) / N
    tg = _targets(rng, 16, 300, 0.0, 1.0)
    for prec, p, bar in ((0, 14, 1e-12), (1, 10, 1e-5)):
        plan = G.Plan(G.PlanSpec(n=(16, 16, 16), h=1 / 16, points=tg, components=3, p=p, leaf_size=32, batch=2,
                                 precision=prec, sources=src, source_volumes=vol))
        rho = torch.as_tensor(rng.normal(size=(2, N)), device="cuda")
        res = torch.as_tensor(rng.normal(size=(2, tg.shape[0], 3)), device="cuda")
        g = plan.eval(rho)
        d = plan.adjoint(res)
        gap = abs(float((g * res).sum()) - float((rho * d).sum())) / (float(g.norm()) * float(res.norm()))
        _say("explicit sources, adjoint dot product prec=%d: %.3e" % (prec, gap))
        assert gap <= bar
        if prec == 0:
            # transpose of the direct sum: d rho_i = V_i sum_t r_t . (t - x_i)/|t - x_i|^3
            # = -V_i * (field at x_i of masses r_t placed at the targets), per component
            dn = d.cpu().numpy()
            rn = res.cpu().numpy()
            ref = np.zeros((2, N))
            for c in range(3):
                for b in range(2):
                    ref[b] -= oracle.points(tg, rn[b, :, c], src, comps=4)[:, 1 + c]
            ref *= vol[None]
            e = oracle.rel_l2(dn, ref)
            _say("explicit sources, adjoint vs the oracle's transpose (FP64 p=14): %.3e" % e)
            assert e <= 1e-6


def test_summation_methods_refuse_explicit_sources():
    src = np.array([[0.2, 0.3, 0.4], [0.7, 0.6, 0.5]])
    plan = G.Plan(G.PlanSpec(n=(4, 4, 4), h=0.25, points=np.array([[0.5, 0.5, 1.5]]), sources=src))
    with pytest.raises(G.GravError) as e:
        plan.direct(torch.ones((1, 2), dtype=torch.float64, device="cuda"))
    assert e.value.code == 4
