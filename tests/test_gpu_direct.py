"""GPU direct summation (grav_direct, the summation method of Sec. 2.1):
parity with the FP64 oracle, and the FMM checked against it on every target
of a medium workload (an independent GPU evaluation of the same sum)."""
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


@pytest.mark.parametrize("q,prec,bar", [(1, 0, 1e-12), (2, 0, 1e-12), (2, 1, 1e-5)])
def test_direct_matches_oracle(q, prec, bar):
    grid = W.Grid(12, 10, 9, (-0.2, 0.1, 0.0), 0.1)
    rho = np.random.default_rng(3).normal(size=grid.shape)
    st = np.concatenate([W.stations(9, 1.1), np.random.default_rng(4).uniform(-0.5, 1.5, (100, 3))])
    spec = G.PlanSpec(n=(grid.nx, grid.ny, grid.nz), h=grid.h, origin=grid.origin, quad_order=q, points=st,
                      voxel_centres=True, components=4, p=8, leaf_size=64, precision=prec)
    plan = G.Plan(spec)
    out = plan.direct(torch.as_tensor(rho, device="cuda")).cpu().numpy()
    tg = np.concatenate([st, grid.centres()])
    ref = oracle.forward(rho, grid.origin, grid.h, q, tg, comps=4)
    e = oracle.rel_l2(out, ref)
    _say("direct q=%d prec=%d vs oracle: %.3e" % (q, prec, e))
    assert e < bar


def test_direct_batched_models():
    grid = W.Grid.unit(8)
    rhos = np.stack([W.gaussian_blobs(grid, 4, 50 + b) for b in range(3)])
    spec = G.PlanSpec(n=(8, 8, 8), h=grid.h, points=W.stations(6, 1.1), components=3, p=6, batch=3)
    plan = G.Plan(spec)
    out = plan.direct(torch.as_tensor(rhos, device="cuda")).cpu().numpy()
    for b in range(3):
        ref = oracle.forward(rhos[b], grid.origin, grid.h, 1, W.stations(6, 1.1), comps=3)
        assert oracle.rel_l2(out[b], ref) < 1e-12


def test_fmm_matches_direct_on_every_target():
    """32^3 cells, 2-point rule (262,144 sources), g at all 32,768 centres:
    the FMM in FP64 at p = 12 against the GPU direct sum on every target."""
    grid = W.Grid.unit(32)
    rho = torch.as_tensor(W.gaussian_blobs(grid, 16, 1002, noise=0.01), device="cuda")
    plan = G.Plan(G.PlanSpec(n=(32, 32, 32), h=grid.h, quad_order=2, voxel_centres=True, components=3,
                             p=12, leaf_size=512))
    a = plan.eval(rho).cpu().numpy()
    b = plan.direct(rho).cpu().numpy()
    e = oracle.rel_l2(a, b)
    _say("FMM p=12 vs GPU direct sum, all 32768 targets: %.3e" % e)
    assert e < 1e-6


def test_direct_mixed_at_volume64_size():
    """64^3 cells, 2-point rule (2,097,152 source points), g at all 262,144
    cell centres: every target sums over all sources, so the partial sums are
    as long as they get at this size; mixed precision meets 1e-4 against the
    oracle on 4096 seeded targets."""
    grid = W.Grid.unit(64)
    rho_h = W.gaussian_blobs(grid, 32, 1002, noise=0.01)
    plan = G.Plan(G.PlanSpec(n=(64, 64, 64), h=grid.h, quad_order=2, voxel_centres=True, components=3,
                             p=10, leaf_size=512, precision=G.GRAV_MIXED))
    out = plan.direct(torch.as_tensor(rho_h, device="cuda"))
    idx = W.sample_indices(grid.ncell, 4096, seed=7)
    g = out.index_select(0, torch.as_tensor(idx, device="cuda")).cpu().numpy()
    ref = oracle.forward(rho_h, grid.origin, grid.h, 2, grid.centres()[idx], comps=3)
    e = oracle.rel_l2(g, ref)
    _say("direct mixed, 64^3 q=2, 4096 sampled targets: %.3e" % e)
    assert e <= 1e-4
