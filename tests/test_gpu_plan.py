"""Plans built on the device: host validation of every index table, and the
work counts against the closed forms of the paper's work model (Sec. 3.2.3):
on a full uniform level with k boxes per axis the near-field leaf pairs are
(3k - 2)^3 (each leaf with its in-range neighbours, itself included) and
the M2L box pairs are (6k - 8)^3 - (3k - 2)^3 summed over levels 2..L."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1107_5951_amd")

SPECS = {
    "stations": dict(n=(16, 16, 16), h=1 / 16, quad_order=1, points=W.stations(32, 1.1), components=3,
                     p=8, leaf_size=32),
    "volume q2": dict(n=(64, 64, 64), h=1 / 64, quad_order=2, voxel_centres=True, components=3, p=10,
                      leaf_size=512),
    "ragged": dict(n=(13, 7, 9), h=0.1, origin=(-0.3, 0.2, -1.0), quad_order=1,
                   points=np.random.default_rng(4).uniform(-1.5, 2.0, size=(300, 3)), components=4,
                   p=12, leaf_size=8),
    "batch": dict(n=(128, 128, 128), h=1 / 128, points=W.stations(256, 1.1), components=1, p=8,
                  leaf_size=64, batch=32),
    "random points": dict(n=(32, 32, 32), h=1 / 32, points=np.random.default_rng(12).uniform(-0.2, 1.3, (20000, 3)),
                          components=1, p=4, leaf_size=8),
}


@pytest.mark.parametrize("name", sorted(SPECS))
def test_plan_tables_validate(name):
    plan = G.Plan(G.PlanSpec(**SPECS[name]))
    assert plan.check() == "ok"


@pytest.mark.parametrize("k", [4, 8, 16])
def test_work_counts_match_closed_forms(k):
    """Volume targets on a k^3-leaf mesh whose root equals the mesh."""
    b = 2
    n = k * b
    plan = G.Plan(G.PlanSpec(n=(n, n, n), h=1.0 / n, quad_order=1, voxel_centres=True, components=1,
                             p=4, leaf_size=b ** 3))
    assert plan.leaf_cells == b and plan.levels == int(np.log2(k))
    m2l, p2p, nsrc = plan.work()
    B = b ** 3  # targets and sources per leaf
    assert p2p == (3 * k - 2) ** 3 * B * B
    expect = sum((6 * kk - 8) ** 3 - (3 * kk - 2) ** 3 for kk in [2 ** l for l in range(2, plan.levels + 1)])
    assert m2l == expect
    assert nsrc == n ** 3
