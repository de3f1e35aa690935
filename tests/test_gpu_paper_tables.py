"""The paper's own convergence experiments run through the GPU FMM.

The model of Sec. 3 (a 100 m cube of density 2000 in a 600 m domain) on the
mesh sequence Mbar = 12, 24, 48, 96, gz at every cell centroid, G in SI
units, 27 cells per leaf as in the paper (Sec. 3.2.3), errors of
Eqs. (15)-(17) against the closed-form prism with a one-point rule per cell.

* Table 1: with the 1- and 2-point rules and an FMM accurate to rounding
  (FP64, p = 16) the rates are the summation rates of Table 1.
* Table 3: the FMM's rates rise towards those rates as p grows.  Ours at
  p = 8 equal the printed p = 8 column (1.45, 1.51, 0.99) and ours at p = 16
  the printed p = 20 column (the 1-point summation rates).  The lowest
  orders (p = 1, 4) depend on the expansion basis and on the meaning of p
  (Sec. 2.3 leaves both open: our p is the number of degrees), so there only
  the trend is compared (parity unpinned for those two columns).
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import prism
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1107_5951_amd")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rates(q, p):
    hs, errs = [], []
    for nbar in (12, 24, 48, 96):
        grid, rho = W.paper_model(nbar)
        plan = G.Plan(G.PlanSpec(n=(nbar, nbar, nbar), h=grid.h, origin=grid.origin, quad_order=q,
                                 voxel_centres=True, components=1, p=p, leaf_size=27 * q ** 3, G=W.G_SI))
        gz = plan.eval(torch.as_tensor(rho, device="cuda"))[:, 0].cpu().numpy()
        ex = prism.prism_gz(grid.centres(), W.PAPER_CUBE, rho=W.PAPER_RHO, G=W.G_SI)
        hs.append(grid.h)
        errs.append(prism.discrete_errors(ex, gz, grid.h))
    errs = np.array(errs)
    return {k: prism.convergence_rate(hs, errs[:, c]) for c, k in enumerate(("E1", "E2", "Einf"))}


@pytest.mark.parametrize("q,name", [(1, "SUM-G1"), (2, "SUM-G2")])
def test_fmm_reproduces_table1_rates(q, name):
    tab = json.load(open(os.path.join(GOLDEN, "table1_sum_rates.json")))
    r = _rates(q, 16)
    _say("q=%d FMM p=16 rates: %s (Table 1: %s)" % (q, {k: round(v, 3) for k, v in r.items()}, tab[name]))
    for k in ("E1", "E2", "Einf"):
        assert round(r[k], 2) == pytest.approx(tab[name][k], abs=1e-9), k


def test_fmm_rates_rise_with_p_towards_table3():
    t3 = json.load(open(os.path.join(GOLDEN, "table3_fmm_rates.json")))
    got = {p: _rates(1, p) for p in (1, 4, 8, 16)}
    for p in (1, 4, 8, 16):
        _say("p=%2d rates %s" % (p, {k: round(v, 2) for k, v in got[p].items()}))
    _say("Table 3 (p = 1, 4, 8, 20): E1 %s  E2 %s  Einf %s" % (t3["E1"], t3["E2"], t3["Einf"]))
    # p = 8 reproduces the printed p = 8 column; the highest order reaches
    # the printed p = 20 column
    for k in ("E1", "E2", "Einf"):
        assert round(got[8][k], 2) == pytest.approx(t3[k][2], abs=1e-9), k
        assert round(got[16][k], 2) == pytest.approx(t3[k][-1], abs=1e-9), k
    # and the E1 rate does not fall as p grows
    e1 = [got[p]["E1"] for p in (1, 4, 8, 16)]
    assert all(b >= a - 0.05 for a, b in zip(e1, e1[1:])), e1
