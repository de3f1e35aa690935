"""Serving loop (continuous batching of forward and adjoint solves): every
result in the mix equals the same request served alone (within the rounding
of the FP32 partial sums; 1e-5, ten times under the mixed bar), graph
replays equal eager solves, admission waits for memory instead of failing,
same-plan requests are batched, and spot checks meet the mixed bar (1e-4)
against the FP64 oracle (forward) and its transpose (adjoint)."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1107_5951_amd")
from paper_1107_5951_amd import serve  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _alone(req):
    srv = serve.GravServer(max_inflight=1, batching=False, graphs=False)
    res, _ = srv.run([req])
    out = res[0].out.cpu().numpy()
    srv.close()
    return out


def test_mix_equals_alone_and_oracle():
    reqs = serve.poisson_trace(24, rate=50.0, seed=1005, n_min=12, n_max=40)
    assert {r.kind for r in reqs} == {"forward", "adjoint"}
    mix = serve.GravServer(max_inflight=4)
    res_mix, stats = mix.run(reqs)
    _say("serve mix: %s" % stats)
    assert stats["served"] == len(reqs) and stats["rejected"] == 0
    out_mix = [r.out.cpu().numpy() for r in res_mix]
    mix.close()
    for i, req in enumerate(reqs):
        d = oracle.rel_l2(out_mix[i], _alone(req))
        assert d <= 1e-5, (i, req.kind, req.n, d)
    # spot checks against the oracle (mixed precision at the server's p = 10)
    for i in (0, 3, 7, 12, 15, 21):
        req = reqs[i]
        grid = W.Grid.unit(req.n)
        st = serve.station_grid(req.n)
        if req.kind == "forward":
            idx = W.sample_indices(st.shape[0], 256, seed=i)
            ref = oracle.forward(req.data.cpu().numpy(), grid.origin, grid.h, req.q, st[idx], comps=1)[:, 0]
            e = oracle.rel_l2(out_mix[i][idx], ref)
        else:
            cells = W.sample_indices(grid.ncell, 256, seed=i)
            ref = oracle.adjoint_cells(req.data.cpu().numpy()[:, None], grid.origin, grid.h, req.q,
                                       grid.shape, st, cells, comps=1)
            e = oracle.rel_l2(out_mix[i].ravel()[cells], ref)
        _say("request %d %s n=%d q=%d: rel err %.3e" % (i, req.kind, req.n, req.q, e))
        assert e <= 1e-4


def test_graph_replays_equal_eager_solves():
    """A slot's captured forward and adjoint graphs, replayed with new inputs
    and with eager work and synchronisations between replays, give exactly
    the eager result of the same plan."""
    slot = serve.Slot(20, 2, 2, 10, G.GRAV_MIXED, graphs=True)
    assert set(slot.graphs) == {"forward", "adjoint"}
    eager = G.Plan(serve.plan_spec(20, 2, batch=2))
    gen = torch.Generator(device="cuda").manual_seed(3)
    for k in range(4):
        rho = torch.rand((2, 20, 20, 20), dtype=torch.float64, device="cuda", generator=gen)
        res = torch.randn((2, 400), dtype=torch.float64, device="cuda", generator=gen)
        fw = slot.launch("forward", [serve.Request(20, 2, rho[b]) for b in range(2)], torch.cuda.current_stream())
        slot.event.synchronize()
        ad = slot.launch("adjoint", [serve.Request(20, 2, res[b], "adjoint") for b in range(2)],
                         torch.cuda.current_stream())
        slot.event.synchronize()
        g_ref = eager.eval(rho)[..., 0]
        d_ref = eager.adjoint(res[..., None].contiguous())
        torch.cuda.synchronize()
        for b in range(2):
            np.testing.assert_array_equal(fw[b].cpu().numpy(), g_ref[b].cpu().numpy())
            np.testing.assert_array_equal(ad[b].cpu().numpy(), d_ref[b].cpu().numpy())
    slot.close()


def test_admission_waits_for_memory_and_rejects_what_never_fits():
    probe = serve.Slot(16, 1, 1, 10, G.GRAV_MIXED, graphs=False)
    one = probe.nbytes
    probe.close()
    gen = torch.Generator(device="cuda").manual_seed(7)
    reqs = [serve.Request(n, 1, torch.rand((n, n, n), dtype=torch.float64, device="cuda", generator=gen))
            for n in (16, 17, 16, 17, 16, 17)]
    srv = serve.GravServer(budget_bytes=int(one * 1.5), max_inflight=4)
    res, stats = srv.run(reqs)
    _say("admission under a budget of 1.5 slots: %s" % stats)
    assert stats["served"] == len(reqs)
    assert srv.used <= srv.budget
    for r, req in zip(res, reqs):
        assert oracle.rel_l2(r.out.cpu().numpy(), _alone(req)) <= 1e-5
    srv.close()
    tiny = serve.GravServer(budget_bytes=1 << 20)
    res, stats = tiny.run(reqs[:2])
    assert stats["rejected"] == 2 and all(r.error for r in res)
    tiny.close()


def test_same_plan_requests_are_batched():
    gen = torch.Generator(device="cuda").manual_seed(11)
    reqs = [serve.Request(18, 1, torch.rand((18, 18, 18), dtype=torch.float64, device="cuda", generator=gen))
            for _ in range(4)]
    reqs.append(serve.Request(22, 2, torch.rand((22, 22, 22), dtype=torch.float64, device="cuda",
                                                generator=gen)))
    srv = serve.GravServer(max_inflight=4)
    res, stats = srv.run(reqs)
    _say("batching: %s" % stats)
    assert [r.batch for r in res] == [4, 4, 4, 4, 1]
    assert stats["batches"] == 2
    for r, req in zip(res, reqs):
        assert oracle.rel_l2(r.out.cpu().numpy(), _alone(req)) <= 1e-5
    srv.close()
