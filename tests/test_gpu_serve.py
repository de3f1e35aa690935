"""Serving loop (many small forward solves): results in a concurrent mix are
bitwise identical to the same requests served one at a time, plans are
reused from the cache, and spot checks match the FP64 oracle."""
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


def test_mix_equals_alone_and_oracle():
    reqs = serve.poisson_trace(24, rate=50.0, seed=1005, n_min=12, n_max=40)
    mix = serve.GravServer(n_streams=4)
    res_mix, stats = mix.run(reqs)
    _say("serve mix: %s" % stats)
    out_mix = [r.out.cpu().numpy() for r in res_mix]
    mix.close()
    assert stats["plan_hits"] + stats["plan_misses"] == len(reqs)
    alone = serve.GravServer(n_streams=1)
    for i, req in enumerate(reqs):
        r = alone.submit(i, req)
        r.event.synchronize()
        np.testing.assert_array_equal(r.out.cpu().numpy(), out_mix[i])
    alone.close()
    # spot checks against the oracle (mixed precision at the server's p = 10)
    for i in (0, 7, 15):
        req = reqs[i]
        st = serve.station_grid(req.n)
        idx = W.sample_indices(st.shape[0], 256, seed=i)
        ref = oracle.forward(req.rho.cpu().numpy(), (0.0, 0.0, 0.0), 1.0 / req.n, req.q, st[idx], comps=1)
        e = oracle.rel_l2(out_mix[i][idx], ref)
        _say("request %d n=%d q=%d: rel err %.3e" % (i, req.n, req.q, e))
        assert e <= 1e-4


def test_cache_budget_evicts_least_recent():
    probe = serve.PlanCache(1 << 40)
    need = sum(probe.get(12, 1).bytes())
    probe.close()
    cache = serve.PlanCache(int(need * 1.5))
    cache.get(12, 1)
    cache.get(13, 1)          # does not fit beside the first: evicts it
    assert cache.evictions == 1 and cache.used <= cache.budget
    cache.get(13, 1)
    assert cache.hits == 1
    with pytest.raises(MemoryError):
        serve.PlanCache(1).get(8, 1)
    cache.close()
