"""grav_direct_noalloc (the allocation-free variant of grav_direct): called
through the C ABI, its output equals grav_direct's element by element (same
kernels and summation order; only the partial sums live elsewhere), on two
calls in a row, the second on a smaller plan, so a stale larger content of
the shared device array cannot leak into the result."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
G = pytest.importorskip("paper_1107_5951_amd")
from paper_1107_5951_amd import _lib  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(name, plan, rho, out):
    lib = _lib.load()
    stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    rc = getattr(lib, name)(plan.handle, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                            stream)
    assert rc == _lib.GRAV_OK, "%s returned %d" % (name, rc)


def _cases():
    rng = np.random.default_rng(21)
    # 8,080 targets, 7,680 cells, 2 models: 16 source chunks (partials 4 MiB)
    big = G.PlanSpec(n=(24, 20, 16), h=1.0 / 24, quad_order=2, points=W.stations(20, 1.1),
                     voxel_centres=True, components=4, p=6, leaf_size=64, batch=2)
    rho_big = rng.normal(size=(2, 16, 20, 24))
    # 770 targets, 720 cells, mixed precision: 3 source chunks
    small = G.PlanSpec(n=(10, 9, 8), h=0.1, origin=(-0.2, 0.1, 0.0), quad_order=1,
                       points=rng.uniform(-0.5, 1.5, size=(50, 3)), voxel_centres=True, components=3, p=6,
                       leaf_size=8, precision=G.GRAV_MIXED)
    rho_small = rng.normal(size=(1, 8, 9, 10))
    return [("larger", big, rho_big), ("smaller", small, rho_small)]


def test_noalloc_direct_equals_direct_two_calls():
    for tag, spec, rho in _cases():
        plan = G.Plan(spec)
        r = torch.as_tensor(rho, device="cuda").reshape(plan.rho_shape).contiguous()
        a = torch.full(plan.out_shape, float("nan"), dtype=torch.float64, device="cuda")
        b = torch.full(plan.out_shape, float("nan"), dtype=torch.float64, device="cuda")
        _say("noalloc direct, %s plan: %d targets" % (tag, plan.n_targets))
        _call("grav_direct_noalloc", plan, r, a)
        _call("grav_direct", plan, r, b)
        torch.cuda.synchronize()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)
