"""The C ABI: the library loads and exports every function include/grav.h
declares; descriptor validation rejects bad input before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1107_5951_amd as G
from paper_1107_5951_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "grav.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(grav_[a-z_]+)\s*\(", txt)))


def test_every_declared_function_is_exported():
    lib = G.load()
    names = _declared()
    assert "grav_plan" in names and "grav_eval" in names and "grav_adjoint" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTS)


def test_desc_layout_matches_header_defaults():
    d = _lib.GravDesc()
    G.load().grav_desc_init(ctypes.byref(d))
    assert (d.quad_order, d.components, d.p, d.leaf_size, d.batch, d.G) == (1, 3, 8, 64, 1, 1.0)
    assert d.precision == G.GRAV_FP64 and d.n_points == 0


@pytest.mark.parametrize("field,value", [
    ("n", (0, 4, 4)), ("h", 0.0), ("h", float("nan")), ("quad_order", 3), ("components", 2),
    ("p", 0), ("leaf_size", 0), ("precision", 7), ("batch", 0), ("G", float("inf")),
])
def test_invalid_descriptor_is_rejected(field, value):
    spec = G.PlanSpec(n=(4, 4, 4), h=0.25, voxel_centres=True)
    setattr(spec, field, value)
    with pytest.raises(G.GravError) as e:
        G.Plan(spec)
    assert e.value.code == _lib.GRAV_EINVAL


def test_unsupported_order_is_reported():
    spec = G.PlanSpec(n=(4, 4, 4), h=0.25, voxel_centres=True, p=17)
    with pytest.raises(G.GravError) as e:
        G.Plan(spec)
    assert e.value.code == _lib.GRAV_EUNSUPPORTED


def test_null_pointers_are_rejected():
    lib = G.load()
    assert lib.grav_eval(None, None, None, None) == _lib.GRAV_EINVAL
    assert lib.grav_adjoint(None, None, None, None) == _lib.GRAV_EINVAL
    assert lib.grav_direct(None, None, None, None) == _lib.GRAV_EINVAL
    assert lib.grav_analytic(None, None, None, None) == _lib.GRAV_EINVAL
    assert lib.grav_plan(None, None) == _lib.GRAV_EINVAL
    assert lib.grav_status_string(_lib.GRAV_EBUSY).decode() != ""


def test_explicit_source_descriptor_is_validated():
    """Explicit sources must lie inside the mesh box, need the 1-point rule
    and positive volumes (checked before any device work)."""
    inside = np.array([[0.1, 0.2, 0.3], [0.9, 0.5, 0.5]])
    for kw in (dict(sources=np.array([[1.2, 0.5, 0.5]])),                  # outside the box
               dict(sources=np.array([[0.5, 0.5, float("nan")]])),         # not finite
               dict(sources=inside, quad_order=2),                          # needs q = 1
               dict(sources=inside, source_volumes=np.array([1e-3, 0.0]))):  # volume <= 0
        spec = G.PlanSpec(n=(4, 4, 4), h=0.25, points=np.array([[0.5, 0.5, 1.5]]), **kw)
        with pytest.raises(G.GravError) as e:
            G.Plan(spec)
        assert e.value.code == _lib.GRAV_EINVAL, kw
    d = _lib.GravDesc()
    G.load().grav_desc_init(ctypes.byref(d))
    assert d.n_sources == 0 and not d.sources and not d.source_volumes
