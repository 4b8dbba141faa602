"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/okrig.h, its struct layouts match the
binding, and argument validation happens before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "okrig.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(okr_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2303_09523_amd as P
    return P.load()


def test_exports_every_declared_function(lib):
    names = _declared()
    assert "okr_execute" in names and "okr_plan_create" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_lists_every_export():
    from paper_2303_09523_amd import _lib
    assert sorted(_lib.EXPORTED) == _declared()


def test_status_strings(lib):
    for s in range(8):
        assert lib.okr_status_string(s)
    assert lib.okr_status_string(3) == b"non-finite known voxel"
    assert lib.okr_version() >= 100


def _prob(**kw):
    from paper_2303_09523_amd import _lib
    d = dict(nx=16, ny=16, nslices=4, upsample=2, radius=1, min_points=4, precision=0, algo=0,
             refine_tol=1e-4, refine_max=1, strict=0, drift=0)
    d.update(kw)
    return _lib.Problem(**d)


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), 2), (dict(ny=70000), 2), (dict(nslices=0), 2), (dict(upsample=0), 2),
    (dict(upsample=16), 2), (dict(radius=4), 2), (dict(radius=-1), 2), (dict(min_points=0), 1),
    (dict(min_points=19), 1), (dict(precision=7), 1), (dict(algo=3), 1),
    (dict(algo=1, precision=1), 6), (dict(refine_max=9), 1), (dict(refine_max=2), 1), (dict(refine_tol=-1.0), 1),
    (dict(drift=2), 1), (dict(drift=1, algo=1), 6),
    (dict(drift=1, upsample=15), 2),
    (dict(nx=65535, ny=65535, nslices=3), 2),
])
def test_plan_validation_before_device(lib, kw, code):
    h = C.c_void_p()
    p = _prob(**kw)
    assert lib.okr_plan_create(C.byref(p), None, C.byref(h)) == code
    assert not h.value


def test_null_arguments(lib):
    assert lib.okr_plan_create(None, None, None) == 1
    h = C.c_void_p()
    assert lib.okr_plan_create(None, None, C.byref(h)) == 1
    assert lib.okr_stats_get(None, None) == 1
    assert lib.okr_plan_destroy(None) == 1
    assert lib.okr_execute(None, None, None, None, None, None, None) == 1


def test_rule_matches_header_documentation():
    # the header documents the canonical candidate order used by okr_select
    src = open(os.path.join(ROOT, "include", "okrig.h")).read()
    assert "c = s*W*W + (dy+radius)*W + (dx+radius)" in src
