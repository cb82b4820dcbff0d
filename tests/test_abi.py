"""CPU checks of the C ABI: the library loads, exports every declared entry point,
and rejects bad arguments before touching the GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psatd.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    from paper_1812_07357_amd import psatd

    return psatd


def test_header_declares_the_contract():
    names = _declared_functions()
    for n in ("psatd_plan_create", "psatd_plan_create_ex", "psatd_push", "guard_fill", "guard_merge",
              "psatd_step_g1", "psatd_plan_destroy", "psatd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for n in _declared_functions():
        assert hasattr(so, n), f"{n} declared in psatd.h but not exported"


def _desc(lib, **kw):
    d = dict(nx=8, ny=8, nz=8, ngx=1, ngy=1, ngz=1, order=4, dx=1.0, dy=1.0, dz=1.0, dt=0.5, c=1.0, eps0=1.0,
             precision=0, flags=0)
    d.update(kw)
    return lib.PlanDesc(**d)


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-3), dict(ngz=-1), dict(order=3), dict(order=-2),
                                 dict(dx=0.0), dict(dt=0.0), dict(c=-1.0), dict(eps0=0.0), dict(precision=7),
                                 dict(flags=4), dict(flags=-1), dict(dt=float("nan"))])
def test_invalid_descriptors_are_rejected_on_the_host(lib, bad):
    h = ctypes.c_void_p()
    rc = lib._lib.psatd_plan_create_ex(ctypes.byref(_desc(lib, **bad)), ctypes.byref(h))
    assert rc == lib.PSATD_EINVAL
    assert h.value is None
    assert lib._lib.psatd_last_error().decode() != ""


def test_null_arguments(lib):
    L = lib._lib
    assert L.psatd_plan_create_ex(None, None) == lib.PSATD_EINVAL
    assert L.psatd_push(None, None, None, None, None, None, None) == lib.PSATD_EINVAL
    assert L.guard_fill(None, None, None, 1, None, None, None) == lib.PSATD_EINVAL
    assert L.guard_merge(None, None, None, 1, None, None, 0, None) == lib.PSATD_EINVAL
    assert L.psatd_step_g1(None, None, None, None, None) == lib.PSATD_EINVAL
    v = ctypes.c_longlong()
    assert L.psatd_plan_query(None, 0, ctypes.byref(v)) == lib.PSATD_EINVAL
    L.psatd_plan_destroy(None)  # NULL-safe
    assert L.psatd_plan_create(0, 8, 8, 0, 0, 1.0, 0.5) is None


def test_mlp_null_and_invalid_arguments(lib):
    L = lib._lib
    h = ctypes.c_void_p()
    fp = ctypes.POINTER(ctypes.c_float)
    init = (ctypes.c_float * lib.MLP_NPARAM)()
    six = (ctypes.c_float * 6)(*([1.0] * 6))
    assert L.psatd_mlp_create(None, six, six, 0.0, 1.0, 16, ctypes.byref(h)) == lib.PSATD_EINVAL
    assert L.psatd_mlp_create(ctypes.cast(init, fp), six, six, 0.0, 1.0, 16, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_create(ctypes.cast(init, fp), six, six, 0.0, 1.0, 0, ctypes.byref(h)) == lib.PSATD_EINVAL
    assert L.psatd_mlp_create(ctypes.cast(init, fp), six, six, 0.0, 0.0, 16, ctypes.byref(h)) == lib.PSATD_EINVAL
    assert h.value is None
    assert L.psatd_mlp_set(None, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_get(None, None, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_predict(None, None, 4, None, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_grad(None, None, None, 4, None, 4, None, None, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_adam(None, 1e-3, 0.9, 0.999, 1e-8, None) == lib.PSATD_EINVAL
    assert L.psatd_mlp_train(None, None, None, 4, None, 1, 4, 1e-3, 0.9, 0.999, 1e-8, None, None) == lib.PSATD_EINVAL
    L.psatd_mlp_destroy(None)  # NULL-safe
    assert "psatd_mlp" in L.psatd_last_error().decode()


def _factor(n):
    out, p = [], 2
    while p * p <= n:
        while n % p == 0:
            out.append(p)
            n //= p
        p += 1
    if n > 1:
        out.append(n)
    return out


RADICES = {2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 16, 17, 18, 20, 24, 32, 36}


def test_default_schedules_factor_the_length(lib):
    """Host schedule choice: a product of compiled radices equal to n (smooth n) or to a Bluestein length >= 2n-1."""
    for n in list(range(2, 300)) + [320, 544, 576, 1056, 1021, 2048, 4096, 6561]:
        radices, m = lib.default_schedule(n)
        assert radices and all(r in RADICES for r in radices), (n, radices)
        assert int(np.prod(radices)) == m, (n, radices, m)
        smooth = max(_factor(n)) <= 17
        if smooth:
            assert m == n, (n, radices, m)
        else:
            assert 2 * n - 1 <= m <= 4 * n, (n, m)
    assert lib.default_schedule(320)[0] in ([20, 16], [16, 20])
    assert len(lib.default_schedule(576)[0]) == 2
    assert lib.default_schedule(1)[1] == 1


def test_default_schedule_rejects_bad_arguments(lib):
    r = (ctypes.c_int * 4)()
    m = ctypes.c_int()
    assert lib._lib.psatd_default_schedule(0, r, 4, ctypes.byref(m)) == lib.PSATD_EINVAL
    assert lib._lib.psatd_default_schedule(64, None, 4, ctypes.byref(m)) == lib.PSATD_EINVAL


def _batch_create(lib, boxes, gdims):
    descs = (lib.PlanDesc * len(boxes))()
    origins = (ctypes.c_int * (3 * len(boxes)))()
    for i, (o, n) in enumerate(boxes):
        descs[i] = _desc(lib, nx=n[0], ny=n[1], nz=n[2])
        for a in range(3):
            origins[3 * i + a] = o[a]
    h = ctypes.c_void_p()
    rc = lib._lib.psatd_batch_create(len(boxes), descs, origins, (ctypes.c_int * 3)(*gdims), ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("boxes", [
    [((0, 0, 0), (8, 8, 8)), ((4, 0, 0), (8, 8, 8))],          # overlap along x, same y and z
    [((0, 0, 0), (8, 8, 8)), ((12, 4, 6), (8, 8, 8))],         # wraps onto box 0 across the periodic edge
    [((0, 0, 0), (16, 16, 16)), ((5, 5, 5), (1, 1, 1))],       # one cell inside another interior
])
def test_batch_rejects_overlapping_interiors_on_the_host(lib, boxes):
    rc, h = _batch_create(lib, boxes, (16, 16, 16))
    assert rc == lib.PSATD_EINVAL
    assert "overlap" in lib._lib.psatd_last_error().decode()
    assert h.value is None


def test_batch_rejects_interiors_outside_the_grid(lib):
    rc, h = _batch_create(lib, [((0, 0, 0), (8, 8, 8)), ((8, 0, 16), (8, 8, 8))], (16, 16, 16))
    assert rc == lib.PSATD_EINVAL and h.value is None


def test_device_budget_gives_enomem_and_leaks_nothing(lib):
    """With a zero budget every constructor fails with ENOMEM before touching the device, and the
    library holds no device memory afterwards (plan and batch cleanup paths)."""
    before = lib.device_bytes_in_use()
    lib.set_device_budget(0)
    try:
        h = ctypes.c_void_p()
        assert lib._lib.psatd_plan_create_ex(ctypes.byref(_desc(lib)), ctypes.byref(h)) == lib.PSATD_ENOMEM
        assert h.value is None
        assert "allocation" in lib._lib.psatd_last_error().decode()
        rc, hb = _batch_create(lib, [((0, 0, 0), (8, 8, 8)), ((8, 0, 0), (8, 8, 8))], (16, 8, 8))
        assert rc == lib.PSATD_ENOMEM and hb.value is None
        assert lib.device_bytes_in_use() == before
    finally:
        lib.set_device_budget(None)


def _write_cache(path, body, schema=3):
    path.write_text('{\n  "psatd_tune_cache": %d,\n  "entries": {\n%s\n  }\n}\n' % (schema, body))
    return str(path)


def test_tune_cache_reader_rejects_stale_and_corrupt_entries(lib, tmp_path):
    good = '    "fp32|x|n=576|m=576|other=320x320": {"radix": [24, 24], "tile": 16}'
    entries = [
        good,
        '    "fp32|z|n=320|m=320|other=576x320": {"radix": [20, 16], "tile": 256, "kern": 4}',
        '    "fp32|y|n=320|m=320|other=320x576": {"radix": [20, 16], "tile": 16, "kern": 99}',  # bad kernel bits
        '    "fp32|y|n=320|m=320|other=320x576": {"radix": [16, 16], "tile": 16}',   # product 256 != 320
        '    "fp32|z|n=19|m=19|other=8x8": {"radix": [19], "tile": 256}',           # radix 19 not compiled
        '    "fp32|z|n=320|m=320|other=8x8": {"radix": [], "tile": 256}',           # empty schedule
        '    "fp32|y|n=64|m=64|other=8x8": {"radix": [8, 8], "tile": -3}',          # bad tile
        '    "fp32|y|n=64|len=64": {"radix": [8, 8], "tile": 4}',                    # key without a length
    ]
    # reading stops at the bad kernel bits: good + the "kern" entry accepted, the rest unread
    assert lib.tune_cache_load(_write_cache(tmp_path / "a.json", ",\n".join(entries))) == (2, 1)
    del entries[2]
    assert lib.tune_cache_load(_write_cache(tmp_path / "a2.json", ",\n".join(entries))) == (2, 5)
    # another schema version: every entry is discarded
    assert lib.tune_cache_load(_write_cache(tmp_path / "b.json", good, schema=2)) == (0, 1)
    # malformed text: reading stops, nothing after the break is taken
    bad = good + ',\n    "fp32|x|n=64|m=64|other=8x8": {"radix": [8, 8 "tile": 4}'
    assert lib.tune_cache_load(_write_cache(tmp_path / "c.json", bad)) == (1, 1)
    (tmp_path / "d.json").write_text("not json at all {{{")
    assert lib.tune_cache_load(str(tmp_path / "d.json")) == (0, 1)
    (tmp_path / "e.json").write_text("")
    assert lib.tune_cache_load(str(tmp_path / "e.json")) == (0, 1)
    assert lib.tune_cache_load(str(tmp_path / "missing.json")) == (0, 0)


def _pic_desc(lib, **kw):
    d = dict(gx=16, gy=16, gz=16, dx=1.0, dy=1.0, dz=1.0, dt=0.5, c=1.0, q=1.0, q_over_m=1.0, max_particles=100,
             tile=8, precision=0, flags=0, shape=0)
    d.update(kw)
    return lib.PicDesc(**d)


@pytest.mark.parametrize("bad,code", [(dict(gx=0), "EINVAL"), (dict(dz=0.0), "EINVAL"), (dict(dt=-0.5), "EINVAL"),
                                      (dict(c=0.0), "EINVAL"), (dict(precision=3), "EINVAL"),
                                      (dict(flags=2), "EINVAL"), (dict(tile=0), "EINVAL"), (dict(tile=17), "EINVAL"),
                                      (dict(max_particles=-1), "EINVAL"), (dict(shape=4), "EINVAL"),
                                      (dict(shape=-1), "EINVAL"), (dict(dt=1.5), "EUNSUPPORTED"),
                                      (dict(dy=0.4), "EUNSUPPORTED")])
def test_pic_descriptors_are_checked_on_the_host(lib, bad, code):
    h = ctypes.c_void_p()
    rc = lib._lib.psatd_pic_create(ctypes.byref(_pic_desc(lib, **bad)), ctypes.byref(h))
    assert rc == getattr(lib, "PSATD_" + code)
    assert h.value is None
    assert lib._lib.psatd_last_error().decode() != ""


def test_pic_null_arguments(lib):
    L = lib._lib
    assert L.psatd_pic_create(None, None) == lib.PSATD_EINVAL
    assert L.psatd_pic_push(None, None, None, None, None, 0, None) == lib.PSATD_EINVAL
    assert L.psatd_pic_deposit(None, None, None, None, None, 0, None) == lib.PSATD_EINVAL
    L.psatd_pic_destroy(None)  # NULL-safe


def test_pml_null_arguments(lib):
    L = lib._lib
    w = (ctypes.c_int * 3)(1, 1, 1)
    assert L.psatd_pml_set(None, w, 1.0, 2.0) == lib.PSATD_EINVAL
    assert L.psatd_pml_step(None, None, None, None) == lib.PSATD_EINVAL

