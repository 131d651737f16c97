"""The C-ABI library loads on a CPU host, exports every symbol include/fks.h declares,
and validates arguments in host-only calls (no device work)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fks.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fks_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1701_01608_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libfks.so is not built (python -m paper_1701_01608_amd.build)")
    return _lib


def test_every_declared_symbol_is_exported(lib):
    h = ctypes.CDLL(lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(h, n), n
    assert set(names) == set(lib.EXPORTS)


def _desc(lib, **kw):
    d = dict(n=16, kernel=lib.FKS_HARD_SPHERES, L=8.0, R=6.0, alpha=0.0, C=0.25, a1=4, a2=4, n_radial=8,
             dtype=lib.FKS_F32, flags=0, reserved=0)
    d.update(kw)
    return lib.CollideDesc(**d)


def _create(lib, desc, max_cells=4):
    h = ctypes.c_void_p()
    st = lib.lib().fks_plan_create(ctypes.byref(desc), max_cells, ctypes.byref(h))
    return st, h


def test_plan_create_sizes_and_destroy(lib):
    L = lib.lib()
    st, h = _create(lib, _desc(lib))
    assert st == 0, L.fks_last_error()
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.fks_plan_sizes(h, ctypes.byref(tb), ctypes.byref(wb)) == 0
    nt, pad = ctypes.c_int32(), ctypes.c_int32()
    assert L.fks_plan_info(h, ctypes.byref(nt), ctypes.byref(pad)) == 0
    assert nt.value == 17 and pad.value == 24
    # [terms][rows][pencils][2]: rows = k_z chunks of the slab fold, pencils = half plane
    assert tb.value % (17 * ((15 * 15 + 1) // 2) * 2 * 4) == 0 and tb.value >= 17 * 15 * 113 * 8
    assert wb.value > 0
    L.fks_plan_destroy(h)
    L.fks_plan_destroy(None)


@pytest.mark.parametrize("bad,status", [
    (dict(n=10), -2), (dict(n=7), -1), (dict(L=-1.0), -1), (dict(R=7.5), -1), (dict(a1=0), -1),
    (dict(kernel=5), -1), (dict(dtype=3), -1), (dict(flags=64), -1), (dict(C=0.0), -1),
    (dict(kernel=1, n_radial=0), -1), (dict(kernel=1, alpha=1.0), -1),
])
def test_plan_create_rejects(lib, bad, status):
    st, h = _create(lib, _desc(lib, **bad))
    assert st == status
    assert h.value is None
    assert lib.lib().fks_last_error()


def test_max_cells_limit(lib):
    # one chunk's launches stay within the 2^32 threads of a grid: max_cells <= 2^19
    for m, ok in ((1 << 19, True), ((1 << 19) + 1, False), (0, False)):
        st, h = _create(lib, _desc(lib), max_cells=m)
        assert (st == 0) == ok, (m, st)
        if ok:
            lib.lib().fks_plan_destroy(h)
        else:
            assert st == -1 and b"max_cells" in lib.lib().fks_last_error()


def test_overlap_flag_allows_large_R(lib):
    st, h = _create(lib, _desc(lib, R=7.5, flags=lib.FKS_ALLOW_OVERLAP))
    assert st == 0
    lib.lib().fks_plan_destroy(h)


def test_calls_before_bind_fail_cleanly(lib):
    L = lib.lib()
    st, h = _create(lib, _desc(lib))
    assert st == 0
    assert L.fks_collide(h, ctypes.c_void_p(256), ctypes.c_void_p(512 * 1024 * 1024), 1, None) == -5
    assert b"bind" in L.fks_last_error()
    L.fks_plan_destroy(h)
    assert L.fks_collide(None, None, None, 1, None) == -1


def test_transport_create_validation(lib):
    L = lib.lib()
    h = ctypes.c_void_p()
    assert L.fks_xport_create(16, 8.0, 0, 4, 4, 0.1, ctypes.byref(h)) == -1
    assert L.fks_xport_create(16, 8.0, 4, 4, 4, -0.1, ctypes.byref(h)) == -1
    assert L.fks_xport_create(20, 8.0, 4, 4, 4, 0.1, ctypes.byref(h)) == L.fks_xport_create(64, 8.0, 4, 4, 4, 0.1, ctypes.byref(h))
    assert L.fks_xport_create(20, 8.0, 4, 4, 4, 0.1, ctypes.byref(h)) < 0 and b"n in" in L.fks_last_error()
    assert L.fks_xport_create(32, 8.0, 1, 256, 256, 0.1, ctypes.byref(h)) < 0 and b"y-z plane" in L.fks_last_error()
    assert L.fks_xport_create(16, 8.0, 4, 4, 4, 0.1, ctypes.byref(h)) == 0
    # not bound yet: both modes of the deferred transport refuse
    assert L.fks_transport_ex(h, None, None, 1, 0.01, 0, None) == -5
    assert L.fks_transport_ex(h, None, None, 1, 0.01, 1, None) == -5
    sb = ctypes.c_size_t()
    assert L.fks_xport_sizes(h, ctypes.byref(sb)) == 0 and sb.value >= 16 ** 3 * 48
    assert L.fks_transport(h, ctypes.c_void_p(256), ctypes.c_void_p(512), 1, 0.1, None) == -5
    L.fks_xport_destroy(h)


def test_surrogate_create_validation(lib):
    L = lib.lib()
    h = ctypes.c_void_p()
    # modes odd / too large, width not a multiple of 128, batch not a multiple of 128, bad scale
    assert L.fks_sur_create(32, 7, 1024, 1024, 1.0, 0, ctypes.byref(h)) == -1
    assert L.fks_sur_create(32, 32, 1024, 1024, 1.0, 0, ctypes.byref(h)) == -1
    assert L.fks_sur_create(32, 8, 1000, 1024, 1.0, 0, ctypes.byref(h)) == -1
    assert L.fks_sur_create(32, 8, 1024, 1000, 1.0, 0, ctypes.byref(h)) == -1
    assert L.fks_sur_create(32, 8, 1024, 1024, 0.0, 0, ctypes.byref(h)) == -1
    assert L.fks_sur_create(12, 4, 128, 128, 1.0, 0, ctypes.byref(h)) == -2   # 12^3 not a multiple of 128
    assert L.fks_sur_create(32, 8, 1024, 1024, 1.0, 4, ctypes.byref(h)) == -1        # unknown flag
    assert L.fks_sur_create(32, 8, 1024, 1024, 1.0, 0, ctypes.byref(h)) == 0
    pb, wb, npar = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int64()
    assert L.fks_sur_sizes(h, ctypes.byref(pb), ctypes.byref(wb), ctypes.byref(npar)) == 0
    n_in, w, n_out = 1024, 1024, 32 ** 3
    assert npar.value == n_in * w + w + w * w + w + n_out * w + n_out
    assert pb.value >= npar.value * (4 * 4 + 2)      # master, m, v, grad (FP32) + BF16 copy
    assert wb.value >= 1024 * n_out * 4              # FP32 outputs of one batch
    # calls before bind
    assert L.fks_sur_forward(h, ctypes.c_void_p(256), ctypes.c_void_p(512), 128, None) == -5
    L.fks_sur_destroy(h)


def test_term_groups_limits(lib):
    L = lib.lib()
    st, big = _create(lib, _desc(lib), max_cells=4096)
    assert st == 0
    assert L.fks_plan_set_term_groups(big, 1) == 0
    assert L.fks_plan_set_term_groups(big, 2) == -2          # large-batch plan: no group workspace
    L.fks_plan_destroy(big)
    st, small = _create(lib, _desc(lib), max_cells=1)
    assert st == 0
    tg, mx = ctypes.c_int32(), ctypes.c_int32()
    assert L.fks_plan_get_term_groups(small, ctypes.byref(tg), ctypes.byref(mx)) == 0
    assert (tg.value, mx.value) == (1, 17)                   # at most one group per term
    assert L.fks_plan_set_term_groups(small, 0) == -1
    assert L.fks_plan_set_term_groups(small, 18) == -2
    assert L.fks_plan_set_term_groups(small, 8) == 0
    # 17 terms in groups of ceil(17/8) = 3: 6 groups are used, none empty
    assert L.fks_plan_get_term_groups(small, ctypes.byref(tg), ctypes.byref(mx)) == 0
    assert tg.value == 6
    assert L.fks_plan_set_term_groups(small, 17) == 0
    assert L.fks_plan_get_term_groups(small, ctypes.byref(tg), ctypes.byref(mx)) == 0
    assert tg.value == 17
    L.fks_plan_destroy(small)


def test_step_ex_validates_options_on_the_host(lib):
    L = lib.lib()
    st, h = _create(lib, _desc(lib))
    assert st == 0
    ok = lib.StepOpts()
    # no plan; unknown enums; missing transport: rejected before any device work
    assert L.fks_step_ex(None, None, None, None, 0.01, 1, ctypes.byref(ok), None) == -1
    for bad in (lib.StepOpts(collision=7), lib.StepOpts(integrator=9)):
        assert L.fks_step_ex(h, None, None, None, 0.01, 1, ctypes.byref(bad), None) == -1
        assert L.fks_last_error()
    bgk = lib.StepOpts(collision=lib.FKS_COLL_BGK, nu=1.0)
    assert L.fks_step_ex(h, None, None, None, 0.01, 1, ctypes.byref(bgk), None) == -1   # null transport
    # the Boltzmann operator needs a bound plan
    assert L.fks_step_ex(h, None, None, None, 0.01, 1, ctypes.byref(ok), None) == -5
    L.fks_plan_destroy(h)
