"""fks_collide_noalloc (the entry point for callers that cannot allocate) against
fks_collide on the same plan and inputs: two calls in a row, the second smaller, through
the C ABI; its limit and the tables-only binding it runs on."""

import ctypes

import numpy as np
import pytest
import torch

import fks_inputs

pytestmark = pytest.mark.gpu


def _tables_only_plan(n, dtype, max_cells):
    # a plan whose only device buffer is its table buffer (no workspace bound)
    from paper_1701_01608_amd import _lib
    L = _lib.lib()
    desc = _lib.CollideDesc(n=n, kernel=_lib.FKS_HARD_SPHERES, L=8.0, R=6.0, alpha=0.0, C=0.25, a1=4, a2=4,
                            n_radial=8, dtype=_lib.FKS_F32 if dtype == "f32" else _lib.FKS_F64, flags=0, reserved=0)
    h = ctypes.c_void_p()
    _lib.check(L.fks_plan_create(ctypes.byref(desc), max_cells, ctypes.byref(h)))
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _lib.check(L.fks_plan_sizes(h, ctypes.byref(tb), ctypes.byref(wb)))
    tables = torch.empty(tb.value, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    _lib.check(L.fks_plan_bind(h, ctypes.c_void_p(tables.data_ptr()), tb.value, None, 0, ctypes.c_void_p(s)))
    return h, tables


@pytest.mark.parametrize("n,dtype,sizes", [(32, "f32", (200, 37)), (16, "f64", (64, 5)), (24, "f32", (120, 9))])
def test_noalloc_matches_collide_twice(n, dtype, sizes):
    from paper_1701_01608_amd import Plan, _lib
    L = _lib.lib()
    print(f"case no-alloc n={n} {dtype} sizes={sizes}", flush=True)
    td = torch.float32 if dtype == "f32" else torch.float64
    ref_plan = Plan(n, 8.0, 6.0, dtype=dtype, max_cells=max(sizes))
    h, tables = _tables_only_plan(n, dtype, max(sizes))
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for i, cells in enumerate(sizes):
        f = torch.tensor(fks_inputs.maxwellian_mixture(n, 8.0, cells, seed=900 + i), dtype=td, device="cuda")
        q = torch.full_like(f, float("nan"))
        _lib.check(L.fks_collide_noalloc(h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), cells, s))
        ref = ref_plan.collide(f)
        torch.cuda.synchronize()
        # same kernels and launch sequence on the same inputs: identical results
        assert torch.equal(q, ref), (n, dtype, cells)
    # the workspace entry points refuse a plan bound without a workspace
    f = torch.zeros((2, n, n, n), dtype=td, device="cuda")
    q = torch.empty_like(f)
    assert L.fks_collide(h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), 2, s) == -5
    L.fks_plan_destroy(h)


def test_noalloc_rejects_batches_beyond_its_scratch():
    from paper_1701_01608_amd import _lib
    L = _lib.lib()
    n = 32
    h, tables = _tables_only_plan(n, "f32", 4096)
    f = torch.zeros((4096, n, n, n), dtype=torch.float32, device="cuda")
    q = torch.empty_like(f)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = L.fks_collide_noalloc(h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), 4096, s)
    assert st == -1
    msg = L.fks_last_error().decode()
    assert "MiB library scratch" in msg
    cap = int(msg.split("(")[-1].split()[0])
    assert 100 <= cap < 4096
    assert L.fks_collide_noalloc(h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), cap, s) == 0
    assert L.fks_collide_noalloc(h, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(q.data_ptr()), cap + 1, s) == -1
    torch.cuda.synchronize()
    L.fks_plan_destroy(h)
