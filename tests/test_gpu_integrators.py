"""Space-homogeneous BKW run (Heun steps on the device) and hipGraph replay, against the oracle."""

import numpy as np
import pytest
import torch

import fks_inputs
from oracle import bkw, make_plan as oracle_plan
from oracle.collide import collide_fast
from oracle.integrators import heun as oracle_heun
from oracle.tables import VHS

pytestmark = pytest.mark.gpu

N, L, R, C = 16, 8.0, 6.0, 1 / (4 * np.pi)


def _plan(dtype="f64"):
    from paper_1701_01608_amd import Plan
    return Plan(N, L, R, kernel="vhs", alpha=0.0, C=C, a1=2, a2=3, n_radial=8, dtype=dtype, max_cells=1)


def test_bkw_heun_trajectory_matches_oracle():
    # Maxwell molecules, M = 6 directions x 8 radial nodes, FP64, dt = 0.01, 100 steps
    f0 = fks_inputs.bkw_initial(N, L, 5.5)
    plan = _plan()
    f = torch.tensor(f0[None], device="cuda")
    plan.heun(f, 0.01, n_steps=100)
    torch.cuda.synchronize()
    got = f[0].cpu().numpy()
    op = oracle_plan(N, L, R, kernel=VHS, alpha=0.0, C=C, a1=2, a2=3, n_radial=8)
    ref = f0
    for _ in range(100):
        ref = oracle_heun(ref, lambda g: collide_fast(g, op), 0.01)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    v1 = fks_inputs.velocity_axis(N, L)
    V = np.stack(np.meshgrid(v1, v1, v1, indexing="ij"), -1)
    exact = bkw.f_bkw(6.5, V)
    bkw_err = np.abs(got - exact).max() / np.abs(exact).max()
    print(f"trajectory rel-L2 vs oracle {err:.2e}; max error vs BKW closed form {bkw_err:.3e}", flush=True)
    assert err <= 1e-10
    # the quadrature (6 directions x 8 radial nodes) limits the accuracy against the
    # closed form; the oracle with the same quadrature lands at 0.125
    assert bkw_err <= 0.15


def test_graph_replay_equals_eager_steps():
    from paper_1701_01608_amd import Graph
    plan = _plan()
    f0 = torch.tensor(fks_inputs.bkw_initial(N, L, 5.5)[None], device="cuda")
    eager = f0.clone()
    fg = f0.clone()
    tmp = (torch.empty_like(fg), torch.empty_like(fg))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with Graph(s) as g:
            plan.heun(fg, 0.01, n_steps=2, tmp=tmp, stream=s)
    torch.cuda.synchronize()
    assert torch.equal(fg, f0)                       # recording runs nothing
    for rep in range(4):
        with torch.cuda.stream(s):
            g.launch()
        s.synchronize()
        plan.heun(eager, 0.01, n_steps=2)            # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(fg, eager), f"replay {rep} differs from eager"


def test_graph_of_split_steps():
    from paper_1701_01608_amd import Graph, Plan, Transport, step
    n, shape, dt = 8, (4, 2, 2), 0.004375
    dx = 2.0 / shape[0]
    f0 = torch.tensor(fks_inputs.wave_box(n, L, shape), dtype=torch.float32, device="cuda")
    plan = Plan(n, L, R, dtype="f32", max_cells=16)
    xa = Transport(n, L, shape, dx)
    xb = Transport(n, L, shape, dx)
    eager = f0.clone()
    fg = f0.clone()
    tmp = torch.empty_like(fg)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with Graph(s) as g:
            step(plan, xb, fg, dt, n_steps=1, f_tmp=tmp, stream=s)
    for rep in range(3):
        with torch.cuda.stream(s):
            g.launch()
        s.synchronize()
        step(plan, xa, eager, dt, n_steps=1)
        torch.cuda.synchronize()
        assert torch.equal(fg, eager), f"replay {rep}"


def test_heun_on_a_batch_beyond_the_bounded_grid():
    # 40960 cells at n = 32 (1.34e9 values): the averaging kernel's grid covers 2^30
    # values and strides over the rest, so the cells past 32768 take the stride path.
    # Four hard-sphere mixtures repeated; sampled cells on both sides against the oracle.
    from paper_1701_01608_amd import Plan
    n, Lh, Rh, dt, reps = 32, 8.0, 6.0, 0.01, 10240
    base = fks_inputs.maxwellian_mixture(n, Lh, 4, seed=11).astype(np.float32)
    f = torch.tensor(base, device="cuda").repeat(reps, 1, 1, 1)
    assert f.numel() > 2 ** 30
    plan = Plan(n, Lh, Rh, a1=4, a2=4, C=0.25, dtype="f32", max_cells=4096)
    plan.heun(f, dt, n_steps=1)
    torch.cuda.synchronize()
    op = oracle_plan(n, Lh, Rh, a1=4, a2=4, C=0.25)
    cells = f.shape[0]
    for c in (5, cells - 1):
        ref = oracle_heun(base[c % 4].astype(np.float64), lambda x: collide_fast(x, op), dt)
        got = f[c].double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-6, (c, err)


def test_graph_recording_allocates_nothing_and_holds_its_buffers():
    # inside a recording the wrappers refuse to allocate (the allocation would be freed
    # while the graph keeps writing to it) and keep every buffer alive with the graph
    import gc
    from paper_1701_01608_amd import FKSError, Graph
    plan = _plan()
    f0 = torch.tensor(fks_inputs.bkw_initial(N, L, 5.5)[None], device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with pytest.raises(FKSError):
            with Graph(s):
                plan.collide(f0, stream=s)            # q omitted
    q = torch.empty_like(f0)
    fin = f0.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with Graph(s) as g:
            plan.collide(fin, q, stream=s)
    fin_id = id(fin)
    del fin                                           # now only the graph refers to it
    gc.collect()
    assert any(id(t) == fin_id for t in g._keep)
    assert any(t is q for t in g._keep) and any(o is plan for o in g._keep)
    with torch.cuda.stream(s):
        g.launch()
    s.synchronize()
    ref = plan.collide(f0)
    torch.cuda.synchronize()
    assert torch.equal(q, ref)
