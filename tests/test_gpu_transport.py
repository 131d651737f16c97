"""Transport and the split step on the GPU against the oracle (bitwise where integer)."""

import numpy as np
import pytest
import torch

import fks_inputs
from oracle import make_plan as oracle_plan
from oracle import transport as otr
from oracle.collide import collide_fast
from oracle.integrators import fks_step as oracle_step
from oracle.conserve import moments as oracle_moments

pytestmark = pytest.mark.gpu


def test_transport_offsets_and_roll_bitwise():
    from paper_1701_01608_amd import Transport
    n, L, shape, dx, dt = 8, 8.0, (4, 3, 5), 1.0 / 16, 0.004375
    xp = Transport(n, L, shape, dx)
    rng = np.random.default_rng(3)
    f = rng.random((np.prod(shape), n, n, n))
    cur = torch.tensor(f, device="cuda")
    vel = otr.velocity_table(n, L)
    s = np.zeros_like(vel)
    host = f.reshape(len(f), -1)
    tot = np.zeros(vel.shape, dtype=np.int64)
    for step in range(25):
        nxt = xp(cur, dt=dt)
        d, s = otr.advance(s, vel, dt, dx)
        tot += d
        host = otr.shift(host, d, shape)
        cur = nxt
    torch.cuda.synchronize()
    gs, go = xp.offsets()
    assert np.array_equal(gs.cpu().numpy(), s)                    # FP64 offsets bitwise
    assert np.array_equal(go.cpu().numpy().astype(np.int64), tot)  # integer shifts exact
    assert np.array_equal(cur.cpu().numpy().reshape(host.shape), host)


@pytest.mark.parametrize("n", [8, 16])
def test_deferred_transport_equals_stepwise(n):
    # offsets advanced for several steps without moving f, then one materialising call:
    # the same f (bit for bit) as moving f every step, and the oracle's composed shift;
    # a Boltzmann step after unmaterialised steps applies the pending shifts with its own
    from paper_1701_01608_amd import Transport
    L, shape, dx, dt = 8.0, (4, 3, 5), 1.0 / 16, 0.004375
    rng = np.random.default_rng(5)
    f = torch.tensor(rng.random((np.prod(shape), n, n, n)), device="cuda")
    xa, xb = Transport(n, L, shape, dx), Transport(n, L, shape, dx)
    cur = f
    for _ in range(7):
        cur = xa(cur, dt=dt)                       # materialised every step
    for _ in range(7):
        xb.advance(dt)                             # offsets only
    deferred = xb.materialize(f)
    torch.cuda.synchronize()
    assert torch.equal(deferred, cur)
    vel = otr.velocity_table(n, L)
    s = np.zeros_like(vel)
    tot = np.zeros(vel.shape, dtype=np.int64)
    for _ in range(7):
        d, s = otr.advance(s, vel, dt, dx)
        tot += d
    host = otr.shift(f.cpu().numpy().reshape(len(f), -1), tot, shape)
    assert np.array_equal(deferred.cpu().numpy().reshape(host.shape), host)
    assert np.array_equal(xb.offsets()[1].cpu().numpy().astype(np.int64), tot)
    # nothing pending after a materialisation: moving again with dt = 0 is the identity
    again = xb.materialize(deferred)
    torch.cuda.synchronize()
    assert torch.equal(again, deferred)


def test_deferred_shifts_enter_the_dm_update():
    # two unmaterialised steps, then a Boltzmann step with eq. DM_update: the conservative
    # variables equal the direct moments of the moved masses (the shift conserves them)
    from paper_1701_01608_amd import Plan, Transport, step_ex
    n, L, R, shape, dx, dt = 8, 8.0, 6.0, (5, 4, 3), 1.0 / 8, 0.02
    f = torch.tensor(fks_inputs.maxwellian_mixture(n, L, int(np.prod(shape)), seed=8), device="cuda")
    plan = Plan(n, L, R, dtype="f64", max_cells=64)
    xp = Transport(n, L, shape, dx)
    cons = plan.moments(f)
    xp.advance(dt)
    xp.advance(dt)
    step_ex(plan, xp, f, 0.0, cons=cons)           # dt = 0: the pending shifts only, no collision change
    torch.cuda.synchronize()
    direct = plan.moments(f)
    np.testing.assert_allclose(cons.cpu().numpy(), direct.cpu().numpy(), rtol=0,
                               atol=1e-13 * direct.abs().max().item())
    vel = otr.velocity_table(n, L)
    s = np.zeros_like(vel)
    tot = np.zeros(vel.shape, dtype=np.int64)
    for _ in range(2):
        d, s = otr.advance(s, vel, dt, dx)
        tot += d
    assert np.any(tot != 0)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fks_step_small_box(dtype):
    from paper_1701_01608_amd import Plan, Transport, step
    n, L, R, shape, dt = 8, 8.0, 6.0, (4, 2, 2), 0.004375
    dx = 2.0 / shape[0]
    f = fks_inputs.wave_box(n, L, shape)
    td = torch.float32 if dtype == "f32" else torch.float64
    plan = Plan(n, L, R, dtype=dtype, max_cells=5)
    xp = Transport(n, L, shape, dx)
    ft = torch.tensor(f, dtype=td, device="cuda")
    fu = ft.double().cpu().numpy()
    mom = torch.empty((np.prod(shape), 5), dtype=torch.float64, device="cuda")
    step(plan, xp, ft, dt, n_steps=3, moments=mom)
    torch.cuda.synchronize()
    op = oracle_plan(n, L, R)
    vel = otr.velocity_table(n, L)
    s = np.zeros_like(vel)
    g = fu
    for _ in range(3):
        g, s, _d = oracle_step(g, s, vel, shape, dx, dt, collide=lambda c: collide_fast(c, op))
        if dtype == "f32":
            g = g.astype(np.float32).astype(np.float64)
    out = ft.double().cpu().numpy()
    tol = 1e-5 if dtype == "f32" else 1e-11
    assert np.linalg.norm(out - g) / np.linalg.norm(g) <= tol
    np.testing.assert_allclose(mom.cpu().numpy(), oracle_moments(out, op.grid), rtol=1e-12, atol=1e-14)


def test_roll_beyond_2_pow_32_elements():
    # 64 x 64 x 33 cells x 32^3 velocities = 4.43e9 values (17.7 GB per FP32 buffer): one
    # launch of one thread per value would exceed the 2^32 threads of a grid, so the roll
    # strides over cells.  Each cell holds its own index (exact in FP32 below 2^24); after
    # one step every sampled cell must hold, per velocity, the index of its source cell.
    from paper_1701_01608_amd import Transport
    n, L, shape, dx, dt = 32, 15.0, (64, 64, 33), 2.0 / 64, 0.07 / 33
    cells, nv = int(np.prod(shape)), n ** 3
    assert cells * nv > 2 ** 32
    f = torch.arange(cells, dtype=torch.float32, device="cuda").reshape(-1, 1).expand(cells, nv).contiguous()
    xp = Transport(n, L, shape, dx)
    out = xp(f.view(cells, n, n, n), dt=dt)
    torch.cuda.synchronize()
    del f
    vel = otr.velocity_table(n, L)
    d, _ = otr.advance(np.zeros_like(vel), vel, dt, dx)
    assert np.abs(d).max() >= 1
    for c in (0, 1, cells // 2 + 7, cells - 1):
        cx, cy, cz = c // (shape[1] * shape[2]), (c // shape[2]) % shape[1], c % shape[2]
        src = (((cx - d[:, 0]) % shape[0]) * shape[1] + (cy - d[:, 1]) % shape[1]) * shape[2] + (cz - d[:, 2]) % shape[2]
        got = out[c].reshape(-1).cpu().numpy()
        assert np.array_equal(got, src.astype(np.float32)), c
