"""FKS split step on the full one-GPU share: 32^3 cells x 32^3 velocities, FP32.

Sampled cells against the oracle after one step (transport + Euler collision), and the
exact properties at full size: transport is a permutation (box mass unchanged by it),
the collision conserves each cell's mass to FP32 rounding.
"""

import numpy as np
import pytest
import torch

import fks_inputs
from oracle import make_plan as oracle_plan
from oracle import transport as otr
from oracle.collide import collide_fast

pytestmark = pytest.mark.gpu

N, L, R = 32, 8.0, 6.0
SHAPE = (32, 32, 32)
DX = 2.0 / 32
DT = 0.004375


def wave_box_device(amp=0.1):
    # f(x, v) = (1 + amp sin(pi x1)) M_{1,0,1}(v), cell centres x1 = (i + 1/2) dx
    M = fks_inputs.maxwellian_on_grid(N, L, [1.0], [[0.0, 0.0, 0.0]], [1.0])[0]
    x1 = (np.arange(SHAPE[0]) + 0.5) * DX
    dens = 1.0 + amp * np.sin(np.pi * x1)
    Mt = torch.tensor(M, dtype=torch.float32, device="cuda").reshape(1, 1, 1, N, N, N)
    dt = torch.tensor(dens, dtype=torch.float32, device="cuda").reshape(SHAPE[0], 1, 1, 1, 1, 1)
    f = (dt * Mt).expand(*SHAPE, N, N, N).contiguous().reshape(-1, N, N, N)
    return f, M, dens


def test_full_box_step_sampled_parity():
    from paper_1701_01608_amd import Plan, Transport, step
    f, M, dens = wave_box_device()
    mass0 = float(f.double().sum())
    plan = Plan(N, L, R, dtype="f32", max_cells=4096)
    xp = Transport(N, L, SHAPE, DX)
    step(plan, xp, f, DT, n_steps=1)
    torch.cuda.synchronize()
    mass1 = float(f.double().sum())
    # oracle for sampled cells: transported profile from the same FP64 offsets, then Euler
    vel = otr.velocity_table(N, L)
    delta, _ = otr.advance(np.zeros_like(vel), vel, DT, DX)
    op = oracle_plan(N, L, R)
    M32 = M.astype(np.float32).reshape(-1)
    cells = [(0, 0, 0), (7, 3, 30), (16, 16, 16), (31, 31, 0)]
    for (i, j, k) in cells:
        src_i = (i - delta[:, 0]) % SHAPE[0]
        fstar = (np.float32(1.0) * dens.astype(np.float32)[src_i] * M32).astype(np.float64)
        fstar = fstar.reshape(N, N, N)
        ref = fstar + DT * collide_fast(fstar, op)
        got = f[(i * SHAPE[1] + j) * SHAPE[2] + k].double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-6, (i, j, k, err)
    # transport permutes, the collision conserves mass per cell to FP32 rounding
    assert abs(mass1 - mass0) <= 1e-6 * mass0
