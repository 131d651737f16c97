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


# The paper's own Boltzmann mesh (§5, 3D Sod explosion): 64^3 cells x 16^3 velocities on
# the velocity box [-15, 15)^3, ball |x - (1,1,1)| < 0.2 at rho = 1, T = 5, elsewhere
# rho = 0.125, T = 4, u = 0; 33 steps to t = 0.07.  Carleman radius R = 0.75 L (the ratio
# of the n = 32 workloads, inside the no-overlap bound 4L/(3+sqrt 2)).
SOD_N, SOD_L = 16, 15.0
SOD_R = 0.75 * SOD_L
SOD_SHAPE = (64, 64, 64)
SOD_DX = 2.0 / 64
SOD_DT = 0.07 / 33


def sod_box_device():
    m_in, m_out = fks_inputs.maxwellian_on_grid(SOD_N, SOD_L, [1.0, 0.125], [[0.0] * 3, [0.0] * 3], [5.0, 4.0])
    xs = (np.arange(SOD_SHAPE[0]) + 0.5) * SOD_DX
    X, Y, Z = np.meshgrid(xs, xs, xs, indexing="ij")
    inside = (((X - 1) ** 2 + (Y - 1) ** 2 + (Z - 1) ** 2) < 0.04).reshape(-1)
    mi = torch.tensor(m_in, dtype=torch.float32, device="cuda").reshape(1, -1)
    mo = torch.tensor(m_out, dtype=torch.float32, device="cuda").reshape(1, -1)
    ins = torch.tensor(inside, device="cuda").reshape(-1, 1)
    f = torch.where(ins, mi, mo).reshape(-1, SOD_N, SOD_N, SOD_N).contiguous()
    return f, m_in, m_out, inside.reshape(SOD_SHAPE)


def test_sod_mesh_step_sampled_parity():
    from paper_1701_01608_amd import Plan, Transport, step
    f, m_in, m_out, inside = sod_box_device()
    mass0 = float(f.double().sum())
    plan = Plan(SOD_N, SOD_L, SOD_R, dtype="f32", max_cells=4096)
    xp = Transport(SOD_N, SOD_L, SOD_SHAPE, SOD_DX)
    step(plan, xp, f, SOD_DT, n_steps=1)
    torch.cuda.synchronize()
    mass1 = float(f.double().sum())
    vel = otr.velocity_table(SOD_N, SOD_L)
    delta, _ = otr.advance(np.zeros_like(vel), vel, SOD_DT, SOD_DX)
    assert np.abs(delta).max() >= 1     # the fastest particles change cell in this step
    op = oracle_plan(SOD_N, SOD_L, SOD_R)
    mi32, mo32 = m_in.astype(np.float32).reshape(-1), m_out.astype(np.float32).reshape(-1)
    # ball centre, ball edge (cells whose velocities come from both states), far corner
    cells = [(31, 31, 31), (32, 25, 32), (38, 32, 32), (0, 63, 5)]
    for (i, j, k) in cells:
        si = (i - delta[:, 0]) % SOD_SHAPE[0]
        sj = (j - delta[:, 1]) % SOD_SHAPE[1]
        sk = (k - delta[:, 2]) % SOD_SHAPE[2]
        fstar = np.where(inside[si, sj, sk], mi32, mo32).astype(np.float64).reshape(SOD_N, SOD_N, SOD_N)
        ref = fstar + SOD_DT * collide_fast(fstar, op)
        got = f[(i * SOD_SHAPE[1] + j) * SOD_SHAPE[2] + k].double().cpu().numpy()
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= 1e-6, (i, j, k, err)
    assert abs(mass1 - mass0) <= 1e-6 * mass0
