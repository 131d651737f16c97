"""fks_noneq (normalised non-equilibrium residual per cell) against the oracle."""

import numpy as np
import pytest
import torch

import fks_inputs
from oracle.bgk import noneq_residual
from oracle.grid import make_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,dtype", [(32, "f32"), (32, "f64"), (16, "f64")])
def test_noneq_matches_oracle(n, dtype):
    from paper_1701_01608_amd import Plan
    L = 8.0
    f = np.concatenate([fks_inputs.maxwellian_mixture(n, L, 5, seed=40 + n),
                        fks_inputs.maxwellian_on_grid(n, L, [0.8], [[0.2, -0.1, 0.0]], [1.0])])
    td = torch.float32 if dtype == "f32" else torch.float64
    ft = torch.tensor(f, dtype=td, device="cuda")
    plan = Plan(n, L, 6.0, dtype=dtype, max_cells=8)
    r = plan.noneq(ft).cpu().numpy()
    g = make_grid(n, L)
    fu = ft.double().cpu().numpy()
    ref = np.array([noneq_residual(fu[c], g) for c in range(len(fu))])
    print("noneq", r, ref, flush=True)
    np.testing.assert_allclose(r, ref, rtol=1e-9, atol=1e-12)
    assert ref[-1] < 1e-6 and ref[:-1].min() > 1e-3
