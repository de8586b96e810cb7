"""The sampled-cell oracle helpers used at full size, checked on boxes the oracle steps
whole: the samples must equal the whole-box oracle at the sampled cells exactly (same
arithmetic, cell by cell)."""
import numpy as np
import pytest

import lbm_workloads as W
import oracle as O
import sampled_oracle as SO


def _fields(dims, seed):
    nx, ny, nz = dims
    rho, u = W.random_near_equilibrium_fields((nz, ny, nx), seed=seed, drho=5e-3, umax=0.04)

    def at(x, y, z):
        return rho[z, y, x], u[:, z, y, x].T
    return rho, u, at


@pytest.mark.parametrize("dims", [(11, 9, 8), (6, 5, 9)])
@pytest.mark.parametrize("space", ["raw", "cumulant"])
def test_one_and_k_step_samples_equal_the_whole_box(dims, space):
    st = O.stencil("D3Q27")
    om = np.random.default_rng(1).uniform(0.7, 1.9, st.q)
    om[st.conserved] = 0.0
    m = O.Method("D3Q27", space, om)
    rho, u, at = _fields(dims, seed=2)
    pts = W.sample_cells(dims, 6, seed=3)
    df0 = O.init_equilibrium(m, rho, u)
    one = O.step(m, df0, 1)
    got1 = SO.one_step_samples(m, pts, dims, at)
    np.testing.assert_allclose(got1, one[:, pts[:, 2], pts[:, 1], pts[:, 0]].T, rtol=0, atol=1e-15)
    three = O.step(m, one, 2)
    got3 = SO.k_step_samples(m, pts, dims, at, 3)  # windows of 7 cells wrap the 5- and 6-cell axes
    np.testing.assert_allclose(got3, three[:, pts[:, 2], pts[:, 1], pts[:, 0]].T, rtol=0, atol=1e-15)
