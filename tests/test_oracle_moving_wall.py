"""Pins of the oracle's moving-wall term (Appendix A, closing remark on
non-stationary walls; reading R10).  What fixes it without retyping it:
  * the term carries no mass (the tangential moments of the reflected
    directions vanish by lattice symmetry): per-species mass stays exact;
  * its momentum, summed over a uniform wall layer at rest, follows from the
    lattice's second moments in closed form;
  * plane Couette flow between halfway walls with equal molar masses (c = 1,
    exact bounce-back) reaches the linear profile exactly; with the paper's
    rho_i w_i weighting the mixture sees the wall at U sum_i w_i^2."""
import numpy as np
import pytest
import torch

from oracle import evd
from oracle.lattice import DTYPE


def _d(n, v=0.05):
    return torch.full((n, n), v, dtype=DTYPE)


@pytest.mark.parametrize("case", ["d2q9_xwall", "d2q9_ywall", "d3q19_zwall"])
def test_moving_walls_conserve_species_mass(case):
    if case == "d2q9_xwall":
        m = evd.Model("D2Q9", 6, 5, 1, [1.0, 3.0, 7.0], _d(3), 0.8, g=[1e-4, 2e-4, 0],
                      walls=(True, False, False),
                      wall_velocity=[[0, 0.02, 0], [0, -0.01, 0]])
    elif case == "d2q9_ywall":
        m = evd.Model("D2Q9", 5, 6, 1, [1.0, 3.0], _d(2), 1.0, walls=(False, True, False),
                      wall_velocity=[[0.01, 0, 0], [0.03, 0, 0]])
    else:
        m = evd.Model("D3Q19", 3, 4, 5, [1.0, 2.0, 4.0], _d(3), 0.9, walls=(False, False, True),
                      wall_velocity=[[0.01, -0.02, 0], [0.0, 0.015, 0]])
    gen = torch.Generator().manual_seed(2)
    x0 = torch.rand(m.N, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE) + 0.1
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    m0 = f.sum(dim=(1, 2, 3, 4))
    f = evd.run(m, f, 60)
    assert ((f.sum(dim=(1, 2, 3, 4)) - m0).abs() / m0).max() < 1e-13


def test_moving_wall_momentum_of_a_uniform_layer():
    """Uniform state at rest, no force, D2Q9 with walls on x: one stream step
    adds to species i at each wall node the tangential momentum
    sum_a e_a 2 w_a rho_i w_i (e_a.u_w)/c_s^2 = 6 rho_i w_i M u_w with
    M_yy = sum over the three reflected directions of w_a c_y^2 = 1/18, i.e.
    rho_i w_i u_w,y / 3 (the species speed drops out)."""
    nx, ny = 4, 3
    U = [0.02, -0.01]
    m = evd.Model("D2Q9", nx, ny, 1, [1.0, 4.0], _d(2), 1.0, walls=(True, False, False),
                  wall_velocity=[[0, U[0], 0], [0, U[1], 0]])
    x = torch.tensor([0.3, 0.7], dtype=DTYPE)[:, None, None, None].expand(2, 1, ny, nx)
    f0 = evd.initial_populations(m, x.clone())
    rho_i = f0.sum(dim=1)[:, 0, 0, 0]
    w_i = rho_i / rho_i.sum()
    ms = evd.Model("D2Q9", nx, ny, 1, [1.0, 4.0], _d(2), 1.0, walls=(True, False, False))
    e = m.velocities()
    jy = lambda f: torch.einsum("nq,nqzyx->nzyx", e[:, :, 1], f)
    d = jy(evd.stream(m, f0)) - jy(evd.stream(ms, f0))               # [N, 1, ny, nx]
    for side, col in ((0, 0), (1, nx - 1)):
        want = rho_i * w_i * U[side] / 3.0
        got = d[:, 0, :, col]
        assert (got - want[:, None]).abs().max() < 1e-15
    assert d[:, 0, :, 1:-1].abs().max() < 1e-16


@pytest.mark.parametrize("x1", [1.0 - 1e-6, 0.5])
def test_couette_profile(x1):
    """Equal masses (both species at c = 1), walls on y at rest (bottom) and
    moving at U along x (top), periodic x: the steady mixture velocity is
    linear, u_x(y) = U_eff (y + 1/2)/ny, with U_eff = U sum_i w_i^2 from the
    rho_i w_i weighting of the wall term."""
    nx, ny, U = 2, 10, 1e-3
    m = evd.Model("D2Q9", nx, ny, 1, [1.0, 1.0], _d(2, 0.1), 1.0, walls=(False, True, False),
                  wall_velocity=[[0, 0, 0], [U, 0, 0]])
    x = torch.tensor([x1, 1.0 - x1], dtype=DTYPE)[:, None, None, None].expand(2, 1, ny, nx)
    f = evd.run(m, evd.initial_populations(m, x.clone()), 3000)
    u = evd.observables(m, f)["u"][0, :, 0, 0].numpy()
    w = np.array([x1, 1.0 - x1])
    want = U * (w * w).sum() * (np.arange(ny) + 0.5) / ny
    assert np.abs(u - want).max() < 1e-9 * U / 1e-3
    assert float(evd.observables(m, f)["u"][0, :, :, 1].abs().max()) < 1e-12


def test_wall_velocity_must_be_tangential():
    with pytest.raises(ValueError):
        evd.Model("D2Q9", 4, 5, 1, [1.0, 2.0], _d(2), 1.0, walls=(False, True, False),
                  wall_velocity=[[0, 0.01, 0], [0, 0, 0]])
