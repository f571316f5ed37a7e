"""Pins of the oracle's diffusion-driven forcing contribution S_diff
(eq. improved_forcing_scheme).  The checks use what the mathematics fixes:
the lattice's moment isotropy up to fourth order gives its velocity moments
in closed form, and the pairwise symmetry of tau_ij makes the Theta_i sum to
zero."""
import math

import numpy as np
import pytest
import torch

from oracle import evd
from oracle.lattice import DTYPE


def _model(lattice, N, forcing="standard", seed=0, shape=None):
    rng = np.random.default_rng(seed)
    masses = [1.0, 3.0, 7.0, 12.0][:N]
    D = rng.uniform(0.03, 0.1, size=(N, N))
    D = (D + D.T) / 2
    shape = shape or ((5, 4, 1) if lattice == "D2Q9" else (3, 3, 3))
    return evd.Model(lattice, *shape, masses, torch.tensor(D), 0.8,
                     g=[1e-3, -2e-3, 5e-4 if lattice == "D3Q19" else 0.0], forcing=forcing)


def _state(m, seed=0):
    gen = torch.Generator().manual_seed(seed)
    x0 = torch.rand(m.N, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE) + 0.1
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    # a velocity and composition field so that u and the u_i^eq differ
    return f * (1 + 0.3 * torch.rand(f.shape, generator=gen, dtype=DTYPE))


def _quantities(m, f):
    rho_i, ueq = evd.species_moments(m, f)
    rho, u, n, p = evd.mixture(m, rho_i, ueq)
    Y = evd.cross_relaxation(m, rho_i, rho, n, p)
    return rho_i, ueq, rho, u, Y


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("N", [2, 3, 4])
def test_diffusion_forcing_moments(lattice, N):
    """sum_a S_diff = 0 and sum_a e S_diff = 0 (no mass or momentum source),
    and sum_a e e S_diff = (u Theta + Theta u)/(2 tau_i - 1): with the
    lattice's fourth-order isotropy, sum_a w e e (e.u)(e.Theta) =
    c^4 (u Theta + Theta u + (u.Theta) I)."""
    m = _model(lattice, N)
    f = _state(m, seed=N)
    rho_i, ueq, rho, u, Y = _quantities(m, f)
    th = evd.theta(m, rho_i, rho, ueq, Y)
    S = evd.diffusion_forcing(m, th, u)                   # [N, Q, z, y, x]
    e = m.velocities()
    tau = m.taus()
    scale = th.abs().max() * u.abs().max()
    for i in range(N):
        assert S[i].sum(0).abs().max() <= 1e-12 * scale
        first = torch.einsum("qc,qzyx->zyxc", e[i], S[i])
        assert first.abs().max() <= 1e-12 * scale
        second = torch.einsum("qc,qd,qzyx->zyxcd", e[i], e[i], S[i])
        want = (u[..., :, None] * th[i][..., None, :] + th[i][..., :, None] * u[..., None, :]) \
            / (2.0 * tau[i] - 1.0)
        assert (second - want).abs().max() <= 1e-12 * scale


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_theta_cancels_pairwise(lattice):
    """tau_ij = tau_ji, so sum_i Theta_i = 0 at every node."""
    m = _model(lattice, 4)
    rho_i, ueq, rho, u, Y = _quantities(m, _state(m, seed=9))
    th = evd.theta(m, rho_i, rho, ueq, Y)
    assert th.sum(0).abs().max() <= 1e-15 * th.abs().max() * 8


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_corrected_collision_changes_only_the_second_moment(lattice):
    """The corrected collision differs from the standard one by
    (1 - 1/(2 tau_i)) S_diff: per-species mass and momentum are unchanged, and
    the second moment moves by (u Theta_i + Theta_i u)/(2 tau_i)."""
    ms = _model(lattice, 3, "standard")
    md = _model(lattice, 3, "diff")
    f = _state(ms, seed=4)
    diff = evd.collide(md, f) - evd.collide(ms, f)
    rho_i, ueq, rho, u, Y = _quantities(ms, f)
    th = evd.theta(ms, rho_i, rho, ueq, Y)
    e = ms.velocities()
    tau = ms.taus()
    scale = th.abs().max() * u.abs().max()
    # the difference of two collisions of O(0.1) populations carries about
    # 1e-17 of absolute rounding
    tol = 1e-14
    for i in range(3):
        assert diff[i].sum(0).abs().max() <= tol
        assert torch.einsum("qc,qzyx->zyxc", e[i], diff[i]).abs().max() <= tol
        second = torch.einsum("qc,qd,qzyx->zyxcd", e[i], e[i], diff[i])
        want = (u[..., :, None] * th[i][..., None, :] + th[i][..., :, None] * u[..., None, :]) \
            / (2.0 * tau[i])
        assert (second - want).abs().max() <= tol + 1e-10 * scale
        assert want.abs().max() > 1e3 * tol      # the correction is visible


def test_diffusion_forcing_vanishes_without_velocity_difference():
    """Equal species velocities give Theta_i = 0 and no correction."""
    m = _model("D2Q9", 3, "diff")
    gen = torch.Generator().manual_seed(3)
    x0 = torch.rand(3, 1, 4, 5, generator=gen, dtype=DTYPE) + 0.1
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)      # all species at u_i0 = -g/2
    ms = _model("D2Q9", 3, "standard")
    assert (evd.collide(m, f) - evd.collide(ms, f)).abs().max() <= 1e-17


# ------------------------------------------------ pressure and density terms
def _walled(lattice, forcing="standard", N=3, seed=0):
    """A wall on x (2-D) or z (3-D) so both gradient forms are exercised."""
    walls = (True, False, False) if lattice == "D2Q9" else (False, False, True)
    shape = (6, 5, 1) if lattice == "D2Q9" else (4, 3, 5)
    rng = np.random.default_rng(seed)
    D = rng.uniform(0.03, 0.1, size=(N, N))
    D = (D + D.T) / 2
    return evd.Model(lattice, *shape, [1.0, 3.0, 7.0, 12.0][:N], torch.tensor(D), 0.8,
                     g=[1e-3, -2e-3, 5e-4 if lattice == "D3Q19" else 0.0], walls=walls,
                     forcing=forcing)


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_gradient_is_exact_for_quadratics_and_wraps_sinusoids(lattice):
    """The central difference and the one-sided wall differences are exact
    for any quadratic along a wall axis; on a periodic axis of n nodes the
    central difference of sin(2 pi k x/n) is cos(2 pi k x/n) sin(2 pi k/n)."""
    m = _walled(lattice)
    wa = 0 if lattice == "D2Q9" else 2
    n = m.shape_axis(wa)
    zz, yy, xx = torch.meshgrid(torch.arange(m.nz, dtype=DTYPE), torch.arange(m.ny, dtype=DTYPE),
                                torch.arange(m.nx, dtype=DTYPE), indexing="ij")
    r = (xx, yy, zz)[wa]
    phi = 0.7 - 0.3 * r + 0.05 * r * r
    g = evd.gradient(m, phi)
    assert (g[..., wa] - (-0.3 + 0.1 * r)).abs().max() < 1e-14
    # periodic axis (y), with the wall axis fixed
    k = 2
    th = 2 * math.pi * k / m.ny
    phi = torch.sin(th * yy) + 0 * xx
    g = evd.gradient(m, phi)
    assert (g[..., 1] - torch.cos(th * yy) * math.sin(th)).abs().max() < 1e-14
    assert g[..., wa].abs().max() < 1e-15
    assert n >= 3


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_pressure_and_density_terms_moments(lattice):
    """Both terms carry no mass and no momentum; their second moments are
    u G + G u (G = c_s^2 grad rho_i) and c_s^2 w_i (u_i^eq grad rho +
    grad rho u_i^eq), by the lattice's fourth-order isotropy."""
    m = _walled(lattice, N=3)
    f = _state(m, seed=6)
    rho_i, ueq, rho, u, Y = _quantities(m, f)
    Sp = evd.pressure_forcing(m, rho_i, u)
    Sr = evd.density_forcing(m, rho_i, rho, ueq)
    e = m.velocities()
    cs2 = m.sound2()
    gr = evd.gradient(m, rho)
    for i in range(3):
        G = cs2[i] * evd.gradient(m, rho_i[i])
        for S, want in (
                (Sp[i], u[..., :, None] * G[..., None, :] + G[..., :, None] * u[..., None, :]),
                (Sr[i], cs2[i] * (rho_i[i] / rho)[..., None, None]
                 * (ueq[i][..., :, None] * gr[..., None, :] + gr[..., :, None] * ueq[i][..., None, :]))):
            scale = want.abs().max()
            assert scale > 0
            assert S.sum(0).abs().max() <= 1e-12 * scale
            assert torch.einsum("qc,qzyx->zyxc", e[i], S).abs().max() <= 1e-12 * scale
            second = torch.einsum("qc,qd,qzyx->zyxcd", e[i], e[i], S)
            assert (second - want).abs().max() <= 1e-12 * scale


@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_full_corrected_collision_moves_only_the_second_moment(lattice):
    """With the whole eq. (improved_forcing_scheme) the collision differs from
    the standard one by (1 - 1/(2 tau_i)) (S_diff - S_p + S_rho): per-species
    mass and momentum are unchanged, and the second moment moves by
    (u Theta + Theta u)/(2 tau_i) + (1 - 1/(2 tau_i)) [c_s^2 w_i (u_i^eq grad rho
    + grad rho u_i^eq) - (u G + G u)]."""
    ms = _walled(lattice, "standard")
    mf = _walled(lattice, "full")
    f = _state(ms, seed=8)
    diff = evd.collide(mf, f) - evd.collide(ms, f)
    rho_i, ueq, rho, u, Y = _quantities(ms, f)
    th = evd.theta(ms, rho_i, rho, ueq, Y)
    e = ms.velocities()
    tau = ms.taus()
    cs2 = ms.sound2()
    gr = evd.gradient(ms, rho)
    tol = 1e-14
    outer = lambda a, b: a[..., :, None] * b[..., None, :] + b[..., :, None] * a[..., None, :]
    for i in range(3):
        G = cs2[i] * evd.gradient(ms, rho_i[i])
        want = outer(u, th[i]) / (2.0 * tau[i]) + (1.0 - 0.5 / tau[i]) * (
            cs2[i] * (rho_i[i] / rho)[..., None, None] * outer(ueq[i], gr) - outer(u, G))
        assert diff[i].sum(0).abs().max() <= tol
        assert torch.einsum("qc,qzyx->zyxc", e[i], diff[i]).abs().max() <= tol
        second = torch.einsum("qc,qd,qzyx->zyxcd", e[i], e[i], diff[i])
        assert (second - want).abs().max() <= tol + 1e-10 * want.abs().max()
        assert want.abs().max() > 1e3 * tol


def test_full_forcing_reduces_to_standard_on_a_uniform_state():
    """A uniform composition at rest relative to the force (no gradients, no
    velocity differences): the three corrections vanish."""
    m = _walled("D2Q9", "full")
    ms = _walled("D2Q9", "standard")
    x0 = torch.tensor([0.2, 0.3, 0.5], dtype=DTYPE)[:, None, None, None].expand(3, 1, 5, 6)
    f = evd.initial_populations(m, x0.clone())
    assert (evd.collide(m, f) - evd.collide(ms, f)).abs().max() <= 1e-17


def test_full_forcing_needs_three_nodes_on_a_wall_axis():
    with pytest.raises(ValueError):
        evd.Model("D2Q9", 2, 4, 1, [1.0, 2.0], torch.tensor([[0, 0.05], [0.05, 0]], dtype=DTYPE),
                  1.0, walls=(True, False, False), forcing="full")
