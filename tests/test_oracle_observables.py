"""Pins of the oracle's observables (Sec. 3): the real species velocity
u_i = u_i^eq - Theta_i/(2 rho_i) of eq. (CE_EQ83), with Theta_i of eq.
(CE_theta_definition).  Nothing else in the method fixes u_i, so it is pinned
by the relations the paper derives from it:
  * for a binary mixture, the cross-relaxation time of Luo and Girimaji (eq.
    Luo&Girimaji_tau) is exactly the one that makes eq. (CE_EQ102) hold:
    rho_1 rho_2/(rho p tau_12)(u_1^eq - u_2^eq) = x_1 x_2/D_12 (u_1 - u_2);
    a sign slip in eq. (CE_EQ83) turns the factor 1 - 1/(2 tau_12) that links
    the two velocity differences into 1 + 1/(2 tau_12), a factor-2 slip into
    1 - 1/tau_12, and either breaks the identity;
  * the species momenta sum to the mixture momentum, sum_i rho_i u_i = rho u
    (sum_i Theta_i = 0 and eq. Sirovich_mixture_velocity), for any N;
  * an absent species takes the limit value (reading R12)."""
import numpy as np
import pytest
import torch

from oracle import evd
from oracle.lattice import DTYPE


def _random_state(lattice, shape, masses, D, tau1, g, seed, spread=0.2):
    rng = np.random.default_rng(seed)
    N = len(masses)
    m = evd.Model(lattice, *shape, masses, torch.tensor(D, dtype=DTYPE), tau1, g=list(g))
    x0 = torch.tensor(rng.uniform(0.1, 1.0, size=(N, shape[2], shape[1], shape[0])))
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    f = f * (1 + spread * torch.tensor(rng.uniform(-1, 1, size=tuple(f.shape))))
    return m, f


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (7, 5, 1)), ("D3Q19", (4, 3, 5))])
@pytest.mark.parametrize("masses", [[1.0, 7.0], [2.0, 44.0], [1.0, 1.0]])
def test_binary_real_velocity_satisfies_ce_eq102(lattice, shape, masses):
    """With tau_12 from eq. (Luo&Girimaji_tau), computed here from the node's
    densities, the oracle's u_i satisfy eq. (CE_EQ102) node by node to
    rounding, in both velocity components."""
    D12 = 0.061
    D = [[0.0, D12], [D12, 0.0]]
    m, f = _random_state(lattice, shape, masses, D, 0.9, (3e-4, -2e-4, 1e-4), 5)
    ob = evd.observables(m, f)
    M = np.array(m.M)
    rho_i = ob["rho_i"].numpy()
    rho = rho_i.sum(0)
    n = (rho_i / M[:, None, None, None]).sum(0)
    p = n * M[0] / 3.0
    x = rho_i / (M[:, None, None, None] * n)
    tau12 = 0.5 + n * n * M[0] * M[1] * D12 / (p * rho)
    ueq = ob["ueq"].numpy()
    ui = ob["u_i"].numpy()
    lhs = (rho_i[0] * rho_i[1] / (rho * p * tau12))[..., None] * (ueq[0] - ueq[1])
    rhs = (x[0] * x[1] / D12)[..., None] * (ui[0] - ui[1])
    scale = np.abs(lhs).max()
    assert scale > 0
    assert np.abs(lhs - rhs).max() < 1e-12 * scale


def test_binary_velocity_difference_factor():
    """The same identity seen through the velocity differences: for N = 2,
    u_1 - u_2 = (1 - 1/(2 tau_12)) (u_1^eq - u_2^eq) exactly, with tau_12 from
    eq. (Luo&Girimaji_tau)."""
    D12 = 0.043
    m, f = _random_state("D2Q9", (9, 4, 1), [1.0, 14.0], [[0, D12], [D12, 0]], 1.0,
                         (1e-4, 0.0, 0.0), 8)
    ob = evd.observables(m, f)
    rho_i = ob["rho_i"].numpy()
    M = np.array(m.M)
    n = (rho_i / M[:, None, None, None]).sum(0)
    tau12 = 0.5 + 3.0 * n * M[0] * M[1] * D12 / rho_i.sum(0)
    du_eq = ob["ueq"][0].numpy() - ob["ueq"][1].numpy()
    du = ob["u_i"][0].numpy() - ob["u_i"][1].numpy()
    want = (1.0 - 0.5 / tau12)[..., None] * du_eq
    assert np.abs(du - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("lattice,shape,masses", [
    ("D2Q9", (6, 5, 1), [1.0, 14.0, 22.0]),
    ("D2Q9", (5, 6, 1), [1.0, 2.0, 3.0, 4.0]),
    ("D3Q19", (3, 4, 5), [1.0, 2.0, 3.0, 4.0]),
])
def test_species_momenta_sum_to_mixture_momentum(lattice, shape, masses):
    """sum_i rho_i u_i = rho u at every node: the Theta_i cancel in pairs
    (tau_ij = tau_ji) and u = sum_i w_i u_i^eq."""
    N = len(masses)
    rng = np.random.default_rng(3)
    d = rng.uniform(0.02, 0.1, size=(N, N))
    m, f = _random_state(lattice, shape, masses, ((d + d.T) / 2).tolist(), 1.0,
                         (2e-4, 1e-4, -1e-4), 4)
    ob = evd.observables(m, f)
    mom_i = (ob["rho_i"][..., None] * ob["u_i"]).sum(0)
    mom = ob["rho"][..., None] * ob["u"]
    assert (mom_i - mom).abs().max() < 1e-13 * mom.abs().max()
    # and the species velocities differ from u^eq by a nonzero amount
    assert (ob["u_i"] - ob["ueq"]).abs().max() > 1e-6 * ob["ueq"].abs().max()


def test_absent_species_takes_the_limit():
    """Reading R12: where rho_i = 0 the real velocity is the limit of
    u_i^eq - Theta_i/(2 rho_i) as rho_i -> 0.  Reading R4 gives an absent
    species u_i^eq = g/2, which is the u_i^eq of a species at rest of any
    density; so a species at rest with densities 1e-12 has nearly the u_i of
    the absent one."""
    masses = [1.0, 5.0, 9.0]
    rng = np.random.default_rng(2)
    d = rng.uniform(0.03, 0.1, size=(3, 3))
    D = ((d + d.T) / 2).tolist()
    m, f = _random_state("D2Q9", (6, 4, 1), masses, D, 1.0, (1e-4, 0.0, 0.0), 9)
    f0 = f.clone()
    f0[1] = 0.0
    ft = f.clone()
    ft[1] = 1e-12 * m.lat.w[:, None, None, None]
    u0 = evd.observables(m, f0)["u_i"][1]
    ut = evd.observables(m, ft)["u_i"][1]
    assert torch.isfinite(u0).all()
    assert (u0 - ut).abs().max() < 1e-9 * ut.abs().max()
