"""Pins of the oracle's lattice, equilibria, forcing term, collision and tau
solve.  Each check uses a fact the paper or the mathematics fixes, not the
oracle's own formula."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import closed_forms, evd, stability
from oracle.lattice import Lattice, DTYPE

torch.manual_seed(1234)


def _model(N=3, lattice="D2Q9", masses=None, g=(2e-3, -1e-3, 0.0), shape=(5, 4, 1),
           walls=(False, False, False), tau1=0.9, seed=0):
    rng = np.random.default_rng(seed)
    masses = masses or [1.0, 14.0, 22.0, 30.0][:N]
    D = rng.uniform(0.02, 0.1, size=(N, N))
    D = (D + D.T) / 2
    nx, ny, nz = shape
    return evd.Model(lattice, nx, ny, nz, masses, torch.tensor(D), tau1, g=list(g),
                     walls=walls)


def _random_state(m, seed=0, amp=0.2):
    gen = torch.Generator().manual_seed(seed)
    x0 = torch.rand(m.N, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE) + 0.1
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    return f * (1 + amp * torch.rand(f.shape, generator=gen, dtype=DTYPE))


# ------------------------------------------------------------------ lattice
@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_lattice_isotropy(name):
    """Weights are a quadrature of the Maxwellian moments up to 4th order:
    sum w = 1, sum w c = 0, sum w c c = I/3, sum w c_a c_b c_c c_d =
    (d_ab d_cd + d_ac d_bd + d_ad d_bc)/9, with exact rationals."""
    lat = Lattice(name)
    d = lat.dim
    w = lat.weights_exact
    assert sum(w) == 1
    for a in range(d):
        assert sum(wi * c[a] for wi, c in zip(w, lat.dirs)) == 0
        for b in range(d):
            s2 = sum(wi * c[a] * c[b] for wi, c in zip(w, lat.dirs))
            assert s2 == (Fraction(1, 3) if a == b else 0)
            for cc in range(d):
                s3 = sum(wi * c[a] * c[b] * c[cc] for wi, c in zip(w, lat.dirs))
                assert s3 == 0
                for dd in range(d):
                    s4 = sum(wi * c[a] * c[b] * c[cc] * c[dd] for wi, c in zip(w, lat.dirs))
                    want = Fraction(int(a == b and cc == dd) + int(a == cc and b == dd)
                                    + int(a == dd and b == cc), 9)
                    assert s4 == want
    for al, o in enumerate(lat.opp):
        assert tuple(-v for v in lat.dirs[al]) == lat.dirs[o]


def test_d2q9_numbering_matches_paper():
    """eq. (discrete_velocity_DLS): alpha = 1..4 at angles (alpha-1) pi/2,
    alpha = 5..8 at (alpha-5) pi/2 + pi/4, i.e. (1,0),(0,1),(-1,0),(0,-1),
    (1,1),(-1,1),(-1,-1),(1,-1)."""
    lat = Lattice("D2Q9")
    assert [d[:2] for d in lat.dirs] == [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                                        (1, 1), (-1, 1), (-1, -1), (1, -1)]


def test_dls_speeds_and_taus():
    """eq. (speed_DLS): c_i/c_1 = sqrt(M_1/M_i); and a common kinematic
    viscosity nu_i = (tau_i - 1/2) c_{s,i}^2 for all species (Sec. 3)."""
    m = _model(masses=[2.0, 28.0, 44.0])
    c = m.speeds()
    assert c[0] == 1.0
    assert abs(c[1] - math.sqrt(2.0 / 28.0)) < 1e-15
    nus = [(t - 0.5) * cs2 for t, cs2 in zip(m.taus(), m.sound2())]
    assert max(nus) - min(nus) < 1e-15


# --------------------------------------------------------------- equilibria
@pytest.mark.parametrize("lattice,N", [("D2Q9", 3), ("D3Q19", 4)])
def test_equilibrium_moments(lattice, N):
    """Hermite-expansion moments: sum f^eq = rho_i, sum e f^eq = rho_i u,
    sum e e f^eq = rho_i (c_s^2 I + u u); and for f^(0) of eq. (feqi0):
    sum f^(0) = rho_i, sum e f^(0) = rho_i u_i^eq (the property that makes
    Omega^ii,(0) = 0, Sec. 3)."""
    m = _model(N=N, lattice=lattice, shape=(3, 2, 2) if lattice == "D3Q19" else (4, 3, 1))
    gen = torch.Generator().manual_seed(3)
    shp = (m.nz, m.ny, m.nx)
    rho_i = 0.2 + torch.rand(N, *shp, generator=gen, dtype=DTYPE)
    ueq = 0.05 * (torch.rand(N, *shp, 3, generator=gen, dtype=DTYPE) - 0.5)
    if lattice == "D2Q9":
        ueq[..., 2] = 0
    u = (rho_i[..., None] * ueq).sum(0) / rho_i.sum(0)[..., None]
    feq, f0 = evd.equilibria(m, rho_i, ueq, u)
    e = m.velocities()
    cs2 = m.sound2()
    d = m.lat.dim
    for i in range(N):
        assert torch.allclose(feq[i].sum(0), rho_i[i], atol=1e-14)
        assert torch.allclose(f0[i].sum(0), rho_i[i], atol=1e-14)
        mom_eq = torch.einsum("qc,qzyx->zyxc", e[i], feq[i])
        mom_0 = torch.einsum("qc,qzyx->zyxc", e[i], f0[i])
        assert torch.allclose(mom_eq, rho_i[i][..., None] * u, atol=1e-14)
        assert torch.allclose(mom_0, rho_i[i][..., None] * ueq[i], atol=1e-14)
        P = torch.einsum("qa,qb,qzyx->zyxab", e[i], e[i], feq[i])
        want = rho_i[i][..., None, None] * (cs2[i] * torch.eye(3, dtype=DTYPE)
                                            + u[..., :, None] * u[..., None, :])
        assert torch.allclose(P[..., :d, :d], want[..., :d, :d], atol=1e-14)


@pytest.mark.parametrize("lattice,N", [("D2Q9", 3), ("D3Q19", 4)])
def test_forcing_moments(lattice, N):
    """eq. (CE_EQ52): sum_a S = 0; eq. (CE_EQ54): sum_a e S = F_i; and the
    second moment sum e e S = u F + F u that removes the spurious term of
    eq. (epecies_momentum_eq) (Sec. 3, before eq. CE_forcing_term_discretized)."""
    m = _model(N=N, lattice=lattice, shape=(3, 2, 2) if lattice == "D3Q19" else (4, 3, 1),
               g=(3e-3, -2e-3, 1e-3 if lattice == "D3Q19" else 0.0))
    gen = torch.Generator().manual_seed(5)
    shp = (m.nz, m.ny, m.nx)
    rho_i = 0.2 + torch.rand(N, *shp, generator=gen, dtype=DTYPE)
    u = 0.05 * (torch.rand(*shp, 3, generator=gen, dtype=DTYPE) - 0.5)
    if lattice == "D2Q9":
        u[..., 2] = 0
    S = evd.forcing_term(m, rho_i, u)
    e = m.velocities()
    d = m.lat.dim
    F = rho_i[..., None] * m.g[None, None, None, None, :]
    for i in range(N):
        assert torch.allclose(S[i].sum(0), torch.zeros_like(rho_i[i]), atol=1e-17)
        mom = torch.einsum("qc,qzyx->zyxc", e[i], S[i])
        assert torch.allclose(mom, F[i], atol=1e-17)
        P = torch.einsum("qa,qb,qzyx->zyxab", e[i], e[i], S[i])
        want = u[..., :, None] * F[i][..., None, :] + F[i][..., :, None] * u[..., None, :]
        assert torch.allclose(P[..., :d, :d], want[..., :d, :d], atol=1e-17)


# ---------------------------------------------------------------- collision
@pytest.mark.parametrize("lattice,N", [("D2Q9", 2), ("D2Q9", 3), ("D2Q9", 4), ("D3Q19", 4)])
def test_collision_invariants(lattice, N):
    """Per node and species: mass is conserved (eq. CE_EQ52 and the zero
    moment of Omega); the momentum changes by F_i - Theta_i (Sec. 3: the first
    moment of eq. CE_EQ24 with eq. CE_theta_definition); summed over species
    the friction cancels pairwise (tau_ij = tau_ji), so the mixture momentum
    changes by exactly sum_i F_i = rho k (recovered NSE, eq. NSE)."""
    m = _model(N=N, lattice=lattice,
               shape=(3, 2, 2) if lattice == "D3Q19" else (5, 4, 1),
               g=(2e-3, -1e-3, 1.5e-3 if lattice == "D3Q19" else 0.0))
    f = _random_state(m)
    ft = evd.collide(m, f)
    obs = evd.observables(m, f)
    e = m.velocities()
    assert torch.allclose(ft.sum(1), f.sum(1), atol=1e-15, rtol=0)
    dmom = torch.einsum("nqc,nqzyx->nzyxc", e, ft - f)
    F = obs["rho_i"][..., None] * m.g
    # Theta_i straight from eq. (CE_theta_definition) with the Luo-Girimaji
    # style y_ij of the oracle's solve (checked separately below).
    assert torch.allclose(dmom, F - obs["theta"], atol=1e-15, rtol=0)
    assert torch.allclose(obs["theta"].sum(0), torch.zeros_like(obs["theta"][0]), atol=1e-16)
    assert torch.allclose(dmom.sum(0), F.sum(0), atol=1e-15, rtol=0)


def test_force_consistent_init_has_zero_velocity():
    """Sec. 4.2: the initial populations use u_i0 = u_i^eq - F_i dt/(2 rho_i)
    so that the force-shifted moment of eq. (first_order_moment_force) gives
    the intended zero velocity."""
    m = _model(g=(1e-3, 2e-3, 0.0))
    x0 = torch.rand(m.N, 1, m.ny, m.nx, dtype=DTYPE) + 0.1
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    obs = evd.observables(m, f)
    assert obs["ueq"].abs().max() < 1e-15   # |k| = 2e-3: rounding only
    assert torch.allclose(obs["x"], x0, atol=1e-15)


# ---------------------------------------------------------------- tau solve
def _node_taus(m, rho_vals):
    rho_i = torch.tensor(rho_vals, dtype=DTYPE).reshape(-1, 1, 1, 1)
    ueq = torch.zeros(len(rho_vals), 1, 1, 1, 3, dtype=DTYPE)
    rho, u, n, p = evd.mixture(m, rho_i, ueq)
    Y = evd.cross_relaxation(m, rho_i, rho, n, p)[:, :, 0, 0, 0]
    return Y


def test_tau_binary_luo_girimaji():
    """N = 2 reduces to eq. (Luo&Girimaji_tau)."""
    m = _model(N=2, masses=[1.0, 7.0])
    for rho in ([0.3, 0.5], [1e-3, 0.9], [0.7, 1e-4]):
        Y = _node_taus(m, rho)
        want = closed_forms.luo_girimaji_tau(rho[0], rho[1], 1.0, 7.0, float(m.diff[0, 1]))
        assert abs(1.0 / Y[0, 1].item() - want) < 1e-13 * want


def test_tau_binary_erf_value():
    """Binary, equal masses, D_12 = 0.05 and n = 1 (rho = 1): p = 1/3 and
    tau_12 = 1/2 + 3 D_12 = 0.65 (eq. Luo&Girimaji_tau)."""
    m = evd.Model("D2Q9", 4, 1, 1, [1.0, 1.0], torch.tensor([[0, .05], [.05, 0]], dtype=DTYPE), 1.0)
    Y = _node_taus(m, [0.4, 0.6])
    assert abs(1.0 / Y[0, 1].item() - 0.65) < 1e-14


def test_tau_ternary_closed_form():
    """N = 3 reproduces the analytic ternary solution printed in Sec. 4.1."""
    m = _model(N=3, masses=[2.016, 16.043, 39.948])
    D = m.diff.tolist()
    for rho in ([0.01, 0.3, 0.6], [0.2, 0.2, 0.2], [0.5, 0.1, 1e-3]):
        Y = _node_taus(m, rho)
        t23, t12, t13 = closed_forms.ternary_taus(rho, m.M, D)
        assert abs(1 / Y[1, 2].item() - t23) < 1e-12 * abs(t23)
        assert abs(1 / Y[0, 1].item() - t12) < 1e-12 * abs(t12)
        assert abs(1 / Y[0, 2].item() - t13) < 1e-12 * abs(t13)


def test_tau_quaternary_reduces_to_ternary():
    """With rho_4 = 0 the pairs among species 1..3 satisfy the ternary system
    (every extra term carries rho_4), so they equal the Sec. 4.1 closed form."""
    m4 = _model(N=4, masses=[1.0, 2.0, 3.0, 4.0])
    D = m4.diff.tolist()
    rho = [0.1, 0.3, 0.25, 0.0]
    Y = _node_taus(m4, rho)
    t23, t12, t13 = closed_forms.ternary_taus(rho[:3], m4.M[:3], [r[:3] for r in D[:3]])
    assert abs(1 / Y[1, 2].item() - t23) < 1e-12 * t23
    assert abs(1 / Y[0, 1].item() - t12) < 1e-12 * t12
    assert abs(1 / Y[0, 2].item() - t13) < 1e-12 * t13


# ---------------------------------------------------------------- stability
def test_relaxation_matrix_predicts_uniform_evolution():
    """At a uniform periodic state the equilibrium velocities evolve as
    u(t+1) = (I - K) u(t) + k (oracle.stability); check one real step."""
    m = _model(N=3, shape=(3, 2, 1), g=(1e-3, 0.0, 0.0))
    x = [0.2, 0.5, 0.3]
    x0 = torch.tensor(x, dtype=DTYPE).reshape(3, 1, 1, 1).expand(3, 1, 2, 3).clone()
    f = evd.initial_populations(m, x0)
    # give the species different velocities through an extra first moment
    e = m.velocities()
    cs2 = torch.tensor(m.sound2(), dtype=DTYPE)
    kick = torch.tensor([[0.01, 0.0], [-0.004, 0.003], [0.002, -0.002]], dtype=DTYPE)
    for i in range(3):
        ev = torch.cat([kick[i], torch.zeros(1, dtype=DTYPE)])
        # additive first-moment kick: sum_a w e = 0 keeps rho_i unchanged
        rho_i = f[i].sum(0)
        f[i] = f[i] + m.lat.w[:, None, None, None] * rho_i[None] \
            * (e[i] @ ev / cs2[i])[:, None, None, None]
    u0 = evd.observables(m, f)["ueq"][:, 0, 0, 0, :2].numpy()
    u1 = evd.observables(m, evd.step(m, f))["ueq"][:, 0, 0, 0, :2].numpy()
    K = stability.relaxation_matrix(m, x)
    pred = (np.eye(3) - K) @ u0 + np.array([1e-3, 0.0])[None, :]
    assert np.abs(u1 - pred).max() < 1e-15


@pytest.mark.parametrize("lattice,shape,walls", [("D2Q9", (40, 3, 1), (True, False, False)),
                                                 ("D3Q19", (6, 5, 7), (False, False, True))])
def test_an_absent_species_changes_nothing(lattice, shape, walls):
    """A species with rho_i = 0 everywhere (reading R4: u_i^eq = g/2, every
    term it enters is multiplied by rho_i) stays exactly 0, and the others
    evolve exactly as the mixture without it (same masses, diffusivities,
    n0 and force): the cross collision x_s x_t (u_t - u_s)/D_st and the
    tau relation lose every term of the absent species."""
    nx, ny, nz = shape
    D3 = torch.tensor([[0, 0.07, 0.05], [0.07, 0, 0.09], [0.05, 0.09, 0]], dtype=DTYPE)
    g = [1e-5, 0.0, 0.0] if lattice == "D2Q9" else [0.0, 0.0, -1e-5]
    rng = np.random.default_rng(6)
    x = np.zeros((3, nz, ny, nx))
    x[0] = rng.uniform(0.2, 0.8, size=(nz, ny, nx))
    x[1] = 1 - x[0]
    m3 = evd.Model(lattice, nx, ny, nz, [2.0, 28.0, 44.0], D3, 1.0, g=g, walls=walls,
                   n0=1 / 44)
    m2 = evd.Model(lattice, nx, ny, nz, [2.0, 28.0], D3[:2, :2].clone(), 1.0, g=g,
                   walls=walls, n0=1 / 44)
    f3 = evd.initial_populations(m3, torch.tensor(x, dtype=DTYPE))
    f2 = evd.initial_populations(m2, torch.tensor(x[:2], dtype=DTYPE))
    for _ in range(12):
        f3 = evd.step(m3, f3)
        f2 = evd.step(m2, f2)
    assert f3[2].abs().max() == 0.0
    assert (f3[:2] - f2).abs().max() < 1e-15
