"""Pins of the oracle against closed forms and against the independent
per-node implementation (oracle.scalar).  The long runs here are the slowest
CPU tests (each about 5-20 s)."""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy.optimize import minimize_scalar

from oracle import closed_forms, evd, scalar
from oracle.lattice import DTYPE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


# ------------------------------------------------------------- brute force
BRUTE = [
    ("D2Q9", (5, 4, 1), [1.0, 14.0, 22.0], (True, False, False), (1e-3, -2e-3, 0.0)),
    ("D2Q9", (4, 5, 1), [1.0, 2.0, 3.0, 4.0], (False, True, False), (0.0, 1e-3, 0.0)),
    ("D2Q9", (5, 3, 1), [1.0, 1.0], (True, False, False), (2e-3, 0.0, 0.0)),
    ("D3Q19", (4, 3, 3), [1.0, 2.0, 3.0, 4.0], (False, False, True), (0.0, 5e-4, -1e-3)),
    ("D3Q19", (3, 3, 4), [1.0, 6.0, 9.0], (False, False, False), (1e-3, 0.0, 0.0)),
]


@pytest.mark.parametrize("lattice,shape,masses,walls,g", BRUTE)
def test_vectorised_equals_scalar_loops(lattice, shape, masses, walls, g):
    """The vectorised pull-form oracle equals the independent node-by-node
    push-form implementation on random states, over three steps."""
    N = len(masses)
    rng = np.random.default_rng(7)
    D = rng.uniform(0.02, 0.1, size=(N, N))
    D = (D + D.T) / 2
    m = evd.Model(lattice, *shape, masses, torch.tensor(D), 0.85, g=list(g), walls=walls)
    sm = scalar.ScalarModel(lattice, *shape, masses, D.tolist(), 0.85, g, walls)
    x0 = torch.tensor(rng.uniform(0.1, 1.0, size=(N, shape[2], shape[1], shape[0])))
    x0 = x0 / x0.sum(0)
    f = evd.initial_populations(m, x0)
    f = f * (1 + 0.2 * torch.tensor(rng.uniform(size=tuple(f.shape))))
    fs = f.tolist()
    for _ in range(3):
        f = evd.step(m, f)
        fs = sm.step(fs)
    assert torch.allclose(f, torch.tensor(fs, dtype=DTYPE), atol=1e-14, rtol=0)


# ------------------------------------------------------------------- erf
def test_binary_loschmidt_erf_and_exact_mass():
    """Binary, equal masses, D_12 = 0.05, tau = 1, 200 x 4, walls at the x
    ends, x_1 = 1 | 0 at the midpoint, 2000 steps: the mole fraction follows
    the erf solution of Fick's law with D_12 (the recovered Maxwell-Stefan
    equation, eq. MS_equation) and each species' mass is exactly conserved
    (Appendix A; Sec. 4.1 on the mass of the tube).  Measured: max deviation
    about 1e-4, fitted D within 0.1 %."""
    D = torch.tensor([[0.0, 0.05], [0.05, 0.0]], dtype=DTYPE)
    m = evd.Model("D2Q9", 200, 4, 1, [1.0, 1.0], D, 1.0, walls=(True, False, False))
    x0 = torch.zeros(2, 1, 4, 200, dtype=DTYPE)
    x0[0, ..., :100] = 1.0
    x0[1, ..., 100:] = 1.0
    f = evd.initial_populations(m, x0)
    m0 = f.sum(dim=(1, 2, 3, 4))
    f = evd.run(m, f, 2000)
    obs = evd.observables(m, f)
    x1 = obs["x"][0, 0, 0].numpy()
    assert np.abs(obs["x"][0].numpy() - x1[None, None]).max() < 1e-15   # y-uniform
    xs = np.arange(200)
    ref = closed_forms.binary_erf_profile(xs, 2000, 99.5, 0.05)
    assert np.abs(x1 - ref).max() < 5e-3
    fit = minimize_scalar(
        lambda Dv: ((closed_forms.binary_erf_profile(xs, 2000, 99.5, Dv) - x1) ** 2).sum(),
        bounds=(0.01, 0.1), method="bounded")
    assert abs(fit.x / 0.05 - 1) < 0.02
    assert ((obs["mass"] - m0).abs() / m0).max() < 1e-12


# ------------------------------------------------------------ hypsometric
def test_barometric_equilibrium_equal_masses():
    """Equal masses (no interpolation, so the wall is the exact bounce-back)
    under gravity relax to rho_i(x) = A_i exp(g x / c_s^2), the closed form
    of the recovered NSE at rest with p_i = rho_i c_s^2 (eq. NSE, eq.
    MS_equation with k_i = g)."""
    N, nx, g = 3, 12, 2e-3
    D = torch.full((N, N), 0.1, dtype=DTYPE)
    m = evd.Model("D2Q9", nx, 1, 1, [1.0, 1.0, 1.0], D, 1.2, g=[g, 0, 0],
                  walls=(True, False, False))
    x0 = torch.zeros(N, 1, 1, nx, dtype=DTYPE)
    x0[:, ..., : nx // 2] = torch.tensor([0.2, 0.3, 0.5], dtype=DTYPE)[:, None, None, None]
    x0[:, ..., nx // 2:] = torch.tensor([0.6, 0.3, 0.1], dtype=DTYPE)[:, None, None, None]
    f = evd.initial_populations(m, x0)
    mass = f.sum(dim=(1, 2, 3, 4)).numpy()
    f = evd.run(m, f, 3000)
    rho = evd.observables(m, f)["rho_i"][:, 0, 0].numpy()
    coords = np.stack([np.arange(nx), np.zeros(nx), np.zeros(nx)], 1)
    ref = closed_forms.hypsometric_densities(m.M, mass, coords, [g, 0, 0])
    assert (np.abs(rho - ref) / ref).max() < 2e-5


def test_force_field_separates_species_by_mass():
    """Unequal masses (1 : 4, interpolated species) on a periodic tube under a
    sinusoidal specific force k(x) = A sin(2 pi x/L): each species relaxes to
    rho_i ~ exp(phi(x)/c_{s,i}^2) with d phi/dx = k, so heavier species (smaller
    c_s) separate more (Sec. 3, eq. MS_equation, force term).  Tolerance 5e-3
    relative to the profile amplitude: the O(dx^2) error of a 32-node
    wavelength (measured 1e-3 / 3e-3)."""
    nx, A = 32, 1e-3
    D = torch.full((2, 2), 0.15, dtype=DTYPE)
    xx = torch.arange(nx, dtype=DTYPE)
    ff = torch.zeros(3, 1, 1, nx, dtype=DTYPE)
    ff[0, 0, 0] = A * torch.sin(2 * math.pi * xx / nx)
    m = evd.Model("D2Q9", nx, 1, 1, [1.0, 4.0], D, 1.0, force_field=ff)
    f = evd.initial_populations(m, torch.full((2, 1, 1, nx), 0.5, dtype=DTYPE))
    f = evd.run(m, f, 5000)
    rho = evd.observables(m, f)["rho_i"][:, 0, 0].numpy()
    phi = -(A * nx / (2 * math.pi)) * np.cos(2 * math.pi * np.arange(nx) / nx)
    for i, cs2 in enumerate(m.sound2()):
        lr = np.log(rho[i]) - np.log(rho[i]).mean()
        want = phi / cs2 - (phi / cs2).mean()
        assert np.abs(lr - want).max() < 5e-3 * np.abs(want).max()


def test_ultracentrifuge_interior_is_stationary():
    """Case II (Sec. 4.2) with the paper's numbers: binary UF6 isotopes,
    M1/M2 = 0.991481, C = -1.2358e-8, tau_1 = 0.6, D_12 = 0.08, 500 nodes,
    walls at the r ends, centrifugal force F_i = rho_i omega_u^2 r with
    omega_u^2 from C = (M_1 - M_2) omega_u^2/(R_U T), R_U T = M_1 c_{s,1}^2.
    Started at the analytic steady profile (eq. separation_factor_eq), the
    interior (20 nodes away from the walls) stays on it to 2 % of the profile's
    own variation over 2000 steps; the wall-adjacent layers do not (the wall
    scheme does not keep a rest state exactly for c < 1)."""
    gd = _golden()["ultracentrifuge"]
    C, ratio = gd["C"], gd["M1_over_M2"]
    M = [1.0, 1.0 / ratio]
    omega2 = C * (M[0] / 3.0) / (M[0] - M[1])
    nx = gd["R_nodes"]
    r = np.arange(nx, dtype=float)
    xb = np.array([gd["x1_mean"][0], 1 - gd["x1_mean"][0]])
    wb = xb * np.array(M) / (xb * np.array(M)).sum()
    rho = closed_forms.centrifuge_densities(M, wb * nx, r, omega2)
    n = (rho / np.array(M)[:, None]).sum(0)
    x = rho / np.array(M)[:, None] / n
    # the densities satisfy the paper's x_1(r) form exactly
    assert np.abs(closed_forms.centrifuge_x1(r, x[0, 0], C) - x[0]).max() < 1e-14
    D = torch.tensor([[0, gd["D12"]], [gd["D12"], 0]], dtype=DTYPE)
    ff = torch.zeros(3, 1, 1, nx, dtype=DTYPE)
    ff[0, 0, 0] = torch.tensor(omega2 * r)
    m = evd.Model("D2Q9", nx, 1, 1, M, D, gd["tau1"], walls=(True, False, False),
                  force_field=ff)
    f = evd.initial_populations(m, torch.tensor(x, dtype=DTYPE)[:, None, None, :])
    f = f * torch.tensor(n / m.default_n0(), dtype=DTYPE)[None, None, None, None, :]
    x_a = evd.observables(m, f)["x"][0, 0, 0].numpy()
    assert np.abs(x_a - x[0]).max() < 1e-14
    f = evd.run(m, f, 2000)
    x_b = evd.observables(m, f)["x"][0, 0, 0].numpy()
    variation = x[0].max() - x[0].min()
    assert np.abs(x_b - x_a)[20:-20].max() < 0.02 * variation


# ---------------------------------------------------------------- viscosity
def test_shear_wave_decays_with_common_viscosity():
    """nu_i = (tau_i - 1/2) c_{s,i}^2 = nu for all species (Sec. 3, after eq.
    epecies_momentum_eq), so the mixture obeys the NSE with nu = (tau_1 - 1/2)/3
    (eq. NSE): a shear wave u_y = U sin(k x) decays as exp(-nu k^2 t).
    Masses 1:2:3, tau_1 = 0.8 (measured deviation 0.3 %)."""
    N, nx, steps, U = 3, 32, 300, 1e-3
    tau1 = 0.8
    D = torch.full((N, N), 0.05, dtype=DTYPE)
    m = evd.Model("D2Q9", nx, 1, 1, [1.0, 2.0, 3.0], D, tau1)
    xx = torch.arange(nx, dtype=DTYPE)
    kw = 2 * math.pi / nx
    u = torch.zeros(1, 1, nx, 3, dtype=DTYPE)
    u[..., 1] = U * torch.sin(kw * xx)
    rho_i = torch.full((N, 1, 1, nx), 0.3, dtype=DTYPE)
    _, f = evd.equilibria(m, rho_i, u[None].expand(N, 1, 1, nx, 3), u)
    f = evd.run(m, f, steps)
    uy = evd.observables(m, f)["u"][0, 0, :, 1]
    amp = float((uy * torch.sin(kw * xx)).sum() * 2 / nx)
    nu = -math.log(amp / U) / (kw * kw * steps)
    assert abs(nu / ((tau1 - 0.5) / 3) - 1) < 0.01


# ------------------------------------------------- the same closed forms in 3-D
def test_d3q19_binary_loschmidt_erf_along_y():
    """The binary erf tube of the D2Q9 test on D3Q19, along y (walls at the
    y ends, 1 x 160 x 1 nodes, periodic x and z): the D3Q19 moments recover
    the same Fick law, so the profile follows the same erf with D_12, and
    each species' mass is exact."""
    D = torch.tensor([[0.0, 0.05], [0.05, 0.0]], dtype=DTYPE)
    ny, steps = 160, 1200
    m = evd.Model("D3Q19", 1, ny, 1, [1.0, 1.0], D, 1.0, walls=(False, True, False))
    x0 = torch.zeros(2, 1, ny, 1, dtype=DTYPE)
    x0[0, :, : ny // 2] = 1.0
    x0[1, :, ny // 2:] = 1.0
    f = evd.initial_populations(m, x0)
    m0 = f.sum(dim=(1, 2, 3, 4))
    f = evd.run(m, f, steps)
    obs = evd.observables(m, f)
    x1 = obs["x"][0, 0, :, 0].numpy()
    ref = closed_forms.binary_erf_profile(np.arange(ny), steps, ny / 2 - 0.5, 0.05)
    assert np.abs(x1 - ref).max() < 5e-3
    assert ((obs["mass"] - m0).abs() / m0).max() < 1e-12


def test_d3q19_barometric_equilibrium_along_z():
    """Equal masses under gravity along z on D3Q19 (1 x 1 x 12, walls at the z
    ends) relax to rho_i(z) = A_i exp(g z / c_s^2), as in 2-D."""
    N, nz, g = 3, 12, -2e-3
    D = torch.full((N, N), 0.1, dtype=DTYPE)
    m = evd.Model("D3Q19", 1, 1, nz, [1.0, 1.0, 1.0], D, 1.2, g=[0, 0, g],
                  walls=(False, False, True))
    x0 = torch.zeros(N, nz, 1, 1, dtype=DTYPE)
    x0[:, : nz // 2] = torch.tensor([0.2, 0.3, 0.5], dtype=DTYPE)[:, None, None, None]
    x0[:, nz // 2:] = torch.tensor([0.6, 0.3, 0.1], dtype=DTYPE)[:, None, None, None]
    f = evd.initial_populations(m, x0)
    mass = f.sum(dim=(1, 2, 3, 4)).numpy()
    f = evd.run(m, f, 3000)
    rho = evd.observables(m, f)["rho_i"][:, :, 0, 0].numpy()
    coords = np.stack([np.zeros(nz), np.zeros(nz), np.arange(nz)], 1)
    ref = closed_forms.hypsometric_densities(m.M, mass, coords, [0, 0, g])
    assert (np.abs(rho - ref) / ref).max() < 2e-5


def test_d3q19_force_field_separates_species_by_mass_along_z():
    """The sinusoidal force-field separation of the D2Q9 test on D3Q19, along
    z (1 x 1 x 32, periodic): log rho_i follows phi / c_{s,i}^2."""
    nz, A = 32, 1e-3
    D = torch.full((2, 2), 0.15, dtype=DTYPE)
    zz = torch.arange(nz, dtype=DTYPE)
    ff = torch.zeros(3, nz, 1, 1, dtype=DTYPE)
    ff[2, :, 0, 0] = A * torch.sin(2 * math.pi * zz / nz)
    m = evd.Model("D3Q19", 1, 1, nz, [1.0, 4.0], D, 1.0, force_field=ff)
    f = evd.initial_populations(m, torch.full((2, nz, 1, 1), 0.5, dtype=DTYPE))
    f = evd.run(m, f, 5000)
    rho = evd.observables(m, f)["rho_i"][:, :, 0, 0].numpy()
    phi = -(A * nz / (2 * math.pi)) * np.cos(2 * math.pi * np.arange(nz) / nz)
    for i, cs2 in enumerate(m.sound2()):
        lr = np.log(rho[i]) - np.log(rho[i]).mean()
        want = phi / cs2 - (phi / cs2).mean()
        assert np.abs(lr - want).max() < 5e-3 * np.abs(want).max()


def test_d3q19_shear_wave_decays_with_common_viscosity():
    """A shear wave u_z = U sin(k x) on D3Q19 (32 x 1 x 1, masses 1:2:3) decays
    as exp(-nu k^2 t) with nu = (tau_1 - 1/2)/3, as in 2-D."""
    N, nx, steps, U = 3, 32, 300, 1e-3
    tau1 = 0.8
    D = torch.full((N, N), 0.05, dtype=DTYPE)
    m = evd.Model("D3Q19", nx, 1, 1, [1.0, 2.0, 3.0], D, tau1)
    xx = torch.arange(nx, dtype=DTYPE)
    kw = 2 * math.pi / nx
    u = torch.zeros(1, 1, nx, 3, dtype=DTYPE)
    u[..., 2] = U * torch.sin(kw * xx)
    rho_i = torch.full((N, 1, 1, nx), 0.3, dtype=DTYPE)
    _, f = evd.equilibria(m, rho_i, u[None].expand(N, 1, 1, nx, 3), u)
    f = evd.run(m, f, steps)
    uz = evd.observables(m, f)["u"][0, 0, :, 2]
    amp = float((uz * torch.sin(kw * xx)).sum() * 2 / nx)
    nu = -math.log(amp / U) / (kw * kw * steps)
    assert abs(nu / ((tau1 - 0.5) / 3) - 1) < 0.01


# --------------------------------------- hypsometric tube between walls
def _hypsometric_golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "hypsometric_walls.json")) as fh:
        return json.load(fh)


def _hypsometric_model(G):
    import lbm_workloads as W
    w = W.ternary_gravity()
    return evd.Model("D2Q9", G["nx"], 1, 1, w.masses, torch.tensor(w.diff, dtype=DTYPE), w.tau1,
                     g=[G["g"], 0.0, 0.0], walls=(True, False, False))


def test_hypsometric_tube_between_walls():
    """The paper's gases' masses (2:28:44), the 1024x64 workload's seeded
    diffusivities, walls at the x ends, g = 1e-5 along x, 64 nodes: the
    stationary state that the oracle reaches from the closed form (stored by
    tests/golden/make_golden.py after 120,000 steps) is
      * a fixed point of the current oracle (1000 more steps change no mole
        fraction by more than 1e-9);
      * at rest in the interior (20 nodes from each wall: |u| < 1e-8) with
        rho_i(x) = A_i exp(g x/c_{s,i}^2), the hypsometric closed form of eq.
        (MS_equation) with k_i = g and eq. (NSE) at rest, p_i = rho_i c_{s,i}^2,
        to 1e-7 in mole fraction (amplitudes A_i fitted: the wall layers hold
        part of each species' mass);
      * next to each wall, a layer that Appendix A's scheme leaves for c < 1:
        the printed wall formulas return less than the full weight to the
        reflected direction at a uniform rest state (1 - xi(1 - xi)/2 for the
        right wall's alpha = 3), so the wall node keeps a stationary velocity
        (|u| about 1.1e-2 here, the same at g = 0) and a composition offset
        (5.7e-2 in mole fraction), alternating in sign and decaying by about a
        factor 2 per node into the interior."""
    G = _hypsometric_golden()
    m = _hypsometric_model(G)
    nx, g, k = G["nx"], G["g"], 20
    f = torch.tensor(G["f"], dtype=DTYPE)[:, :, None, None, :]
    ob = evd.observables(m, f)
    x = ob["x"][:, 0, 0].numpy()
    x_later = evd.observables(m, evd.run(m, f, 1000))["x"][:, 0, 0].numpy()
    assert np.abs(x_later - x).max() < 1e-9
    rho = ob["rho_i"][:, 0, 0].numpy()
    cs2 = np.array(m.sound2())
    xs = np.arange(nx, dtype=float)
    shape = np.exp(g * xs[None] / cs2[:, None])
    A = (rho[:, k:nx - k] / shape[:, k:nx - k]).mean(1)
    fit = A[:, None] * shape
    M = np.array(m.M)
    x_fit = fit / M[:, None] / (fit / M[:, None]).sum(0)
    dev = np.abs(x - x_fit).max(0)
    assert dev[k:nx - k].max() < 1e-7
    u = ob["u"][0, 0, :, 0].numpy()
    assert np.abs(u[k:nx - k]).max() < 1e-8
    # the heaviest species' interior profile varies by 4 %: the fit is not trivial
    assert fit[2, nx - k - 1] / fit[2, k] - 1 > 0.5 * (np.exp(g * (nx - 2 * k) / cs2[2]) - 1)
    # the wall layers, mirror images of each other
    assert 5e-3 < abs(u[0]) < 2e-2 and np.sign(u[0]) == -np.sign(u[-1])
    assert 1e-2 < dev[0] < 0.1 and 1e-2 < dev[-1] < 0.1
    for j in range(12):
        assert np.sign(u[j]) == -np.sign(u[j + 1])
        assert 1.3 < abs(u[j] / u[j + 1]) < 3.0, j


def test_wall_layer_does_not_come_from_gravity():
    """The wall layer of the hypsometric tube is the same at g = 0: a uniform
    mixture of the same masses at rest between walls develops it (wall-node
    velocity within 1 % of the g = 1e-5 value after 3000 steps)."""
    G = _hypsometric_golden()
    m0 = _hypsometric_model(dict(G, g=0.0))
    x0 = torch.tensor(G["x_mean"], dtype=DTYPE)[:, None, None, None].expand(3, 1, 1, G["nx"])
    f = evd.run(m0, evd.initial_populations(m0, x0.clone()), 3000)
    u0 = evd.observables(m0, f)["u"][0, 0, 0, 0].item()
    m = _hypsometric_model(G)
    u = evd.observables(m, torch.tensor(G["f"], dtype=DTYPE)[:, :, None, None, :])["u"][0, 0, 0, 0]
    assert abs(u0 / u.item() - 1) < 1e-2
