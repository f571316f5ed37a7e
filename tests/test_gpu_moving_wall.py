"""GPU tests of the moving-wall term (Appendix A's closing remark; rho_i and
w_i of the streamed populations at the wall node) against the oracle, through
the C ABI: small lattices with moving walls on every kind of wall axis, both
execution variants, and with the whole corrected forcing; plane Couette flow
against its closed form.  Bars as for the resting walls: mole fractions within
1e-5, populations within 2e-6 of the largest, mass drift below 1e-6."""
import dataclasses

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE
from tests._decode import populations

pytestmark = pytest.mark.gpu

X_TOL = 1e-5
MASS_TOL = 1e-6
F_RTOL = 2e-6


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _wk(name, lattice, shape, masses, walls, g, uw, steps, seed=11, diff=None, forcing="standard"):
    N = len(masses)
    if diff is None:
        rng = np.random.default_rng(seed)
        d = rng.uniform(0.06, 0.1, size=(N, N))
        diff = ((d + d.T) / 2).tolist()
    return W.Workload(name, lattice, *shape, masses, diff, 1.0, list(g), list(walls), steps,
                      "random", seed=seed, forcing=forcing, wall_velocity=uw)


TERNARY = W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3)
CASES = [
    _wk("d2q9_n3_xwall", "D2Q9", (130, 37, 1), [2.0, 28.0, 44.0], (True, False, False),
        (1e-5, 2e-6, 0), [[0, 0.02, 0], [0, -0.01, 0]], 24, diff=TERNARY),
    _wk("d2q9_n2_ywall", "D2Q9", (70, 40, 1), [1.0, 3.0], (False, True, False), (0, -2e-5, 0),
        [[0.01, 0, 0], [-0.02, 0, 0]], 24),
    _wk("d3q19_n4_zwall", "D3Q19", (40, 21, 19), [1.0, 2.0, 3.0, 4.0], (False, False, True),
        (0, 0, -1e-5), [[0.01, -0.005, 0], [0, 0.02, 0]], 16),
    _wk("d3q19_n3_xwall", "D3Q19", (23, 18, 17), [1.0, 2.0, 6.0], (True, False, False),
        (2e-5, 0, 0), [[0, 0.01, 0.01], [0, 0, -0.02]], 16),
    _wk("d2q9_n3_xwall_full", "D2Q9", (130, 37, 1), [2.0, 28.0, 44.0], (True, False, False),
        (1e-5, 2e-6, 0), [[0, 0.02, 0], [0, -0.01, 0]], 24, diff=TERNARY, forcing="full"),
    # walls two nodes apart: every node next to both moving walls
    _wk("d2q9_n2_two_columns", "D2Q9", (2, 9, 1), [1.0, 3.0], (True, False, False),
        (1e-5, 0, 0), [[0, 0.02, 0], [0, -0.01, 0]], 24),
    _wk("d3q19_n3_two_layers", "D3Q19", (9, 5, 2), [1.0, 2.0, 6.0], (False, False, True),
        (0, 0, -1e-5), [[0.01, 0, 0], [0, -0.02, 0]], 16),
]


def _shape(w, variant):
    if variant:
        return (64, 1, 4, 0, 1) if w.lattice == "D2Q9" else (16, 4, 3, 0, 1)
    return (64, 1, 4, 0, 0) if w.lattice == "D2Q9" else (16, 4, 3, 0, 0)


@pytest.mark.parametrize("variant", [0, 1], ids=["joint", "split"])
@pytest.mark.parametrize("w", CASES, ids=[w.name for w in CASES])
def test_moving_walls_match_oracle(w, variant):
    _announce(f"moving walls {w.name} variant {variant}")
    lbm = _lbm()
    m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                  w.tau1, g=w.g, walls=w.walls, forcing=w.forcing,
                  wall_velocity=torch.tensor(w.wall_velocity, dtype=DTYPE))
    f = evd.run(m, evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE)), w.steps)
    ob = evd.observables(m, f)
    ft = evd.collide(m, f)
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(*_shape(w, variant))
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(w.steps)
    out = sim.moments()
    sim.sync()
    dx = (sim.field(out, "x").double().cpu() - ob["x"]).abs().max().item()
    du = (sim.field(out, "u").double().cpu()
          - ob["u"].permute(3, 0, 1, 2)[:sim.dim]).abs().max().item()
    fg = populations(sim).double().cpu()
    df = ((fg - ft).abs().max() / ft.abs().max()).item()
    drift = np.abs(out["mass"][0] / m0 - 1).max()
    sim.close()
    assert dx < X_TOL, dx
    assert df < F_RTOL, df
    assert du < 1e-6, du
    assert drift < MASS_TOL, drift


@pytest.mark.parametrize("x1", [1.0 - 1e-6, 0.5])
def test_couette_profile(x1):
    """Equal masses, walls on y at rest (bottom) and moving at U along x
    (top), periodic x: the steady mixture velocity is the closed form
    u_x(y) = U sum_i w_i^2 (y + 1/2)/ny (U for the nearly pure species, U/2
    for the 50/50 binary), to 2e-5 U."""
    nx, ny, U, steps = 64, 24, 1e-3, 12000
    _announce(f"couette x1 = {x1}")
    lbm = _lbm()
    p = lbm.make_params("D2Q9", nx, ny, 1, [1.0, 1.0], [[0, 0.1], [0.1, 0]], 1.0,
                        walls=(False, True, False), wall_velocity=[[0, 0, 0], [U, 0, 0]])
    x0 = np.zeros((2, 1, ny, nx))
    x0[0] = x1
    x0[1] = 1.0 - x1
    sim = lbm.LbmMc(p, x0)
    sim.step(steps)
    out = sim.moments()
    sim.sync()
    u = sim.field(out, "u").double().cpu().numpy()        # [2, 1, ny, nx]
    sim.close()
    w = np.array([x1, 1.0 - x1])
    want = U * (w * w).sum() * (np.arange(ny) + 0.5) / ny
    # FP32 state: the velocity is a small difference of O(0.1) populations,
    # so its steady-state rounding is about 1e-8 here (5.8e-9 measured)
    assert np.abs(u[0, 0] - want[:, None]).max() < 2e-5 * U
    assert np.abs(u[1]).max() < 2e-5 * U


def test_adjoint_rejects_moving_walls():
    lbm = _lbm()
    w = CASES[1]
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    s_prev = sim.buffers()[0].clone()
    lam = torch.zeros_like(s_prev)
    grad = torch.zeros(4, dtype=torch.float64, device=s_prev.device)
    from paper_2504_07059_amd._lib import LbmError
    with pytest.raises(LbmError) as e:
        sim.adjoint_step(s_prev, lam, torch.zeros_like(s_prev), grad)
    assert e.value.status == 2 and "moving" in str(e.value)
    sim.close()
