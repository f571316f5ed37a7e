"""GPU tests of boxes with walls on several axes (edges and corners; reading
R11 of the oracle: what a wall node's populations would stream beyond the
walls returns to the node, split by the set of walls crossed) against the
oracle, through the C ABI, in both execution variants; plus species mass over
a long run.  Bars as for single walls: mole fractions within 1e-5,
populations within 2e-6 of the largest, mass drift below 1e-6."""
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


def _wk(name, lattice, shape, masses, walls, g, steps, seed=11, diff=None, forcing="standard"):
    N = len(masses)
    if diff is None:
        rng = np.random.default_rng(seed)
        d = rng.uniform(0.06, 0.1, size=(N, N))
        diff = ((d + d.T) / 2).tolist()
    return W.Workload(name, lattice, *shape, masses, diff, 1.0, list(g), list(walls), steps,
                      "random", seed=seed, forcing=forcing)


TERNARY = W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3)
CASES = [
    _wk("d2q9_n3_xy_box", "D2Q9", (130, 37, 1), [2.0, 28.0, 44.0], (True, True, False),
        (1e-5, -2e-5, 0), 24, diff=TERNARY),
    _wk("d2q9_n2_xy_box_small", "D2Q9", (5, 3, 1), [1.0, 3.0], (True, True, False),
        (2e-5, 1e-5, 0), 30),
    _wk("d3q19_n4_xyz_box", "D3Q19", (40, 21, 19), [1.0, 2.0, 3.0, 4.0], (True, True, True),
        (1e-5, 0, -1e-5), 16),
    _wk("d3q19_n3_xz_box", "D3Q19", (23, 18, 17), [1.0, 2.0, 6.0], (True, False, True),
        (2e-5, 0, 1e-5), 16),
    _wk("d3q19_n2_yz_box", "D3Q19", (20, 26, 11), [1.0, 5.0], (False, True, True),
        (0, 1e-5, -1e-5), 16),
    _wk("d2q9_n3_xy_box_full", "D2Q9", (130, 37, 1), [2.0, 28.0, 44.0], (True, True, False),
        (1e-5, -2e-5, 0), 24, diff=TERNARY, forcing="full"),
    # the smallest boxes the full corrected forcing takes (3 nodes per wall axis)
    _wk("d2q9_n3_3x3_box_full", "D2Q9", (3, 3, 1), [1.0, 2.0, 5.0], (True, True, False),
        (1e-5, -1e-5, 0), 24, forcing="full"),
    _wk("d3q19_n2_3x3x3_box_full", "D3Q19", (3, 3, 3), [1.0, 4.0], (True, True, True),
        (1e-5, 1e-5, -1e-5), 16, forcing="full"),
]


def _shape(w, variant):
    if variant:
        return (64, 1, 4, 0, 1) if w.lattice == "D2Q9" else (16, 4, 3, 0, 1)
    return (64, 1, 4, 0, 0) if w.lattice == "D2Q9" else (16, 4, 3, 0, 0)


@pytest.mark.parametrize("variant", [0, 1], ids=["joint", "split"])
@pytest.mark.parametrize("w", CASES, ids=[w.name for w in CASES])
def test_boxes_match_oracle(w, variant):
    _announce(f"box {w.name} variant {variant}")
    lbm = _lbm()
    m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                  w.tau1, g=w.g, walls=w.walls, forcing=w.forcing)
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
    fg = populations(sim).double().cpu()
    df = ((fg - ft).abs().max() / ft.abs().max()).item()
    drift = np.abs(out["mass"][0] / m0 - 1).max()
    dmass = np.abs(out["mass"][0] / ob["mass"].numpy() - 1).max()
    sim.close()
    assert dx < X_TOL, dx
    assert df < F_RTOL, df
    assert drift < MASS_TOL, drift
    assert dmass < MASS_TOL, dmass


def test_closed_box_keeps_species_mass_over_a_long_run():
    """A 3-D box closed on every face, 4 species, gravity, 5000 steps: the
    FP64 mass of every species stays within 1e-6 (the corners return what
    they would lose)."""
    w = CASES[2]
    _announce("closed 3-D box, 5000 steps")
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(5000)
    out = sim.moments()
    sim.sync()
    sim.close()
    assert np.abs(out["mass"][0] / m0 - 1).max() < MASS_TOL
