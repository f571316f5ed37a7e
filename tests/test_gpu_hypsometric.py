"""GPU run of the hypsometric tube between walls: the masses of the paper's
gases (2:28:44), the 1024x64 workload's seeded diffusivities, walls at the x
ends, g = 1e-5 along x, 64 nodes (16 identical rows).  The GPU starts from
the oracle's stationary state (tests/golden/hypsometric_walls.json, itself
pinned against the hypsometric closed form and stationarity on the CPU) and
runs 20,000 steps: the FP32 state must stay within the parity bar (1e-5 in
mole fraction) of the oracle's fixed point everywhere, wall layers included,
drift less than 1e-6 in the interior, and keep each species' mass to 1e-6."""
import json
import os

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE
from tests._decode import encode

pytestmark = pytest.mark.gpu

X_TOL = 1e-5


def test_hypsometric_state_is_stationary_on_the_gpu():
    from paper_2504_07059_amd import lbm
    with open(os.path.join(os.path.dirname(__file__), "golden", "hypsometric_walls.json")) as fh:
        G = json.load(fh)
    print("\n[gpu case] hypsometric tube 64x16, 20000 steps", flush=True)
    nx, ny, g = G["nx"], 16, G["g"]
    base = W.ternary_gravity()
    m = evd.Model("D2Q9", nx, 1, 1, base.masses, torch.tensor(base.diff, dtype=DTYPE),
                  base.tau1, g=[g, 0.0, 0.0], walls=(True, False, False))
    f = torch.tensor(G["f"], dtype=DTYPE)[:, :, None, None, :]          # f(t), post-stream
    x_ref = evd.observables(m, f)["x"][:, 0, 0].numpy()                  # [N, nx]
    s = encode(evd.collide(m, f)).float()                               # stored f~(t)
    w = W.Workload("hypsometric_64x16", "D2Q9", nx, ny, 1, base.masses, base.diff,
                   base.tau1, [g, 0.0, 0.0], [True, False, False], 20000, "given",
                   x0_args={"x": np.broadcast_to(x_ref[:, None, None, :], (3, 1, ny, nx))})
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    state = torch.zeros_like(sim.fa)
    sim.view(state).copy_(s.expand(-1, -1, 1, ny, -1).to(state.device))
    # at the fixed point f~(t-1) = f~(t): the same state serves as both
    sim.restore(state, state, 1)
    out = sim.moments()
    m0 = out["mass"][0].copy()
    x0 = sim.field(out, "x").double().cpu().numpy()[:, 0]               # [N, ny, nx]
    assert np.abs(x0 - x_ref[:, None, :]).max() < 1e-6
    sim.step(20000)
    out = sim.moments()
    sim.sync()
    x1 = sim.field(out, "x").double().cpu().numpy()[:, 0]
    drift = np.abs(out["mass"][0] / m0 - 1).max()
    sim.close()
    err = np.abs(x1 - x_ref[:, None, :]).max()
    k = 20
    interior_drift = np.abs(x1 - x0)[:, :, k:nx - k].max()
    print(f"max |dx| vs oracle fixed point {err:.2e}, interior drift {interior_drift:.2e}, "
          f"mass drift {drift:.2e}")
    assert err < X_TOL, err
    assert interior_drift < 1e-6, interior_drift
    assert drift < 1e-6, drift
