"""Full-size GPU parity of the optional physics on the 16384 x 1024 ternary
tube, the lattice `bench.py` times them on: the diffusion-driven forcing
term (forcing 1), the whole corrected forcing (forcing 2) and a force field
k(x) in place of g, each in both execution variants; and the equilibrium
comparison boundary in place of the Appendix A walls.

The lattice is too large for the FP64 oracle to run whole, so sampled nodes
are checked after a few steps against the oracle run on a crop around each
sample: after s steps a node's post-collision populations depend on its
neighbourhood of radius s (forcing 0 and 1) or 2 s + 1 (forcing 2, whose
density gradients reach one node further each step), so a crop of radius
2 s + 2 is exact at its centre whatever happens at its artificial faces;
crops that reach a real wall keep it.  Bar: populations within 2e-6 of the
oracle relative to the largest population (FP32 rounding of a few steps)."""
import dataclasses

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE

pytestmark = pytest.mark.gpu

F_RTOL = 2e-6
STEPS = 2
WTS = torch.tensor([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=DTYPE)


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _tube():
    return W.ternary_gravity(16384, 1024, 500, name="ternary_gravity_16384x1024")


def _field(w):
    """A centrifuge-like ramp along x plus a y modulation, float32 [2, 1, ny, nx]."""
    xx = np.arange(w.nx)[None, :]
    yy = np.arange(w.ny)[:, None]
    acc = np.zeros((2, 1, w.ny, w.nx))
    acc[0, 0] = 2e-6 * (xx / w.nx - 0.5) + 5e-7 * np.sin(2 * np.pi * yy / w.ny)
    acc[1, 0] = 1e-6 * np.cos(2 * np.pi * xx / 97.0) + 0 * yy
    return acc.astype(np.float32)


def _samples(w):
    half = w.nx // 2
    pts = [(0, 0), (1, 511), (2, w.ny - 1), (w.nx - 1, 7), (w.nx - 2, w.ny - 1), (w.nx - 3, 0),
           (half - 1, 0), (half, w.ny - 1), (half + 1, 300), (half - 2, 77), (half + 3, 1023),
           (half, 512)]
    rng = np.random.default_rng(9)
    while len(pts) < 20:
        pts.append((int(rng.integers(w.nx)), int(rng.integers(w.ny))))
    return pts


def _crop(w, x0, acc, c, R):
    x, y = c
    xa, xb = max(0, x - R), min(w.nx, x + R + 1)
    ys = [(y + k) % w.ny for k in range(-R, R + 1)]
    sub = x0[:, :, ys][:, :, :, xa:xb]
    a = None if acc is None else acc[:, :, ys][:, :, :, xa:xb]
    return sub, a, (R, x - xa)


CASES = [("diff", False), ("full", False), ("standard", True)]
SHAPES = [(64, 1, 32, 0, 1), (64, 1, 32, 0, 0)]


@pytest.mark.parametrize("shape", SHAPES, ids=["split", "joint"])
@pytest.mark.parametrize("forcing,field", CASES, ids=["forcing1", "forcing2", "force_field"])
def test_full_tube_sampled_nodes_match_oracle_crops(forcing, field, shape):
    w = dataclasses.replace(_tube(), forcing=forcing)
    if field:
        w = dataclasses.replace(w, g=[0.0, 0.0, 0.0])
    _announce(f"{w.name} forcing {forcing} field {field} shape {shape}")
    lbm = _lbm()
    x0 = w.x0()
    acc = _field(w) if field else None
    sim = lbm.LbmMc(lbm.params_from_workload(w), x0,
                    accel=None if acc is None else torch.tensor(acc, device="cuda"))
    sim.set_tuning(*shape)
    sim.step(STEPS)
    raw = sim.raw("cur")
    pts = _samples(w)
    got = torch.stack([raw[:, :, 0, y, x] for (x, y) in pts]).double().cpu()   # [P, N, Q]
    sim.sync()
    sim.close()
    R = 2 * STEPS + 2
    for k, c in enumerate(pts):
        sub, a, (cy, cx) = _crop(w, x0, acc, c, R)
        ff = None
        if a is not None:
            ff = torch.zeros((3,) + a.shape[1:], dtype=DTYPE)
            ff[:2] = torch.tensor(a, dtype=DTYPE)
        m = evd.Model("D2Q9", sub.shape[3], sub.shape[2], 1, w.masses,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g, walls=(True, False, False),
                      force_field=ff, forcing=forcing)
        f = evd.run(m, evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE)), STEPS)
        ref = evd.collide(m, f)[:, :, 0, cy, cx]                      # [N, Q]
        s = got[k]
        pop = (WTS / WTS[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, (c, err)


def test_full_tube_equilibrium_boundary_sampled_nodes_match_oracle_crops():
    """The equilibrium comparison boundary on the same tube, at the shape
    `bench.py` times it with (one thread per column, 256-column tiles of 32
    layers), against the oracle's evd.stream_equilibrium_walls on crops (the
    solid nodes' values depend on the fluid node next to them, so influence
    still spreads one node per step and the crops of radius 2 s + 2 are exact
    at their centres)."""
    w = dataclasses.replace(_tube(), wall_kind="equilibrium")
    _announce(f"{w.name} equilibrium boundary")
    lbm = _lbm()
    x0 = w.x0()
    sim = lbm.LbmMc(lbm.params_from_workload(w), x0)
    sim.set_tuning(256, 1, 32, 0, 0)
    sim.step(STEPS)
    raw = sim.raw("cur")
    pts = _samples(w)
    got = torch.stack([raw[:, :, 0, y, x] for (x, y) in pts]).double().cpu()   # [P, N, Q]
    sim.sync()
    sim.close()
    R = 2 * STEPS + 2
    for k, c in enumerate(pts):
        sub, _, (cy, cx) = _crop(w, x0, None, c, R)
        m = evd.Model("D2Q9", sub.shape[3], sub.shape[2], 1, w.masses,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g, walls=(True, False, False))
        f = evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE))
        for _ in range(STEPS):
            f = evd.stream_equilibrium_walls(m, evd.collide(m, f))
        ref = evd.collide(m, f)[:, :, 0, cy, cx]                      # [N, Q]
        s = got[k]
        pop = (WTS / WTS[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, (c, err)
