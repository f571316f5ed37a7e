"""GPU tests of the three-dimensional layer workload (D3Q19, 4 species,
masses 1:2:3:4, walls at z = 0 and nz-1, periodic x and y, g = -1e-6 along z,
dense layer over a light carrier with a seeded 1 % perturbation).

The 256x128x128 lattice is too large for the FP64 oracle to run whole, so
full size is checked two ways:
  * sampled nodes after a few steps against the oracle run on a crop around
    each sample (after s steps a node depends only on its radius-s
    neighbourhood, so a crop of radius s+1 with any boundary treatment at its
    artificial faces is exact at the centre; crops that reach a real wall keep
    it);
  * properties over the full 5000 steps (per-species FP64 mass, bounds).
A 16x8x32 sub-problem of the same workload is compared whole against stored
oracle results at 500 and 5000 steps."""
import json
import os

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
X_TOL = 1e-5
MASS_TOL = 1e-6
F_RTOL = 2e-6


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def test_layer_small_matches_stored_oracle():
    """16x8x32 sub-problem, whole field against the oracle at 500 and 5000
    steps; FP64 mass against the oracle's."""
    with open(os.path.join(GOLDEN, "layer_mixing_3d_small.json")) as fh:
        G = json.load(fh)["checkpoints"]
    w = W.layer_mixing_3d(16, 8, 32, steps=5000)
    _announce(w.name)
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(block_x=32, block_y=2, rows=8)     # several tiles along every axis
    m0 = sim.moments(fields=False)["mass"][0].copy()
    t = 0
    for cp in (500, 5000):
        sim.step(cp - t)
        t = cp
        out = sim.moments()
        sim.sync()
        x = sim.field(out, "x").double().cpu().numpy()
        dx = np.abs(x - np.asarray(G[str(cp)]["x"])).max()
        assert dx < X_TOL, (cp, dx)
        assert np.abs(out["mass"][0] / np.asarray(G[str(cp)]["mass"]) - 1).max() < MASS_TOL
        assert np.abs(out["mass"][0] / m0 - 1).max() < MASS_TOL
    sim.close()


def _samples(w, rng, count):
    pts = [(0, 0, 0), (w.nx - 1, w.ny - 1, w.nz - 1), (5, w.ny - 1, 1), (w.nx - 1, 3, w.nz - 2),
           (17, 40, 2), (100, 64, w.nz - 3), (128, 1, 95), (31, 127, 96), (200, 77, 97)]
    while len(pts) < count:
        pts.append((int(rng.integers(w.nx)), int(rng.integers(w.ny)), int(rng.integers(w.nz))))
    return pts


def _crop(w, x0, c, R):
    """x0 crop [N, cz, cy, cx] of radius R around c (periodic wrap in x, y;
    clipped at the z walls), and the centre's index inside it."""
    x, y, z = c
    xs = [(x + k) % w.nx for k in range(-R, R + 1)]
    ys = [(y + k) % w.ny for k in range(-R, R + 1)]
    z0, z1 = max(0, z - R), min(w.nz, z + R + 1)
    sub = x0[:, z0:z1][:, :, ys][:, :, :, xs]
    return sub, (R, R, z - z0)


@pytest.mark.parametrize("steps", [1, 3])
def test_layer_full_size_sampled_nodes_match_oracle_crops(steps):
    """256x128x128 at the library's default execution shape: post-collision
    populations of 24 sampled nodes (corners, walls, the layer interface,
    periodic seams, random) after `steps` steps against the oracle on crops."""
    w = W.layer_mixing_3d()
    _announce(f"{w.name} sampled nodes, {steps} steps")
    lbm = _lbm()
    x0 = w.x0()
    sim = lbm.LbmMc(lbm.params_from_workload(w), x0)
    sim.step(steps)
    raw = sim.raw("cur")
    pts = _samples(w, np.random.default_rng(5), 24)
    got = torch.stack([raw[:, :, z, y, x] for (x, y, z) in pts]).double().cpu()
    sim.sync()
    sim.close()
    Q = 19
    wts = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=DTYPE)
    R = steps + 1
    for k, c in enumerate(pts):
        sub, (cx, cy, cz) = _crop(w, x0, c, R)
        m = evd.Model("D3Q19", sub.shape[3], sub.shape[2], sub.shape[1], w.masses,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g,
                      walls=(False, False, True))
        f = evd.run(m, evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE)), steps)
        ref = evd.collide(m, f)[:, :, cz, cy, cx]                  # [N, Q]
        s = got[k]
        pop = (wts / wts[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, (c, err)


def test_layer_full_size_5000_steps_properties():
    """The full workload (256x128x128, 5000 steps) at the default execution
    shape: per-species FP64 mass conserved to 1e-6, mole fractions in [0, 1]
    and summing to 1, and the dense species still above the carrier's mean
    in the top layer (gravity has not been reversed)."""
    w = W.layer_mixing_3d()
    _announce(f"{w.name} 5000 steps")
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(5000)
    out = sim.moments()
    sim.sync()
    assert np.abs(out["mass"][0] / m0 - 1).max() < MASS_TOL
    x = sim.field(out, "x")                                   # [N, nz, ny, nx]
    assert float(x.min()) >= 0.0 and float(x.max()) <= 1.0
    assert float((x.sum(0) - 1).abs().max()) < 1e-5
    prof = x.double().mean(dim=(2, 3)).cpu().numpy()          # [N, nz]
    assert prof[3, -1] > prof[3, 0]
    sim.close()


def test_layer_full_size_tile_seams_after_16_steps():
    """256x128x128 at the library's default execution shape (64-column rows,
    16-layer tiles), 16 steps: the post-collision populations and mole
    fractions of ten nodes on the tile seams (x = 63|64, 127|128, 191|192,
    255|0; z = 15|16, 31|32, 95|96, 111|112; every y row is a seam) and on both
    z walls, against the stored oracle crops of radius 17
    (tests/golden/layer_crops_16.json)."""
    with open(os.path.join(GOLDEN, "layer_crops_16.json")) as fh:
        G = json.load(fh)
    w = W.layer_mixing_3d()
    _announce(f"{w.name} tile seams, {G['steps']} steps")
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    assert sim.get_tuning()[:3] == (64, 1, 16)
    sim.step(G["steps"])
    raw = sim.raw("cur")
    out = sim.moments()
    x = sim.field(out, "x")
    sim.sync()
    wts = torch.tensor([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12, dtype=DTYPE)
    for rec in G["nodes"]:
        cx, cy, cz = rec["node"]
        s = raw[:, :, cz, cy, cx].double().cpu()
        pop = (wts / wts[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        ref = torch.tensor(rec["f_post"], dtype=DTYPE)
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, (rec["node"], err)
        dx = (x[:, cz, cy, cx].double().cpu() - torch.tensor(rec["x"], dtype=DTYPE)).abs().max()
        assert dx.item() < X_TOL, (rec["node"], dx.item())
    sim.close()


@pytest.mark.skipif(not os.path.exists(os.path.join(GOLDEN, "layer_mixing_3d_64x32x32.npz")),
                    reason="stored oracle field not generated (tests/golden/make_golden.py "
                           "layer_mixing_3d_64)")
def test_layer_64x32x32_5000_steps_whole_field():
    """A 64x32x32 sub-problem of the layer workload (interface at z = 24),
    whole mole-fraction field against the stored oracle at 100, 1000 and
    5000 steps (tests/golden/layer_mixing_3d_64x32x32.npz), at the library's
    default shape and at a shape with several tiles along every axis; FP64
    mass against the oracle's."""
    G = np.load(os.path.join(GOLDEN, "layer_mixing_3d_64x32x32.npz"))
    w = W.layer_mixing_3d(64, 32, 32, steps=5000)
    lbm = _lbm()
    for tuning in (None, dict(block_x=32, block_y=2, rows=8)):
        _announce(f"{w.name} whole field, tuning {tuning}")
        sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        if tuning:
            sim.set_tuning(**tuning)
        t = 0
        for cp in (100, 1000, 5000):
            sim.step(cp - t)
            t = cp
            out = sim.moments()
            sim.sync()
            x = sim.field(out, "x").double().cpu().numpy()
            dx = np.abs(x - G[f"x_{cp}"].astype(np.float64)).max()
            assert dx < X_TOL, (tuning, cp, dx)
            assert np.abs(out["mass"][0] / G[f"mass_{cp}"] - 1).max() < MASS_TOL
        sim.close()
