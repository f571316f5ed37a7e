"""The largest lattices the library accepts: each species' Q planes just
under 2 GiB, four species to a buffer of 8.6 GB.  A D2Q9 box of 32768 x 1820
nodes with walls on x and y (edges and corners), and a D3Q19 box of
256 x 128 x 862 nodes closed on all three axes.  The last species' planes
then start beyond 6 GiB in the buffer and their own last planes sit at byte
offsets near 2^31 within the species, where the solid-source markers and the
buffer range checks of the gather are at their limits.  Sampled nodes after
two steps against the oracle on crops (exact at their centres: influence
spreads one node per step), including the four corners and nodes of the last
species; one more row is rejected before any device work.  Bar: populations
within 2e-6 of the largest (FP32 rounding of two steps)."""
import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE

F_RTOL = 2e-6
STEPS = 2
NX, NY = 32768, 1820
NZ3 = 862
MASSES = [1.0, 2.0, 3.0, 4.0]


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _workload(ny=NY):
    rng = np.random.default_rng(21)
    d = rng.uniform(0.06, 0.1, size=(4, 4))
    diff = ((d + d.T) / 2).tolist()
    return W.Workload("max_box", "D2Q9", NX, ny, 1, MASSES, diff, 1.0, [1e-5, -1e-5, 0.0],
                      [True, True, False], STEPS, "random", seed=21)


def test_one_row_more_is_rejected_before_device_work():
    lbm = _lbm()
    w = _workload(NY + 1)
    st, _, msg = lbm.check_problem(lbm.params_from_workload(w), np.full((4, 1, 1, 1), 0.25))
    assert st == 2 and "2 GiB" in msg, msg


@pytest.mark.gpu
@pytest.mark.parametrize("shape", [None, (64, 1, 32, 0, 0)], ids=["default", "joint"])
def test_largest_lattice_sampled_nodes_match_oracle_crops(shape):
    lbm = _lbm()
    w = _workload()
    print(f"\n[gpu case] max-size box {NX}x{NY}, 4 species, shape {shape}", flush=True)
    x0 = w.x0()
    total, _, pitch, _ = lbm.layout(lbm.params_from_workload(w))
    species_bytes = pitch[0] * NY * 9 * 4
    assert species_bytes < 2 ** 31 and species_bytes > 2 ** 31 - 2 ** 26
    assert total * 4 > 4 * (2 ** 31 - 2 ** 26)   # four species of nearly 2 GiB: 8.6 GB
    sim = lbm.LbmMc(lbm.params_from_workload(w), x0)
    if shape:
        sim.set_tuning(*shape)
    sim.step(STEPS)
    raw = sim.raw("cur")
    pts = [(0, 0), (NX - 1, 0), (0, NY - 1), (NX - 1, NY - 1), (1, NY - 2), (NX - 2, 1),
           (NX // 2, 0), (NX // 2, NY - 1), (0, NY // 2), (NX - 1, NY // 2), (12345, 321),
           (NX - 7, NY - 3)]
    got = torch.stack([raw[:, :, 0, y, x] for (x, y) in pts]).double().cpu()   # [P, N, Q]
    out = sim.moments(fields=False)
    sim.sync()
    sim.close()
    assert np.isfinite(out["mass"]).all()
    R = STEPS + 2
    wts = torch.tensor([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=DTYPE)
    for k, (x, y) in enumerate(pts):
        xa, xb = max(0, x - R), min(NX, x + R + 1)
        ya, yb = max(0, y - R), min(NY, y + R + 1)
        sub = x0[:, :, ya:yb, xa:xb]
        m = evd.Model("D2Q9", xb - xa, yb - ya, 1, MASSES, torch.tensor(w.diff, dtype=DTYPE),
                      w.tau1, g=w.g, walls=(True, True, False))
        f = evd.run(m, evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE)), STEPS)
        ref = evd.collide(m, f)[:, :, 0, y - ya, x - xa]          # [N, Q]
        s = got[k]
        pop = (wts / wts[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, ((x, y), err)


def _workload_3d():
    rng = np.random.default_rng(22)
    d = rng.uniform(0.06, 0.1, size=(4, 4))
    diff = ((d + d.T) / 2).tolist()
    return W.Workload("max_box_3d", "D3Q19", 256, 128, NZ3, MASSES, diff, 1.0,
                      [1e-5, 0.0, -1e-5], [True, True, True], STEPS, "random", seed=22)


@pytest.mark.gpu
def test_largest_3d_lattice_sampled_nodes_match_oracle_crops():
    lbm = _lbm()
    w = _workload_3d()
    print(f"\n[gpu case] max-size 3-D box 256x128x{NZ3}, 4 species", flush=True)
    x0 = w.x0()
    total, _, _, _ = lbm.layout(lbm.params_from_workload(w))
    species_bytes = 256 * 128 * NZ3 * 19 * 4
    assert species_bytes < 2 ** 31 and species_bytes > 2 ** 31 - 2 ** 26
    assert total * 4 > 4 * (2 ** 31 - 2 ** 26)   # four species of nearly 2 GiB: 8.6 GB
    sim = lbm.LbmMc(lbm.params_from_workload(w), x0)
    sim.step(STEPS)
    raw = sim.raw("cur")
    dims = (w.nx, w.ny, w.nz)
    L = NZ3 - 1
    pts = [(0, 0, 0), (255, 127, L), (0, 127, L), (255, 0, 0), (128, 0, NZ3 // 2),
           (0, 64, L), (255, 127, 0), (77, 33, 600), (1, 126, L - 1)]
    got = torch.stack([raw[:, :, z, y, x] for (x, y, z) in pts]).double().cpu()   # [P, N, Q]
    sim.sync()
    sim.close()
    R = STEPS + 2
    m_ = evd.Model("D3Q19", 3, 3, 3, MASSES, torch.tensor(w.diff, dtype=DTYPE), w.tau1)
    wts = m_.lat.w
    for k, c in enumerate(pts):
        lo = [max(0, c[d] - R) for d in range(3)]
        hi = [min(dims[d], c[d] + R + 1) for d in range(3)]
        sub = x0[:, lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        m = evd.Model("D3Q19", hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], MASSES,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g,
                      walls=(True, True, True))
        f = evd.run(m, evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE)), STEPS)
        ref = evd.collide(m, f)[:, :, c[2] - lo[2], c[1] - lo[1], c[0] - lo[0]]   # [N, Q]
        s = got[k]
        pop = (wts / wts[0])[None, :] * s[:, :1] + s
        pop[:, 0] = s[:, 0]
        err = ((pop - ref).abs().max() / ref.abs().max()).item()
        assert err < F_RTOL, (c, err)
