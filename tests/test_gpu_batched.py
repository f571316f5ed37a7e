"""GPU tests of the batched form: many independent lattices of uneven sizes,
each with its own masses, diffusivities and gravity, advanced together
(one persistent launch per step, or one launch per lattice)."""
import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE

pytestmark = pytest.mark.gpu

X_TOL = 1e-5
MASS_TOL = 1e-6


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _batch(tubes, **tuning):
    lbm = _lbm()
    sim = lbm.LbmMc([lbm.params_from_workload(w) for w in tubes], W.concat_x0(tubes))
    if tuning:
        sim.set_tuning(**tuning)
    return sim


@pytest.mark.parametrize("one_launch,persistent,variant", [(1, 0, 0), (1, 96, 0), (0, 0, 0),
                                                           (1, 96, 1)])
def test_batched_equals_single_lattice_runs(one_launch, persistent, variant):
    """Every lattice of a batch evolves bit-identically to the same lattice
    run alone (the per-node arithmetic does not depend on the batch), in both
    launch modes, with a persistent grid and in both kernel variants."""
    tubes = [W.batched_tubes(count=40)[i] for i in (0, 5, 17, 23, 31, 39)]
    _announce(f"batch of {len(tubes)} one_launch={one_launch} persistent={persistent} "
              f"variant={variant}")
    lbm = _lbm()
    sim = _batch(tubes, block_x=64, rows=8, persistent=persistent, variant=variant)
    sim.set_batched_mode(one_launch)
    sim.step(37)
    sim.sync()
    for l, w in enumerate(tubes):
        one = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        one.set_tuning(block_x=64, rows=8, variant=variant)    # same kernel variant
        one.step(37)
        one.sync()
        assert torch.equal(sim.raw("cur", l), one.raw("cur")), (l, w.nx, w.ny)
        one.close()


def test_batched_tubes_match_oracle():
    """Three tubes of the batch against the FP64 oracle (one row: the tubes are
    uniform along their periodic y axis) after 300 steps."""
    tubes = [W.batched_tubes(count=60)[i] for i in (2, 41, 57)]
    _announce("batched tubes vs oracle")
    sim = _batch(tubes)
    m0 = sim.moments(fields=False)["mass"].copy()
    sim.step(300)
    out = sim.moments()
    sim.sync()
    for l, w in enumerate(tubes):
        m = evd.Model("D2Q9", w.nx, 1, 1, w.masses, torch.tensor(w.diff, dtype=DTYPE), w.tau1,
                      g=w.g, walls=w.walls)
        f = evd.run(m, evd.initial_populations(m, torch.tensor(w.x0()[:, :, :1, :])), 300)
        ref = evd.observables(m, f)["x"][:, 0, 0, :].numpy()
        x = sim.field(out, "x", l).double().cpu().numpy()[:, 0]          # [N, ny, nx]
        assert np.abs(x - ref[:, None, :]).max() < X_TOL, l
        assert np.abs(out["mass"][l] / m0[l] - 1).max() < MASS_TOL, l


def test_full_batch_of_512_tubes_properties():
    """The full 512-tube batch (about 22.8 M nodes) at the execution shape the
    benchmark uses: per-tube FP64 mass conserved to 1e-6, every row of a tube
    identical (the tubes are y-uniform, so this holds at any size), and mole
    fractions inside [0, 1]."""
    tubes = W.batched_tubes()
    _announce("512 tubes")
    sim = _batch(tubes)
    m0 = sim.moments(fields=False)["mass"].copy()
    sim.step(64)
    out = sim.moments()
    sim.sync()
    assert np.abs(out["mass"] / m0 - 1).max() < MASS_TOL
    for l in range(0, len(tubes), 37):
        x = sim.field(out, "x", l)[:, 0]                 # [N, ny, nx]
        assert torch.equal(x, x[:, :1, :].expand_as(x)), l
        assert float(x.min()) >= 0.0 and float(x.max()) <= 1.0


def _mixed_walls(tubes):
    """The same tubes with walls on x and y (boxes) for every other one."""
    import dataclasses
    return [dataclasses.replace(w, walls=[True, True, False]) if i % 2 else w
            for i, w in enumerate(tubes)]


@pytest.mark.parametrize("one_launch,persistent,variant", [(1, 0, 1), (1, 96, 0), (0, 0, 1)])
def test_batch_of_boxes_and_tubes_equals_single_runs(one_launch, persistent, variant):
    """A batch mixing tubes (x walls) and boxes (walls on x and y, with
    corners) keeps every lattice bit-identical to its run alone: the wall
    mask is per lattice."""
    tubes = _mixed_walls([W.batched_tubes(count=40)[i] for i in (2, 7, 11, 19, 29)])
    _announce(f"batch of boxes and tubes one_launch={one_launch} persistent={persistent} "
              f"variant={variant}")
    lbm = _lbm()
    sim = _batch(tubes, block_x=64, rows=8, persistent=persistent, variant=variant)
    sim.set_batched_mode(one_launch)
    m0 = sim.moments(fields=False)["mass"].copy()
    sim.step(41)
    sim.sync()
    for l, w in enumerate(tubes):
        one = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        one.set_tuning(block_x=64, rows=8, variant=variant)
        one.step(41)
        one.sync()
        assert torch.equal(sim.raw("cur", l), one.raw("cur")), (l, w.walls)
        one.close()
    m1 = sim.moments(fields=False)["mass"]
    sim.sync()
    sim.close()
    assert np.abs(m1 / m0 - 1).max() < MASS_TOL


@pytest.mark.parametrize("one_launch,persistent", [(1, 0), (1, 96), (0, 0)])
def test_batch_with_the_equilibrium_boundary_equals_single_runs(one_launch, persistent):
    """The equilibrium comparison boundary in a batch (every lattice with it,
    as the library requires; tubes and boxes mixed), one thread per column:
    bit-identical to each lattice run alone."""
    import dataclasses
    tubes = [dataclasses.replace(w, wall_kind="equilibrium")
             for w in _mixed_walls([W.batched_tubes(count=40)[i] for i in (3, 8, 21, 33)])]
    _announce(f"equilibrium-boundary batch one_launch={one_launch} persistent={persistent}")
    lbm = _lbm()
    sim = _batch(tubes, block_x=64, rows=8, persistent=persistent, variant=0)
    sim.set_batched_mode(one_launch)
    sim.step(29)
    sim.sync()
    for l, w in enumerate(tubes):
        one = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        one.set_tuning(block_x=64, rows=8, variant=0)
        one.step(29)
        one.sync()
        assert torch.equal(sim.raw("cur", l), one.raw("cur")), (l, w.walls)
        one.close()
    sim.close()


@pytest.mark.parametrize("one_launch", [1, 0])
def test_batch_with_moving_walls_equals_single_runs(one_launch):
    """Tubes with moving walls (velocities along their walls) batched with
    tubes whose walls rest: the wall velocities are per lattice.  A batch
    runs one kernel specialisation for all its lattices, the moving-wall one
    here: the moving tubes are bit-identical to their runs alone, the resting
    ones (alone they run the plain specialisation, whose multiply-adds the
    compiler may contract differently) agree to rounding, 2e-6 of the
    largest population as between execution variants."""
    import dataclasses
    base = [W.batched_tubes(count=40)[i] for i in (1, 6, 13, 27)]
    tubes = [dataclasses.replace(w, wall_velocity=[[0.0, 0.01 * (i + 1), 0.0],
                                                   [0.0, -0.005, 0.0]]) if i % 2 == 0 else w
             for i, w in enumerate(base)]
    _announce(f"moving-wall batch one_launch={one_launch}")
    lbm = _lbm()
    sim = _batch(tubes, block_x=64, rows=8, variant=1)
    sim.set_batched_mode(one_launch)
    sim.step(33)
    sim.sync()
    for l, w in enumerate(tubes):
        one = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        one.set_tuning(block_x=64, rows=8, variant=1)
        one.step(33)
        one.sync()
        a, b = sim.raw("cur", l), one.raw("cur")
        if w.wall_velocity is not None:
            assert torch.equal(a, b), (l, w.wall_velocity)
        else:
            assert ((a - b).abs().max() / b.abs().max()).item() < 2e-6, l
        one.close()
    sim.close()


@pytest.mark.parametrize("one_launch", [1, 0])
def test_batch_with_force_fields_equals_single_runs(one_launch):
    """Every tube of a batch with its own force field k(x) in place of g (the
    fields concatenated per lattice, [lattice][d][nodes]): each lattice
    bit-identical to its run alone with its own field."""
    import dataclasses
    tubes = [dataclasses.replace(W.batched_tubes(count=40)[i], g=[0.0, 0.0, 0.0])
             for i in (4, 9, 22)]
    rng = np.random.default_rng(17)
    fields = [(rng.uniform(-2e-6, 2e-6, size=(2, 1, w.ny, w.nx))).astype(np.float32)
              for w in tubes]
    _announce(f"force-field batch one_launch={one_launch}")
    lbm = _lbm()
    acc = torch.tensor(np.concatenate([f.reshape(-1) for f in fields]), device="cuda")
    sim = lbm.LbmMc([lbm.params_from_workload(w) for w in tubes], W.concat_x0(tubes), accel=acc)
    sim.set_tuning(block_x=64, rows=8, variant=1)
    sim.set_batched_mode(one_launch)
    sim.step(29)
    sim.sync()
    for l, w in enumerate(tubes):
        one = lbm.LbmMc(lbm.params_from_workload(w), w.x0(),
                        accel=torch.tensor(fields[l], device="cuda"))
        one.set_tuning(block_x=64, rows=8, variant=1)
        one.step(29)
        one.sync()
        assert torch.equal(sim.raw("cur", l), one.raw("cur")), l
        one.close()
    sim.close()


def test_full_batch_10000_steps_matches_stored_oracle():
    """The whole 512-tube batch for its configured 10,000 steps, one launch per
    step at the default shape: six sampled tubes (first and last, longest and
    shortest, strongest gravity, heaviest third species; stored FP64 oracle
    results, one row each) within 1e-5 in mole fraction on every row, and
    every tube's FP64 mass within 1e-6."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "batched_sample.json")) as fh:
        G = json.load(fh)["tubes"]
    tubes = W.batched_tubes()
    _announce("full batch, 10000 steps")
    sim = _batch(tubes)
    m0 = sim.moments(fields=False)["mass"].copy()
    sim.step(10000)
    out = sim.moments()
    sim.sync()
    assert np.abs(out["mass"] / m0 - 1).max() < MASS_TOL
    for k, rec in G.items():
        ref = np.array(rec["10000"]["x"])
        x = sim.field(out, "x", lattice=int(k)).double().cpu().numpy()[:, 0]
        err = np.abs(x - ref[:, None, :]).max()
        assert err < X_TOL, (k, err)
    sim.close()
