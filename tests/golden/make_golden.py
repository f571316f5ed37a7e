"""Write the stored oracle results the GPU parity tests compare against.
Calls only the oracle (and the seeded input generators).  Run from the repo
root:  python -m tests.golden.make_golden [name ...]

The tube workloads are uniform along their periodic y axis (initial halves
differ only along x, the force is along x), so by translation invariance the
oracle runs them on a one-row lattice (ny = 1), which gives the same result
for every row; tests/test_oracle_stream.py checks that reduction.
"""
import json
import os
import sys
import time

import numpy as np
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE

HERE = os.path.dirname(os.path.abspath(__file__))


def tube_model(w, ny=1):
    return evd.Model(w.lattice, w.nx, ny, 1, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                     w.tau1, g=w.g, walls=w.walls, n0=w.n0)


def run_tube(w, checkpoints):
    m = tube_model(w)
    x0 = torch.tensor(w.x0()[:, :, :1, :], dtype=DTYPE)
    f = evd.initial_populations(m, x0)
    out = {}
    t = 0
    t0 = time.time()
    for cp in sorted(checkpoints):
        f = evd.run(m, f, cp - t)
        t = cp
        ob = evd.observables(m, f)
        out[str(cp)] = {
            "x": ob["x"][:, 0, 0, :].tolist(),
            "mass_per_row": ob["mass"].tolist(),
        }
        print(f"  t={cp} done ({time.time() - t0:.0f} s)", flush=True)
    return out


def ternary_gravity():
    w = W.ternary_gravity()
    return {"workload": w.name, "steps": w.steps,
            "checkpoints": run_tube(w, [0, 100, 2000, 20000])}


def binary_erf():
    w = W.binary_erf()
    return {"workload": w.name, "steps": w.steps,
            "checkpoints": run_tube(w, [0, 2000])}


def layer_mixing_3d_small():
    """D3Q19 layer workload on a 16x8x32 box (z walls, interface at z = 24,
    seeded 1 % perturbation), mole fractions at 500 and 5000 steps."""
    w = W.layer_mixing_3d(16, 8, 32, steps=5000)
    m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                  w.tau1, g=w.g, walls=w.walls, n0=w.n0)
    f = evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE))
    out, t, t0 = {}, 0, time.time()
    for cp in (500, 5000):
        with torch.no_grad():
            f = evd.run(m, f, cp - t)
        t = cp
        ob = evd.observables(m, f)
        out[str(cp)] = {"x": ob["x"].tolist(), "mass": ob["mass"].tolist()}
        print(f"  t={cp} done ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": w.name, "steps": w.steps, "checkpoints": out}


def layer_mixing_3d_64():
    """D3Q19 layer workload on a 64x32x32 box (z walls, interface at z = 24,
    seeded 1 % perturbation): the whole mole-fraction field at 100, 1000 and
    5000 steps, stored as float32 (its rounding, 6e-8, is far below the 1e-5
    parity bar) in a compressed npz next to this file."""
    w = W.layer_mixing_3d(64, 32, 32, steps=5000)
    m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                  w.tau1, g=w.g, walls=w.walls, n0=w.n0)
    f = evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE))
    arrays, t, t0 = {}, 0, time.time()
    for cp in (100, 1000, 5000):
        with torch.no_grad():
            while t < cp:
                n = min(100, cp - t)
                f = evd.run(m, f, n)
                t += n
                print(f"  t={t} ({time.time() - t0:.0f} s)", flush=True)
        ob = evd.observables(m, f)
        arrays[f"x_{cp}"] = ob["x"].numpy().astype(np.float32)
        arrays[f"mass_{cp}"] = ob["mass"].numpy()
    np.savez_compressed(os.path.join(HERE, "layer_mixing_3d_64x32x32.npz"),
                        workload=np.array(w.name), **arrays)
    return None


BATCH_SAMPLE = (0, 168, 206, 378, 444, 511)   # first, longest, shortest, strongest g,
                                              # heaviest, last tube


def batched_sample():
    """Six tubes of the 512-tube batch (first and last, the longest and the
    shortest, the strongest gravity, the heaviest third species), each run on
    one row for the batch's 10,000 steps; x at 1000 and 10,000 steps."""
    tubes = W.batched_tubes()
    out = {}
    for k in BATCH_SAMPLE:
        print(f" tube {k}", flush=True)
        out[str(k)] = run_tube(tubes[k], [1000, 10000])
    return {"workload": "batched_512_ternary_tubes", "steps": 10000, "tubes": out}


LAYER_SEAMS = [(64, 0, 0), (63, 127, 127), (128, 50, 16), (127, 51, 15), (192, 100, 96),
               (191, 101, 95), (0, 64, 112), (255, 65, 111), (64, 127, 32), (128, 0, 127)]


def layer_crops_16():
    """The 256x128x128 D3Q19 layer workload after 16 steps at ten nodes on the
    seams of the library's default tiles (x = 63|64, 127|128, 191|192, 255|0;
    z = 15|16, 31|32, 95|96, 111|112; every y row) and on both z walls: the
    post-collision populations f~ and the mole fractions there, from the
    oracle run on a crop of radius 17 around each node (after s steps a node
    depends only on its radius-s neighbourhood; the crop wraps periodically in
    x and y and keeps the z walls it reaches, so its centre is exact)."""
    w = W.layer_mixing_3d()
    x0 = w.x0()
    steps, R = 16, 17
    out = []
    t0 = time.time()
    for (x, y, z) in LAYER_SEAMS:
        xs = [(x + k) % w.nx for k in range(-R, R + 1)]
        ys = [(y + k) % w.ny for k in range(-R, R + 1)]
        z0, z1 = max(0, z - R), min(w.nz, z + R + 1)
        sub = np.ascontiguousarray(x0[:, z0:z1][:, :, ys][:, :, :, xs])
        m = evd.Model("D3Q19", len(xs), len(ys), z1 - z0, w.masses,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g,
                      walls=(False, False, z0 == 0 or z1 == w.nz), n0=w.n0)
        with torch.no_grad():
            f = evd.run(m, evd.initial_populations(m, torch.tensor(sub, dtype=DTYPE)), steps)
        ft = evd.collide(m, f)[:, :, z - z0, R, R]
        xo = evd.observables(m, f)["x"][:, z - z0, R, R]
        out.append({"node": [x, y, z], "f_post": ft.tolist(), "x": xo.tolist()})
        print(f"  node {(x, y, z)} ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": w.name, "steps": steps, "radius": R, "nodes": out}


HYPS = dict(nx=64, g=1e-5, x_mean=(0.4005, 0.249, 0.3505), steps=120000)


def hypsometric_model():
    """Ternary tube of the paper's gases' masses (2:28:44) with the seeded
    diffusivities of the 1024x64 workload, walls at the x ends, one row,
    gravity g along +x (ten times the workload's, so that the heaviest
    species' density varies by 4 % over the 64 nodes)."""
    w = W.ternary_gravity()
    return evd.Model("D2Q9", HYPS["nx"], 1, 1, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                     w.tau1, g=[HYPS["g"], 0.0, 0.0], walls=(True, False, False))


def hypsometric_walls():
    """Stationary state of the hypsometric tube: started at the closed form
    rho_i(x) = A_i exp(g x/c_{s,i}^2) (eq. MS_equation with k_i = g and eq.
    NSE at rest, with p_i = rho_i c_{s,i}^2) of a uniform mean composition,
    run until the state no longer changes (120,000 steps); stores the
    post-stream populations f and the last 10,000 steps' largest change in x."""
    from oracle import closed_forms
    m = hypsometric_model()
    nx, g = HYPS["nx"], HYPS["g"]
    M = np.array(m.M)
    xs = np.arange(nx, dtype=float)
    n0 = m.default_n0()
    mass = np.array(HYPS["x_mean"]) * M * n0 * nx
    rho = closed_forms.hypsometric_densities(list(M), mass, np.stack([xs, 0 * xs, 0 * xs], 1),
                                             [g, 0.0, 0.0])
    n = (rho / M[:, None]).sum(0)
    x = rho / M[:, None] / n
    f = evd.initial_populations(m, torch.tensor(x)[:, None, None, :])
    f = f * torch.tensor(n / n0)[None, None, None, None, :]
    t0, t, last = time.time(), 0, None
    while t < HYPS["steps"]:
        with torch.no_grad():
            f = evd.run(m, f, 10000)
        t += 10000
        xn = evd.observables(m, f)["x"][:, 0, 0, :]
        change = None if last is None else float((xn - last).abs().max())
        last = xn
        print(f"  t={t} change {change} ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": "hypsometric_walls_64", "nx": nx, "g": g, "x_mean": HYPS["x_mean"],
            "steps": t, "change_last_10000": change, "f": f[:, :, 0, 0, :].tolist()}


def adjoint_tube():
    """Adjoint workload: target profile from the true diffusivities, then the
    misfit and its gradient at the evaluation point by reverse mode (segments
    of 100 steps) and by central differences (relative step 1e-4)."""
    from oracle import adjoint as OA
    truth, ev = W.adjoint_tube()
    tube = OA.Tube("D2Q9", ev.nx, 1, 1, ev.masses, ev.tau1, ev.walls,
                   torch.tensor(ev.x0()[:, :, :1, :], dtype=DTYPE))
    pt = [truth.diff[0][1], truth.diff[0][2], truth.diff[1][2]]
    pe = [ev.diff[0][1], ev.diff[0][2], ev.diff[1][2]]
    t0 = time.time()
    with torch.no_grad():
        target = OA.profile(tube, torch.tensor(pt, dtype=DTYPE),
                            torch.tensor(truth.g, dtype=DTYPE), ev.steps)
    print(f"  target done ({time.time() - t0:.0f} s)", flush=True)
    L, dp, dg = OA.gradient(tube, pe, list(ev.g), target, ev.steps, segment=100)
    print(f"  reverse mode done ({time.time() - t0:.0f} s)", flush=True)
    fd = OA.central_fd(tube, pe, list(ev.g), target, ev.steps, h=1e-4)
    print(f"  finite differences done ({time.time() - t0:.0f} s)", flush=True)
    return {"workload": ev.name, "steps": ev.steps, "pairs_truth": pt, "pairs_eval": pe,
            "g_truth": list(truth.g), "g_eval": list(ev.g), "target": target.tolist(),
            "loss": L, "grad_pairs": dp, "grad_g": dg, "fd": fd, "fd_h": 1e-4}


JOBS = {"ternary_gravity": ternary_gravity, "binary_erf": binary_erf,
        "adjoint_tube": adjoint_tube, "layer_mixing_3d_small": layer_mixing_3d_small,
        "layer_mixing_3d_64": layer_mixing_3d_64, "hypsometric_walls": hypsometric_walls,
        "batched_sample": batched_sample, "layer_crops_16": layer_crops_16}


def main(names):
    for n in names or JOBS:
        if "torch_threads" in os.environ:
            torch.set_num_threads(int(os.environ["torch_threads"]))
        print(n, flush=True)
        res = JOBS[n]()
        if res is None:     # the job wrote its own file
            continue
        res["_about"] = ("oracle (FP64) result written by tests/golden/make_golden.py; "
                         "x[species][x-node] on a one-row lattice")
        with open(os.path.join(HERE, f"{n}.json"), "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main(sys.argv[1:])
