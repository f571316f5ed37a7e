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
        "adjoint_tube": adjoint_tube, "layer_mixing_3d_small": layer_mixing_3d_small}


def main(names):
    for n in names or JOBS:
        print(n, flush=True)
        res = JOBS[n]()
        res["_about"] = ("oracle (FP64) result written by tests/golden/make_golden.py; "
                         "x[species][x-node] on a one-row lattice")
        with open(os.path.join(HERE, f"{n}.json"), "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main(sys.argv[1:])
