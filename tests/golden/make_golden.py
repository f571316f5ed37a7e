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


JOBS = {"ternary_gravity": ternary_gravity, "binary_erf": binary_erf}


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
