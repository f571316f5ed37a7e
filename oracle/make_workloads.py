"""Decide which seeded diffusivity draws the workloads keep, and store them in
lbm_workloads/accepted.json.  Run as ``python -m oracle.make_workloads``.

Rule (a reading; the paper only warns about instability, Sec. 3 after
eq. Luo&Girimaji_tau): draw D_ij ~ U[0.01, 0.1] from numpy's default_rng(seed)
and keep the first draw whose velocity-difference relaxation matrix K
(oracle.stability) has all eigenvalues in [0, 1.9] at 41 compositions on the
segment between the workload's two initial mixtures.  The number of rejected
draws is stored with the result.
"""
import json
import sys

import torch

import lbm_workloads as W
from . import evd, stability
from .lattice import DTYPE

LAM_LIMIT = 1.9


def _model(lattice, masses, D, tau1=1.0):
    n = len(masses)
    dims = (4, 1, 1) if lattice == "D2Q9" else (2, 2, 2)
    return evd.Model(lattice, dims[0], dims[1], dims[2], masses,
                     torch.tensor(D, dtype=DTYPE), tau1)


def accept(seed, lattice, masses, segment, extra_checks=()):
    n = len(masses)
    for tries, pairs in enumerate(W.diffusivity_candidates(seed, n, 100000)):
        D = W.pairs_to_matrix(pairs, n)
        ok, worst = stability.is_stable(_model(lattice, masses, D), segment, LAM_LIMIT)
        if ok and all(chk(D) for chk in extra_checks):
            return {"pairs": [float(p) for p in pairs], "rejected": tries,
                    "lambda_max": worst}
    raise RuntimeError("no stable draw")


def main(out_path=W.ACCEPTED_PATH):
    res = {}
    seg3 = W.composition_segment(W.GAS_A, W.GAS_B)
    res["ternary_gravity"] = accept(1, "D2Q9", [2.0, 28.0, 44.0], seg3)
    seg4 = W.composition_segment(W.LAYER_CARRIER, W.LAYER_DENSE)
    res["layer_mixing_3d"] = accept(2, "D3Q19", [1.0, 2.0, 3.0, 4.0], seg4)

    # Adjoint truth: the perturbed evaluation point must be stable as well.
    import numpy as np
    fac = np.random.default_rng(4).uniform(-1.0, 1.0, size=3)

    def eval_point_ok(D):
        pairs = [D[0][1], D[0][2], D[1][2]]
        pert = [p * (1.0 + 0.2 * f) for p, f in zip(pairs, fac)]
        ok, _ = stability.is_stable(
            _model("D2Q9", [2.0, 28.0, 44.0], W.pairs_to_matrix(pert, 3)), seg3, LAM_LIMIT)
        return ok

    res["adjoint_tube"] = accept(4, "D2Q9", [2.0, 28.0, 44.0], seg3, (eval_point_ok,))

    tubes = []
    geo = W.batched_tube_geometry(3, 512)
    for t, gm in enumerate(geo):
        # each tube draws from its own stream: seed 3 * 100000 + t
        tubes.append(accept(300000 + t, "D2Q9", gm["masses"], seg3))
    res["batched_tubes"] = {"tubes": tubes}
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    print(f"wrote {out_path}")
    return res


if __name__ == "__main__":
    main(*sys.argv[1:])
