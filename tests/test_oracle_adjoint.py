"""Pins of the oracle's discrete adjoint (reverse mode through the FP64
oracle steps, oracle/adjoint.py): against central finite differences of the
plain forward runs, and checkpointed against plain reverse mode."""
import json
import os

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import adjoint as OA
from oracle.lattice import DTYPE

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tube(nx=40, steps=150):
    truth, ev = W.adjoint_tube(nx=nx, ny=1, steps=steps)
    tube = OA.Tube("D2Q9", nx, 1, 1, ev.masses, ev.tau1, ev.walls,
                   torch.tensor(ev.x0(), dtype=DTYPE))
    pairs_t = [truth.diff[0][1], truth.diff[0][2], truth.diff[1][2]]
    pairs_e = [ev.diff[0][1], ev.diff[0][2], ev.diff[1][2]]
    with torch.no_grad():
        target = OA.profile(tube, torch.tensor(pairs_t, dtype=DTYPE),
                            torch.tensor(truth.g, dtype=DTYPE), steps)
    return tube, pairs_e, list(ev.g), target, steps


def test_autograd_matches_central_differences():
    """Reverse mode through 150 oracle steps against central FD with relative
    steps 1e-4 (truncation O(h^2) ~ 1e-8 relative): the three diffusivities and
    g_x agree to 1e-6 relative."""
    tube, pairs, g, target, steps = _tube()
    L, dp, dg = OA.gradient(tube, pairs, g, target, steps, segment=0)
    assert L > 0
    fd = OA.central_fd(tube, pairs, g, target, steps)
    ad = {"D0": dp[0], "D1": dp[1], "D2": dp[2], "gx": dg[0]}
    for k, v in fd.items():
        assert abs(ad[k] - v) <= 1e-6 * abs(v), (k, ad[k], v)


def test_truth_is_stationary():
    """At the true parameters the misfit and its gradient vanish."""
    truth, _ = W.adjoint_tube(nx=40, ny=1, steps=60)
    tube = OA.Tube("D2Q9", 40, 1, 1, truth.masses, truth.tau1, truth.walls,
                   torch.tensor(truth.x0(), dtype=DTYPE))
    pairs = [truth.diff[0][1], truth.diff[0][2], truth.diff[1][2]]
    with torch.no_grad():
        target = OA.profile(tube, torch.tensor(pairs, dtype=DTYPE),
                            torch.tensor(truth.g, dtype=DTYPE), 60)
    L, dp, dg = OA.gradient(tube, pairs, truth.g, target, 60, segment=0)
    assert L == 0.0
    assert max(abs(v) for v in dp + dg) == 0.0


def test_checkpointed_reverse_mode_is_exact():
    """Checkpoint segments (recomputation) give the same gradient as keeping
    the whole graph, to rounding."""
    tube, pairs, g, target, steps = _tube(nx=32, steps=90)
    a = OA.gradient(tube, pairs, g, target, steps, segment=0)
    b = OA.gradient(tube, pairs, g, target, steps, segment=25)
    assert abs(a[0] - b[0]) <= 1e-14 * abs(a[0])
    for u, v in zip(a[1] + a[2], b[1] + b[2]):
        assert abs(u - v) <= 1e-12 * max(abs(u), 1e-30)


def test_golden_adjoint_gradient_agrees_with_its_finite_differences():
    """The stored full-size reference (512x64 tube, 4000 steps, reduced to one
    row by y-uniformity): reverse-mode and FD gradients agree to 1e-6."""
    with open(os.path.join(GOLDEN, "adjoint_tube.json")) as fh:
        G = json.load(fh)
    ad = {"D0": G["grad_pairs"][0], "D1": G["grad_pairs"][1], "D2": G["grad_pairs"][2],
          "gx": G["grad_g"][0]}
    for k, v in G["fd"].items():
        assert abs(ad[k] - v) <= 1e-6 * abs(v), (k, ad[k], v)
    assert np.asarray(G["target"]).shape == (3, 512)
