"""Gradients through the time stepping: a torch.autograd.Function whose
forward runs the library's fused steps and whose backward runs the library's
hand-written adjoint kernels (reverse mode of the discrete scheme), with
checkpoints every K steps and recomputation of each segment.

The differentiable inputs are the pair diffusivities D_ij (i < j, row-major)
and the specific body force g (F_i = rho_i g, eq. MS_equation); the output is
the stored state s(T) after T steps, from which a loss is built with torch
operations (``mole_fractions`` gives x_i = rho_i/(M_i n), Sec. 3).  Every
step of the forward and reverse sweeps runs in the library's kernels; the
parameter gradients are accumulated in FP64 on the device.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import lbm

WEIGHTS = lbm.LATTICE_WEIGHTS


@dataclass
class Problem:
    """Everything but the differentiated parameters: geometry, masses, tau_1,
    walls, initial mole fractions [N, nz, ny, nx], number of steps and the
    checkpoint interval."""
    lattice: str
    nx: int
    ny: int
    nz: int
    masses: Sequence[float]
    tau1: float
    walls: Sequence[bool]
    x0: np.ndarray
    steps: int
    checkpoint_every: int = 100
    n0: float = 0.0
    tuning: Optional[dict] = None
    stats: dict = field(default_factory=dict)

    @property
    def n_species(self):
        return len(self.masses)

    @property
    def n_pairs(self):
        n = self.n_species
        return n * (n - 1) // 2


def pairs_to_matrix(pairs, n):
    D = [[0.0] * n for _ in range(n)]
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            D[i][j] = D[j][i] = float(pairs[k])
            k += 1
    return D


def _sim(problem, pairs, g):
    p = lbm.make_params(problem.lattice, problem.nx, problem.ny, problem.nz, problem.masses,
                        pairs_to_matrix(pairs, problem.n_species), problem.tau1, g,
                        problem.walls, problem.n0)
    sim = lbm.LbmMc(p, problem.x0)
    if problem.tuning:
        sim.set_tuning(**problem.tuning)
    return sim


class Evolve(torch.autograd.Function):
    """s(T) = Phi^T(s(0; D, g); D, g) with s(0) the initialised state."""

    @staticmethod
    def forward(ctx, pairs, g, problem):
        pv = [float(v) for v in pairs.detach().cpu().tolist()]
        gv = [float(v) for v in g.detach().cpu().tolist()]
        sim = _sim(problem, pv, gv)
        K = int(problem.checkpoint_every)
        if K < 1:
            raise ValueError("checkpoint_every must be >= 1")
        ckpts = {}
        t = 0
        while t < problem.steps:
            ckpts[t] = sim.buffers()[0].clone()
            n = min(K, problem.steps - t)
            sim.step(n)
            t += n
        out = sim.raw("cur").clone()
        ctx.sim, ctx.ckpts, ctx.problem = sim, ckpts, problem
        ctx.pairs_meta = (pairs.device, pairs.dtype)
        ctx.g_meta = (g.device, g.dtype)
        return out

    @staticmethod
    def backward(ctx, lam_T):
        sim, problem = ctx.sim, ctx.problem
        dev = sim.device
        lam_a = torch.zeros(sim.total, dtype=torch.float32, device=dev)
        lam_b = torch.zeros_like(lam_a)
        sim.view(lam_a).copy_(lam_T.to(torch.float32))
        grad = torch.zeros(problem.n_pairs + 3, dtype=torch.float64, device=dev)
        K = int(problem.checkpoint_every)
        stride = (sim.total + 63) // 64 * 64
        seg = torch.empty((min(K, problem.steps), stride), dtype=torch.float32, device=dev)
        for t0 in sorted(ctx.ckpts, reverse=True):
            n = min(K, problem.steps - t0)
            seg[0, : sim.total].copy_(ctx.ckpts[t0])
            if n > 1:
                sim.replay(seg[0], n - 1, seg[1:n])
            sim.adjoint_run(seg, n, lam_a, lam_b, grad)
            lam_a, lam_b = lam_b, lam_a
        sim.adjoint_init(lam_a, grad)
        ctx.sim = None
        ctx.ckpts = None
        npair = problem.n_pairs
        return (grad[:npair].to(*ctx.pairs_meta), grad[npair:].to(*ctx.g_meta), None)


def evolve(pairs, g, problem):
    """Differentiable run: returns the stored state s(T) [N, Q, nz, ny, nx]
    (float32, on the device) for parameters pairs [n_pairs] and g [3]."""
    return Evolve.apply(pairs, g, problem)


def densities(state, Q):
    """Species densities rho_i = P0/w_0 + sum_{a>=1} g_a of a stored state
    [N, Q, ...], in float64 (the collision conserves rho_i, so these are also
    the densities of the streamed populations)."""
    s = state.double()
    return s[:, 0] / WEIGHTS[Q][0] + s[:, 1:].sum(dim=1)


def mole_fractions(state, masses, Q):
    """x_i = rho_i/(M_i n), n = sum_j rho_j/M_j (Sec. 3), of a stored state."""
    rho = densities(state, Q)
    M = torch.tensor([m / masses[0] for m in masses], dtype=torch.float64,
                     device=rho.device).view(-1, *([1] * (rho.dim() - 1)))
    nm = rho / M
    return nm / nm.sum(dim=0, keepdim=True)


def profile_misfit(state, masses, Q, target):
    """sum_s sum_x (xbar_s(x) - target_s(x))^2 with xbar the mean of the mole
    fraction over y and z: target [N, nx]."""
    x = mole_fractions(state, masses, Q)              # [N, nz, ny, nx]
    xbar = x.mean(dim=(1, 2))
    return ((xbar - target) ** 2).sum()
