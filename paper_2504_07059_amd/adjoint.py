"""Gradients through the time stepping: a torch.autograd.Function whose
forward runs the library's fused steps and whose backward runs the library's
hand-written adjoint kernels (reverse mode of the discrete scheme), with
checkpoints every K steps and recomputation of each segment.

The differentiable inputs are the pair diffusivities D_ij (i < j, row-major)
and the specific body force g (F_i = rho_i g, eq. MS_equation); the output is
the mole-fraction profile xbar_i(x) after T steps (the mean over y and z of
x_i = rho_i/(M_i n), Sec. 3), computed by the library, whose backward starts
from the library's vector-Jacobian product of that profile.  A loss is any
torch function of the profile (``profile_misfit`` is the L2 misfit).  Every
step of the forward and reverse sweeps runs in the library's kernels; the
parameter gradients are accumulated in FP64 on the device.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import lbm

@dataclass
class Problem:
    """Everything but the differentiated parameters: geometry, masses, tau_1,
    walls, initial mole fractions [N, nz, ny, nx], number of steps and the
    checkpoint interval.  checkpoint_every = K >= 1 keeps every K-th state
    and recomputes each segment in the backward; checkpoint_every = 0 records
    every state in the forward (steps + 1 states of the population layout in
    device memory) and recomputes nothing; None records every state when
    they take at most half of the free device memory, else uses K = 100."""
    lattice: str
    nx: int
    ny: int
    nz: int
    masses: Sequence[float]
    tau1: float
    walls: Sequence[bool]
    x0: np.ndarray
    steps: int
    checkpoint_every: Optional[int] = 100
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


def _interval(problem, sim):
    """The checkpoint interval to use (0: record every state)."""
    if problem.checkpoint_every is not None:
        return int(problem.checkpoint_every)
    stride = (sim.total + 63) // 64 * 64
    need = 4 * stride * (problem.steps + 1)
    free, _ = torch.cuda.mem_get_info(sim.device)
    return 0 if need <= free // 2 else 100


class Evolve(torch.autograd.Function):
    """xbar(T): the profile of s(T) = Phi^T(s(0; D, g); D, g), s(0) the
    initialised state."""

    @staticmethod
    def forward(ctx, pairs, g, problem):
        pv = [float(v) for v in pairs.detach().cpu().tolist()]
        gv = [float(v) for v in g.detach().cpu().tolist()]
        sim = _sim(problem, pv, gv)
        K = _interval(problem, sim)
        if K < 0:
            raise ValueError("checkpoint_every must be >= 0")
        ctx.K = K
        ctx.pairs_meta = (pairs.device, pairs.dtype)
        ctx.g_meta = (g.device, g.dtype)
        ctx.sim, ctx.problem = sim, problem
        if K == 0:
            # every state, s(0) .. s(T), one row each: the forward itself
            # writes them (lbm_mc_replay), the backward reads them
            stride = (sim.total + 63) // 64 * 64
            states = torch.empty((problem.steps + 1, stride), dtype=torch.float32,
                                 device=sim.device)
            states[0, : sim.total].copy_(sim.buffers()[0])
            if problem.steps > 0:
                sim.replay(states[0], problem.steps, states[1:])
            ctx.states, ctx.ckpts = states, None
            ctx.s_T = states[problem.steps, : sim.total]
            return sim.profile(ctx.s_T)
        ctx.states = None
        ckpts = {}
        t = 0
        while t < problem.steps:
            ckpts[t] = sim.buffers()[0].clone()
            n = min(K, problem.steps - t)
            sim.step(n)
            t += n
        s_T = sim.buffers()[0].clone()
        xbar = sim.profile(s_T)
        ctx.ckpts, ctx.s_T = ckpts, s_T
        return xbar

    @staticmethod
    def backward(ctx, dxbar):
        sim, problem = ctx.sim, ctx.problem
        dev = sim.device
        lam_a = torch.zeros(sim.total, dtype=torch.float32, device=dev)
        lam_b = torch.zeros_like(lam_a)
        sim.profile_vjp(ctx.s_T, dxbar, lam_a)
        grad = torch.zeros(problem.n_pairs + 3, dtype=torch.float64, device=dev)
        K = ctx.K
        if K == 0:
            if problem.steps > 0:
                sim.adjoint_run(ctx.states, problem.steps, lam_a, lam_b, grad)
                lam_a, lam_b = lam_b, lam_a
        else:
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
        ctx.states = None
        ctx.s_T = None
        npair = problem.n_pairs
        return (grad[:npair].to(*ctx.pairs_meta), grad[npair:].to(*ctx.g_meta), None)


def evolve(pairs, g, problem):
    """Differentiable run: returns the mole-fraction profile xbar [N, nx]
    (float64, on the device) after problem.steps steps, for parameters
    pairs [n_pairs] and g [3]."""
    return Evolve.apply(pairs, g, problem)


def profile_misfit(xbar, target):
    """sum_s sum_x (xbar_s(x) - target_s(x))^2, target [N, nx]."""
    return ((xbar - target) ** 2).sum()
