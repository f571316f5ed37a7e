"""Reference gradients through the oracle's time stepping (test infrastructure:
see the package header for who may use it).

The discrete adjoint of the scheme is the reverse mode of its time stepping.
Here it is obtained by torch.autograd through the FP64 oracle steps of
``evd`` (``torch.utils.checkpoint`` segments keep the memory bounded; they
recompute, they do not approximate), and independently by central finite
differences of the plain forward runs.  The FD gradient pins the autograd one
(``tests/test_oracle_adjoint.py``).

The loss is a mole-fraction profile misfit, the inverse problem of fitting
the Maxwell-Stefan diffusivities (Sec. 3, Table 2) and the body force
(Sec. 4.1) to a measured composition profile:
    L = sum_s sum_x (xbar_s(x, T) - xbar*_s(x))^2,
xbar the mole fraction x_s = rho_s/(M_s n) (Sec. 3) averaged over y and z.
"""
from dataclasses import dataclass
from typing import Sequence

import torch
from torch.utils.checkpoint import checkpoint

from . import evd
from .lattice import DTYPE


@dataclass
class Tube:
    """Everything but the differentiated parameters."""
    lattice: str
    nx: int
    ny: int
    nz: int
    masses: Sequence[float]
    tau1: float
    walls: Sequence[bool]
    x0: torch.Tensor            # [N, nz, ny, nx] float64
    n0: float = None


def pair_matrix(pairs, n):
    """Symmetric [n, n] diffusivity matrix from the pairs i < j (row-major),
    built with differentiable operations."""
    D = torch.zeros((n, n), dtype=DTYPE)
    k = 0
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in range(i + 1, n):
            rows += [i, j]
            cols += [j, i]
            vals += [pairs[k], pairs[k]]
            k += 1
    return D.index_put((torch.tensor(rows), torch.tensor(cols)), torch.stack(vals))


def model(tube, pairs, g):
    return evd.Model(tube.lattice, tube.nx, tube.ny, tube.nz, tube.masses,
                     pair_matrix(pairs, len(tube.masses)), tube.tau1, g=g,
                     walls=tube.walls, n0=tube.n0)


def profile(tube, pairs, g, steps, segment=0):
    """xbar [N, nx] at t = steps; segment > 0 wraps every `segment` steps in a
    checkpoint (for autograd runs)."""
    m = model(tube, pairs, g)
    f = evd.initial_populations(m, tube.x0)
    t = 0
    while t < steps:
        n = min(segment, steps - t) if segment else steps - t
        if segment and f.requires_grad:
            f = checkpoint(lambda h, n=n: evd.run(m, h, n), f, use_reentrant=False)
        else:
            f = evd.run(m, f, n)
        t += n
    x = evd.observables(m, f)["x"]                  # [N, nz, ny, nx]
    return x.mean(dim=(1, 2))


def misfit(xbar, target):
    return ((xbar - target) ** 2).sum()


def gradient(tube, pairs, g, target, steps, segment=100):
    """(L, dL/dpairs, dL/dg) by reverse mode through the oracle steps."""
    p = torch.tensor(pairs, dtype=DTYPE, requires_grad=True)
    gg = torch.tensor(g, dtype=DTYPE, requires_grad=True)
    L = misfit(profile(tube, p, gg, steps, segment), target)
    L.backward()
    return L.item(), p.grad.tolist(), gg.grad.tolist()


def central_fd(tube, pairs, g, target, steps, h=1e-4, which=None):
    """Central differences with relative steps theta (1 +- h) for the pairs
    and the nonzero components of g (a zero parameter has no relative step
    and is skipped).  Returns {name: derivative}."""
    def loss(p, gg):
        with torch.no_grad():
            return misfit(profile(tube, torch.tensor(p, dtype=DTYPE),
                                  torch.tensor(gg, dtype=DTYPE), steps), target).item()

    out = {}
    names = [f"D{k}" for k in range(len(pairs))] + ["gx", "gy", "gz"]
    for k, name in enumerate(names):
        if which is not None and name not in which:
            continue
        base = list(pairs) + list(g)
        if base[k] == 0.0:
            continue
        dh = h * base[k]
        lo, hi = list(base), list(base)
        lo[k] -= dh
        hi[k] += dh
        n = len(pairs)
        out[name] = (loss(hi[:n], hi[n:]) - loss(lo[:n], lo[n:])) / (2 * dh)
    return out
