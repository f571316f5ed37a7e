"""Linear stability of the velocity-difference relaxation (reading of the
paper, which only warns that the velocity-dependent form of the tau relation
may be unstable, Sec. 3 after eq. Luo&Girimaji_tau).

At a spatially uniform node the collision changes the momentum of species i
by exactly F_i - Theta_i (Sec. 3: first moment of the forcing term,
eq. CE_EQ54, and Theta_i of eq. CE_theta_definition), and streaming leaves a
uniform state unchanged.  Hence the equilibrium velocities evolve as

    u^eq(t+1) = (I - K) u^eq(t) + k,
    K_ii = sum_{j != i} rho_j y_ij / rho,   K_ij = -rho_j y_ij / rho,

with y_ij = 1/tau_ij.  diag(rho)^(1/2) K diag(rho)^(-1/2) is symmetric, so the
eigenvalues of K are real; the velocity-difference modes are stable iff they
all lie in [0, 2).
"""
import numpy as np
import torch

from . import evd
from .lattice import DTYPE


def relaxation_matrix(model, x):
    """K at a uniform node at rest with mole fractions x (length N), with the
    densities of the initial state rho_i = x_i M_i n0 (Sec. 4.1)."""
    N = model.N
    x = torch.as_tensor(x, dtype=DTYPE).reshape(N, 1, 1, 1)
    M = torch.tensor(model.M, dtype=DTYPE).reshape(N, 1, 1, 1)
    rho_i = x * M * model.default_n0()
    ueq = torch.zeros(N, 1, 1, 1, 3, dtype=DTYPE)
    rho, u, n, p = evd.mixture(model, rho_i, ueq)
    Y = evd.cross_relaxation(model, rho_i, rho, n, p)[:, :, 0, 0, 0].numpy()
    r = rho_i.reshape(N).numpy()
    R = float(rho.reshape(()))
    K = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            if i != j:
                K[i, j] = -r[j] * Y[i, j] / R
                K[i, i] += r[j] * Y[i, j] / R
    return K


def eig_range(model, x):
    """(lambda_min, lambda_max) of K, computed from the symmetric form."""
    K = relaxation_matrix(model, x)
    N = model.N
    M = np.array(model.M)
    r = np.asarray(x, dtype=float) * M * model.default_n0()
    s = np.sqrt(np.maximum(r, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        Ks = (s[:, None] * K) / np.where(s[None, :] == 0, 1.0, s[None, :])
    Ks = 0.5 * (Ks + Ks.T)
    ev = np.linalg.eigvalsh(Ks)
    return float(ev[0]), float(ev[-1])


def is_stable(model, compositions, lam_max=2.0):
    """True if every composition gives eigenvalues in [0, lam_max)."""
    worst = 0.0
    for x in compositions:
        lo, hi = eig_range(model, x)
        if lo < -1e-12:
            return False, hi
        worst = max(worst, hi)
    return worst < lam_max, worst
