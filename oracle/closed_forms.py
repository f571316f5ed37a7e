"""Analytic results the method must reproduce.  Lattice units, M_1 = 1,
c_{s,1}^2 = 1/3.  These are independent of ``oracle.evd`` (they share no code
with it) and serve as its pins."""
import math

import numpy as np
from scipy.special import erfc


def binary_erf_profile(x, t, x_interface, D):
    """Binary interdiffusion of two species of equal molar mass from a step
    x_1 = 1 | 0 at x_interface: x_1(x, t) = erfc((x - x0)/(2 sqrt(D t)))/2.
    For an ideal binary mixture of equal masses the Maxwell-Stefan equation
    recovered by the method (eq. MS_equation with k_i = 0 and uniform p) is
    Fick's law with the diffusivity D_12."""
    return 0.5 * erfc((np.asarray(x, dtype=float) - x_interface) / (2.0 * math.sqrt(D * t)))


def luo_girimaji_tau(rho1, rho2, M1, M2, D):
    """Binary tau_12 = dt/2 + n^2 M_1 M_2 D_12/(p rho), eq. (Luo&Girimaji_tau),
    with n = rho1/M1 + rho2/M2 and p = n M_1 c_{s,1}^2, c_{s,1}^2 = 1/3."""
    n = rho1 / M1 + rho2 / M2
    p = n * M1 / 3.0
    return 0.5 + n * n * M1 * M2 * D / (p * (rho1 + rho2))


def ternary_taus(rho, M, D):
    """tau_23, tau_12, tau_13 of the analytic ternary solution of Sec. 4.1:
      tau_23 = (A_23 - rho1 rho2/(A_13 D13 D23)) / (B_23 - rho1 B_13/(A_13 D23))
      tau_12 = (B_12/A_12 - rho3/(A_12 D12 tau_23))^-1
      tau_13 = (B_13/A_13 - rho2/(A_13 D13 tau_23))^-1
    with A_ij = (rho_i+rho_j)/D_ij + 2 n^2 M_i M_j/(p dt), B_ij = 2 rho/(D_ij dt),
    p = n M_1 c_{s,1}^2.  Indices here are 0-based: rho = (rho1, rho2, rho3)."""
    r1, r2, r3 = rho
    n = r1 / M[0] + r2 / M[1] + r3 / M[2]
    p = n * M[0] / 3.0
    R = r1 + r2 + r3

    def A(i, j):
        return (rho[i] + rho[j]) / D[i][j] + 2.0 * n * n * M[i] * M[j] / p

    def B(i, j):
        return 2.0 * R / D[i][j]

    t23 = (A(1, 2) - r1 * r2 / (A(0, 2) * D[0][2] * D[1][2])) / \
        (B(1, 2) - r1 * B(0, 2) / (A(0, 2) * D[1][2]))
    t12 = 1.0 / (B(0, 1) / A(0, 1) - r3 / (A(0, 1) * D[0][1] * t23))
    t13 = 1.0 / (B(0, 2) / A(0, 2) - r2 / (A(0, 2) * D[0][2] * t23))
    return t23, t12, t13


def hypsometric_densities(masses_norm, species_mass, coords, k, weights=None):
    """Equilibrium of an ideal mixture at rest under a uniform specific force k
    (the same for all species): eq. (MS_equation) with k_i = k loses its force
    term, the recovered NSE at rest gives grad p = rho k, and with
    p_i = rho_i c_{s,i}^2 (Sec. 3 before eq. NSE) every species obeys
    grad p_i = rho_i k, so rho_i(x) = A_i exp(k.x / c_{s,i}^2),
    c_{s,i}^2 = 1/(3 M_i).  A_i is fixed by the conserved mass of the species.

    coords: [P, 3] node coordinates; weights: multiplicity of each coordinate
    (e.g. the number of nodes in a y-row) for the mass sum."""
    coords = np.asarray(coords, dtype=float)
    k = np.asarray(k, dtype=float)
    wts = np.ones(len(coords)) if weights is None else np.asarray(weights, float)
    out = []
    for Mi, mi in zip(masses_norm, species_mass):
        cs2 = 1.0 / (3.0 * Mi)
        shape = np.exp(coords @ k / cs2)
        out.append(mi * shape / (wts * shape).sum())
    return np.array(out)


def centrifuge_densities(masses_norm, species_mass, r, omega2, weights=None):
    """Equilibrium under the centrifugal specific force k = omega_u^2 r along r
    (Sec. 4.2): the potential of k is omega^2 r^2/2, so as above
    rho_i(r) = A_i exp(omega^2 r^2 / (2 c_{s,i}^2))."""
    r = np.asarray(r, dtype=float)
    wts = np.ones(len(r)) if weights is None else np.asarray(weights, float)
    out = []
    for Mi, mi in zip(masses_norm, species_mass):
        cs2 = 1.0 / (3.0 * Mi)
        shape = np.exp(omega2 * r * r / (2.0 * cs2))
        out.append(mi * shape / (wts * shape).sum())
    return np.array(out)


def centrifuge_x1(r, x1_at_0, C):
    """Steady mole fraction of species 1, Sec. 4.2: solving
    x1 (1 - x1|0) / (x1|0 (1 - x1)) = exp(C r^2/2) for x1."""
    a = x1_at_0 / (1.0 - x1_at_0) * np.exp(C * np.asarray(r, float) ** 2 / 2.0)
    return a / (1.0 + a)


def centrifuge_constant(M1, M2, omega2):
    """C = (M_1 - M_2) omega_u^2 / (R_U T) with R_U T = M_1 c_{s,1}^2 (Sec. 4.2)."""
    return (M1 - M2) * omega2 / (M1 / 3.0)
