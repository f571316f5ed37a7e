"""The paper's comparison of wall schemes (Sec. 4.1, the Ga = 0 Loschmidt
tube): with the equilibrium boundary, solid nodes holding f^(0)(rho_s, 0) of
the adjacent fluid node, the total mass is not conserved once species of
different molar mass need the interpolation; with the proposed scheme of
Appendix A it is constant from initialisation.  The oracle reproduces that
contrast on a small tube with the paper's gases A and B and masses 2:28:44."""
import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd
from oracle.lattice import DTYPE


def _tube():
    D = torch.tensor(W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3),
                     dtype=DTYPE)
    m = evd.Model("D2Q9", 48, 1, 1, [2.0, 28.0, 44.0], D, 1.0, walls=(True, False, False))
    x0 = np.zeros((3, 1, 1, 48))
    x0[:, 0, 0, :24] = np.array([0.001, 0.299, 0.7])[:, None]
    x0[:, 0, 0, 24:] = np.array([0.8, 0.199, 0.001])[:, None]
    return m, evd.initial_populations(m, torch.tensor(x0, dtype=DTYPE))


def test_equilibrium_boundary_loses_mass_where_appendix_a_conserves_it():
    m, f = _tube()
    m0 = f.sum(dim=(1, 2, 3, 4))
    fa, fe = f, f
    drift_e = []
    for _ in range(6):
        for _ in range(100):
            fa = evd.stream(m, evd.collide(m, fa))
            fe = evd.stream_equilibrium_walls(m, evd.collide(m, fe))
        drift_e.append(((fe.sum(dim=(1, 2, 3, 4)) - m0) / m0).abs().max().item())
    drift_a = ((fa.sum(dim=(1, 2, 3, 4)) - m0) / m0).abs().max().item()
    assert drift_a < 1e-13
    # the equilibrium boundary's species masses wander by parts in 1e4 (the
    # pressure waves of the mixing reflect from walls that do not return the
    # mass they take), at every checkpoint
    assert min(drift_e) > 1e-5 and max(drift_e) > 1e-4


def test_equilibrium_boundary_keeps_a_uniform_rest_state():
    """Sanity of the comparison scheme: at a uniform composition at rest the
    solid nodes hold exactly the fluid's own populations, so nothing moves."""
    m, _ = _tube()
    x = torch.tensor([0.2, 0.3, 0.5], dtype=DTYPE)[:, None, None, None].expand(3, 1, 1, 48)
    f = evd.initial_populations(m, x.clone())
    g = evd.stream_equilibrium_walls(m, evd.collide(m, f))
    assert (g - f).abs().max() < 1e-15
