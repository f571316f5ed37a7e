"""Discrete-velocity lattices used by the oracle.

D2Q9 follows the paper's direction numbering (Sec. 2, equation defining the
species discrete velocities e_alpha^i): alpha = 0 is rest, alpha = 1..4 point
along (cos, sin) of (alpha-1) pi/2, alpha = 5..8 along the diagonals at
(alpha-5) pi/2 + pi/4.  The weights omega_alpha are the standard D2Q9 values;
the paper only calls them "weights" (Sec. 2, after the equilibrium).

D3Q19 is not in the paper (it uses D2Q9 throughout, Sec. 4 opening).  The
three-dimensional workload uses the standard D3Q19 set with weights 1/3, 1/18,
1/36; the species velocities are again c_i times the integer directions.
"""
import math
from fractions import Fraction

import torch

DTYPE = torch.float64


def _d2q9_from_paper():
    """Integer directions from the paper's cos/sin definition, rounded."""
    dirs = [(0, 0)]
    for a in range(1, 5):
        ang = (a - 1) * math.pi / 2
        dirs.append((round(math.cos(ang)), round(math.sin(ang))))
    for a in range(5, 9):
        ang = (a - 5) * math.pi / 2 + math.pi / 4
        dirs.append((round(math.sqrt(2) * math.cos(ang)),
                     round(math.sqrt(2) * math.sin(ang))))
    return [(cx, cy, 0) for cx, cy in dirs]


D2Q9_DIRS = _d2q9_from_paper()
D2Q9_W = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4

D3Q19_DIRS = [
    (0, 0, 0),
    (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
    (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
    (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
    (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1),
]
D3Q19_W = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12


class Lattice:
    """Direction table, weights and opposite-direction map of one lattice."""

    def __init__(self, name):
        if name == "D2Q9":
            dirs, w, dim = D2Q9_DIRS, D2Q9_W, 2
        elif name == "D3Q19":
            dirs, w, dim = D3Q19_DIRS, D3Q19_W, 3
        else:
            raise ValueError(f"unknown lattice {name!r}")
        self.name = name
        self.dim = dim
        self.Q = len(dirs)
        self.dirs = dirs                       # list of integer 3-tuples
        self.weights_exact = w                 # Fractions
        self.c = torch.tensor(dirs, dtype=DTYPE)          # [Q, 3]
        self.w = torch.tensor([float(x) for x in w], dtype=DTYPE)  # [Q]
        self.opp = [dirs.index(tuple(-v for v in d)) for d in dirs]
