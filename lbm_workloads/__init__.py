"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module draws random numbers and lays out initial mole-fraction
fields; it contains none of the lattice Boltzmann method's arithmetic.

The workloads stand in for the paper's Case I (a ternary H2/CH4/Ar Loschmidt
tube under gravity, Sec. 4.1): the paper's conversion of its physical data to
lattice units is not given, so the workloads keep its structure (two halves of
different uniform composition, gravity, impermeable end walls) and draw their
transport coefficients from seeds.

Pair diffusivities are drawn here as *candidates*; whether a draw is kept
depends on the linear stability of the cross-relaxation times, which is the
method's arithmetic and so is decided once, offline, by
``oracle/make_workloads.py``.  The kept values are stored in ``accepted.json``
next to this file, and this module only reads them.
"""
import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ACCEPTED_PATH = os.path.join(_HERE, "accepted.json")

# Case I gases (Sec. 4.1): gas A has x_1 = 0.001, x_3 = 0.7; gas B has
# x_1 = 0.8, x_3 = 0.001; x_2 fills the rest.
GAS_A = (0.001, 0.299, 0.7)
GAS_B = (0.8, 0.199, 0.001)
# Three-dimensional layer workload: a dense layer over a light carrier.
LAYER_DENSE = (0.05, 0.05, 0.05, 0.85)
LAYER_CARRIER = (0.85, 0.10, 0.04, 0.01)

D_RANGE = (0.01, 0.1)


@dataclass
class Workload:
    """One lattice of a workload: everything the problem statement needs."""
    name: str
    lattice: str                 # "D2Q9" | "D3Q19"
    nx: int
    ny: int
    nz: int
    masses: List[float]          # molar masses, ascending
    diff: List[List[float]]      # symmetric pair diffusivities, lattice units
    tau1: float
    g: List[float]               # specific force (x, y, z)
    walls: List[bool]            # impermeable walls at both ends, per axis
    steps: int
    x0_kind: str                 # how x0() lays out the initial composition
    seed: int = 0
    x0_args: dict = field(default_factory=dict)
    n0: Optional[float] = None
    forcing: str = "standard"    # "standard"; "diff": plus the diffusion-driven term;
                                 # "full": the whole corrected forcing
    wall_velocity: Optional[List[List[float]]] = None   # [low, high] wall velocities
    wall_kind: str = "appendix_a"   # or "equilibrium": the comparison boundary of Sec. 4.1

    @property
    def n_species(self):
        return len(self.masses)

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    def x0(self):
        """Initial mole fractions, float64 array [N, nz, ny, nx]."""
        return make_x0(self)


# ------------------------------------------------------------ x0 generators
def _halves(nx, ny, nz, xa, xb):
    N = len(xa)
    x = np.empty((N, nz, ny, nx))
    h = nx // 2
    for s in range(N):
        x[s, :, :, :h] = xa[s]
        x[s, :, :, h:] = xb[s]
    return x


def _step(nx, ny, nz, split):
    x = np.zeros((2, nz, ny, nx))
    x[0, :, :, :split] = 1.0
    x[1, :, :, split:] = 1.0
    return x


def _layer(nx, ny, nz, z_split, dense, carrier, seed, amp):
    N = len(dense)
    x = np.empty((N, nz, ny, nx))
    for s in range(N):
        x[s, :z_split] = carrier[s]
        x[s, z_split:] = dense[s]
    rng = np.random.default_rng(seed)
    x *= 1.0 + amp * rng.uniform(-1.0, 1.0, size=x.shape)
    x /= x.sum(axis=0, keepdims=True)
    return x


def _random(nx, ny, nz, n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.05, 1.0, size=(n, nz, ny, nx))
    return x / x.sum(axis=0, keepdims=True)


def make_x0(w):
    a = w.x0_args
    if w.x0_kind == "halves":
        return _halves(w.nx, w.ny, w.nz, a.get("xa", GAS_A), a.get("xb", GAS_B))
    if w.x0_kind == "step":
        return _step(w.nx, w.ny, w.nz, a["split"])
    if w.x0_kind == "layer":
        return _layer(w.nx, w.ny, w.nz, a["z_split"], a.get("dense", LAYER_DENSE),
                      a.get("carrier", LAYER_CARRIER), w.seed, a.get("amp", 0.01))
    if w.x0_kind == "random":
        return _random(w.nx, w.ny, w.nz, w.n_species, a.get("seed", w.seed))
    if w.x0_kind == "given":
        return np.asarray(a["x"], dtype=float)
    raise ValueError(w.x0_kind)


# ------------------------------------------------------------ random draws
def diffusivity_candidates(seed, n_species, count):
    """Successive candidate draws D_ij ~ U[0.01, 0.1] for the pairs i < j
    (row-major), from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    npair = n_species * (n_species - 1) // 2
    for _ in range(count):
        yield list(rng.uniform(D_RANGE[0], D_RANGE[1], size=npair))


def pairs_to_matrix(vals, n):
    D = [[0.0] * n for _ in range(n)]
    k = 0
    for i in range(n):
        for j in range(i + 1, n):
            D[i][j] = D[j][i] = float(vals[k])
            k += 1
    return D


def batched_tube_geometry(seed=3, count=512):
    """Geometry, masses and gravity of the batched tubes: nx ~ U{128..2048},
    ny ~ U{16..64}, M = (1, M_2, M_3) with M_2 ~ U[2, 16], M_3 ~ U[M_2, 25],
    g_x ~ U[0, 2e-6]."""
    rng = np.random.default_rng(seed)
    tubes = []
    for t in range(count):
        nx = int(rng.integers(128, 2049))
        ny = int(rng.integers(16, 65))
        m2 = float(rng.uniform(2.0, 16.0))
        m3 = float(rng.uniform(m2, 25.0))
        gx = float(rng.uniform(0.0, 2e-6))
        tubes.append({"nx": nx, "ny": ny, "masses": [1.0, m2, m3], "g": [gx, 0.0, 0.0]})
    return tubes


def composition_segment(xa, xb, points=41):
    """Compositions on the straight segment between two mixtures."""
    xa, xb = np.asarray(xa, float), np.asarray(xb, float)
    return [tuple((1 - t) * xa + t * xb) for t in np.linspace(0.0, 1.0, points)]


# ------------------------------------------------------------ workloads
def load_accepted():
    if not os.path.exists(ACCEPTED_PATH):
        raise FileNotFoundError(
            f"{ACCEPTED_PATH} missing: run `python -m oracle.make_workloads`")
    with open(ACCEPTED_PATH) as fh:
        return json.load(fh)


def binary_erf(nx=200, ny=4, steps=2000):
    """Binary Loschmidt tube, equal masses, x_1 = 1 | 0 at the midpoint,
    D_12 = 0.05, tau = 1, walls at the x ends, periodic in y, no force."""
    return Workload("binary_erf_200x4", "D2Q9", nx, ny, 1, [1.0, 1.0],
                    [[0.0, 0.05], [0.05, 0.0]], 1.0, [0.0, 0.0, 0.0],
                    [True, False, False], steps, "step", x0_args={"split": nx // 2})


def ternary_gravity(nx=1024, ny=64, steps=20000, name=None):
    """Ternary tube, masses 2:28:44, g = +1e-6 along x, walls at the x ends,
    periodic in y, halves of gas A (x < nx/2) and gas B, tau_1 = 1,
    diffusivities drawn from seed 1."""
    acc = load_accepted()["ternary_gravity"]
    return Workload(name or f"ternary_gravity_{nx}x{ny}", "D2Q9", nx, ny, 1,
                    [2.0, 28.0, 44.0], pairs_to_matrix(acc["pairs"], 3), 1.0,
                    [1e-6, 0.0, 0.0], [True, False, False], steps, "halves", seed=1)


def layer_mixing_3d(nx=256, ny=128, nz=128, steps=5000, z_split=None):
    """D3Q19, 4 species with masses 1:2:3:4, walls at z = 0 and nz-1, periodic
    in x and y, g = 1e-6 along -z, dense layer on top of a light carrier with a
    seeded 1 % perturbation of the mole fractions, diffusivities from seed 2."""
    acc = load_accepted()["layer_mixing_3d"]
    zs = (3 * nz) // 4 if z_split is None else z_split
    return Workload(f"layer_mixing_3d_{nx}x{ny}x{nz}", "D3Q19", nx, ny, nz,
                    [1.0, 2.0, 3.0, 4.0], pairs_to_matrix(acc["pairs"], 4), 1.0,
                    [0.0, 0.0, -1e-6], [False, False, True], steps, "layer", seed=2,
                    x0_args={"z_split": zs})


def batched_tubes(count=512, steps=10000):
    """The batched workload: `count` independent ternary tubes with their own
    geometry, masses, gravity and diffusivities (seed 3)."""
    acc = load_accepted()["batched_tubes"]
    geo = batched_tube_geometry(3, 512)[:count]
    out = []
    for t, (gm, ac) in enumerate(zip(geo, acc["tubes"][:count])):
        out.append(Workload(f"tube{t}", "D2Q9", gm["nx"], gm["ny"], 1, gm["masses"],
                            pairs_to_matrix(ac["pairs"], 3), 1.0, gm["g"],
                            [True, False, False], steps, "halves", seed=3))
    return out


def concat_x0(workloads):
    """Initial mole fractions of a batch, flattened lattice after lattice in the
    [lattice][species][z][y][x] order the batched interface expects."""
    return np.concatenate([w.x0().reshape(-1) for w in workloads])


def adjoint_tube(nx=512, ny=64, steps=4000):
    """Adjoint workload: ternary tube 2:28:44, walls at the x ends, g = 1e-6;
    the true diffusivities come from seed 4, the evaluation point perturbs
    them by (1 + 0.2 U[-1, 1]) and uses g = 1.2e-6."""
    acc = load_accepted()["adjoint_tube"]
    truth = Workload(f"adjoint_tube_{nx}x{ny}", "D2Q9", nx, ny, 1, [2.0, 28.0, 44.0],
                     pairs_to_matrix(acc["pairs"], 3), 1.0, [1e-6, 0.0, 0.0],
                     [True, False, False], steps, "halves", seed=4)
    rng = np.random.default_rng(4)
    fac = rng.uniform(-1.0, 1.0, size=3)
    pert = [p * (1.0 + 0.2 * f) for p, f in zip(acc["pairs"], fac)]
    evalp = Workload(truth.name + "_eval", "D2Q9", nx, ny, 1, [2.0, 28.0, 44.0],
                     pairs_to_matrix(pert, 3), 1.0, [1.2e-6, 0.0, 0.0],
                     [True, False, False], steps, "halves", seed=4)
    return truth, evalp
