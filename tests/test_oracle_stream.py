"""Pins of the oracle's streaming (second-order interpolation) and of the
impermeable-wall scheme, against the formulas the paper prints and against
exact properties (mass conservation, polynomial exactness, bounce-back)."""
import itertools

import numpy as np
import pytest
import torch

from oracle import evd
from oracle.lattice import DTYPE


def _model(lattice="D2Q9", shape=(6, 5, 1), masses=(1.0, 3.0), walls=(False, False, False)):
    N = len(masses)
    D = torch.full((N, N), 0.05, dtype=DTYPE)
    return evd.Model(lattice, *shape, list(masses), D, 1.0, walls=walls)


def _rand(m, seed=0):
    gen = torch.Generator().manual_seed(seed)
    return torch.rand(m.N, m.lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)


CASES = [
    ("D2Q9", (6, 5, 1), (True, False, False)),
    ("D2Q9", (6, 5, 1), (False, True, False)),
    ("D2Q9", (6, 5, 1), (False, False, False)),
    ("D3Q19", (4, 3, 5), (False, False, True)),
    ("D3Q19", (4, 5, 3), (True, False, False)),
    ("D3Q19", (3, 3, 3), (False, False, False)),
]


@pytest.mark.parametrize("lattice,shape,walls", CASES)
def test_stream_conserves_every_population(lattice, shape, walls):
    """Appendix A: with the proposed wall scheme the information of every
    streamed population is used exactly once, i.e. every column of the linear
    stream+wall operator sums to one (per species, so mass is conserved).
    Checked by streaming each unit population separately."""
    m = _model(lattice, shape, masses=(1.0, 2.7), walls=walls)
    ft = torch.zeros(m.N, m.lat.Q, m.nz, m.ny, m.nx, dtype=DTYPE)
    worst = 0.0
    for idx in itertools.product(range(m.N), range(m.lat.Q), range(m.nz), range(m.ny),
                                 range(m.nx)):
        ft[idx] = 1.0
        out = evd.stream(m, ft)
        ft[idx] = 0.0
        # nothing leaks to another species
        s = idx[0]
        assert out[[i for i in range(m.N) if i != s]].abs().sum() == 0
        worst = max(worst, abs(out[s].sum().item() - 1.0))
    assert worst < 1e-14


@pytest.mark.parametrize("lattice,shape,walls", CASES)
def test_unit_speed_is_shift_plus_halfway_bounce_back(lattice, shape, walls):
    """c_i = 1 (equal masses): the interpolation is the exact shift
    f(O) = f~(O - e) and the wall scheme collapses to the halfway bounce-back
    f_alphabar(x, t+1) = f~_alpha(x, t), eq. (standard_BBscheme) (Appendix A,
    last paragraph)."""
    m = _model(lattice, shape, masses=(1.0, 1.0), walls=walls)
    ft = _rand(m, 1)
    out = evd.stream(m, ft)
    n = (m.nx, m.ny, m.nz)
    want = torch.zeros_like(ft)
    for s, al in itertools.product(range(m.N), range(m.lat.Q)):
        c = m.lat.dirs[al]
        for z, y, x in itertools.product(range(m.nz), range(m.ny), range(m.nx)):
            src = [x - c[0], y - c[1], z - c[2]]
            solid = False
            for a in range(3):
                if walls[a] and not (0 <= src[a] < n[a]):
                    solid = True
                src[a] %= n[a]
            if solid:
                want[s, al, z, y, x] = ft[s, m.lat.opp[al], z, y, x]
            else:
                want[s, al, z, y, x] = ft[s, al, src[2], src[1], src[0]]
    assert torch.equal(out, want)


# --------------------------------------------------------- paper formulas
def _labels(ft, s, al, z, y, x, nx, ny):
    """Post-collision values at O and its eight neighbours, labelled as in
    eq. (Second_order_spatial_interpolation) under reading R1 (source offsets
    A=(+1,0) B=(0,+1) C=(-1,0) D=(0,-1) E=(+1,+1) F=(-1,+1) G=(-1,-1) H=(+1,-1)).
    Out-of-range neighbours are returned as NaN so that using one fails."""
    off = {"O": (0, 0), "A": (1, 0), "B": (0, 1), "C": (-1, 0), "D": (0, -1),
           "E": (1, 1), "F": (-1, 1), "G": (-1, -1), "H": (1, -1)}
    out = {}
    for k, (dx, dy) in off.items():
        xx, yy = x + dx, y + dy
        if 0 <= xx < nx and 0 <= yy < ny:
            out[k] = float(ft[s, al, z, yy, xx])
        else:
            out[k] = float("nan")
    return out


def _paper_interior(L, xi, eta):
    """eq. (Second_order_spatial_interpolation), term by term."""
    return ((1 - eta**2) * (1 - xi**2) * L["O"] + xi * (1 - eta**2) * (1 + xi) / 2 * L["C"]
            + eta * (1 + eta) * (1 - xi**2) / 2 * L["D"]
            + eta * xi * (1 + eta) * (1 + xi) / 4 * L["G"]
            - xi * (1 - xi) * (1 - eta**2) / 2 * L["A"]
            - eta * (1 - eta) * (1 - xi**2) / 2 * L["B"]
            - eta * xi * (1 + xi) * (1 - eta) / 4 * L["F"]
            - eta * xi * (1 - xi) * (1 + eta) / 4 * L["H"]
            + eta * xi * (1 - xi) * (1 - eta) / 4 * L["E"])


def test_interior_matches_paper_nine_point_formula():
    m = _model("D2Q9", (7, 6, 1), masses=(1.0, 5.0, 17.0))
    ft = _rand(m, 2)
    out = evd.stream(m, ft)
    e = m.velocities()
    for s, al in itertools.product(range(m.N), range(9)):
        xi, eta = float(e[s, al, 0]), float(e[s, al, 1])
        for y in range(1, m.ny - 1):
            for x in range(1, m.nx - 1):
                L = _labels(ft, s, al, 0, y, x, m.nx, m.ny)
                assert abs(out[s, al, 0, y, x].item() - _paper_interior(L, xi, eta)) < 1e-14


def _paper_wall(wall, al, e, Lf):
    """The wall formulas of Appendix A for the directions they are given for.
    Lf[alpha] are the labelled neighbour values of direction alpha.  e[alpha]
    = (xi_alpha, eta_alpha).  Returns None for directions not listed."""
    xi, eta = e[al]
    L = Lf[al]
    opp = {1: 3, 2: 4, 3: 1, 4: 2, 5: 7, 6: 8, 7: 5, 8: 6}
    xi1 = e[1][0]
    eta2 = e[2][1]
    if wall == "right":
        if al == 3:
            return (Lf[3]["O"] + xi1**2 / 2 * (Lf[1]["O"] + Lf[3]["C"] - Lf[3]["O"])
                    + xi1 / 2 * (Lf[1]["O"] - Lf[3]["C"] - Lf[3]["O"]))
        if al in (6, 7):
            return (((1 - eta**2) * (1 - xi**2) + xi * (1 + xi) / 2) * L["O"]
                    + xi * (1 + xi) * (1 - eta**2) / 2 * L["C"]
                    + eta * (1 + eta) * (1 - xi**2) / 2 * L["D"]
                    + eta * xi * (1 + eta) * (1 + xi) / 4 * L["G"]
                    - eta * (1 - eta) * (1 - xi**2) / 2 * L["B"]
                    - eta * xi * (1 + xi) * (1 - eta) / 4 * L["F"]
                    - xi * (1 - xi) / 2 * Lf[opp[al]]["O"])
    if wall == "left":
        if al == 1:
            return (Lf[1]["O"] + xi1**2 / 2 * (Lf[3]["O"] + Lf[1]["A"] - Lf[1]["O"])
                    + xi1 / 2 * (Lf[3]["O"] - Lf[1]["A"] - Lf[1]["O"]))
        if al in (5, 8):
            return (((1 - eta**2) * (1 - xi**2) - xi * (1 - xi) / 2) * L["O"]
                    - xi * (1 - xi) * (1 - eta**2) / 2 * L["A"]
                    - eta * (1 - eta) * (1 - xi**2) / 2 * L["B"]
                    + eta * (1 + eta) * (1 - xi**2) / 2 * L["D"]
                    - eta * xi * (1 - xi) * (1 + eta) / 4 * L["H"]
                    + eta * xi * (1 - xi) * (1 - eta) / 4 * L["E"]
                    + xi * (1 + xi) / 2 * Lf[opp[al]]["O"])
    if wall == "upper":
        if al == 4:
            return (Lf[4]["O"] + eta2**2 / 2 * (Lf[2]["O"] + Lf[4]["D"] - Lf[4]["O"])
                    + eta2 / 2 * (Lf[2]["O"] - Lf[4]["D"] - Lf[4]["O"]))
        if al in (7, 8):
            return (((1 - eta**2) * (1 - xi**2) + eta * (1 + eta) / 2) * L["O"]
                    + eta * (1 - xi**2) * (1 + eta) / 2 * L["D"]
                    + xi * (1 + xi) * (1 - eta**2) / 2 * L["C"]
                    - xi * (1 - xi) * (1 - eta**2) / 2 * L["A"]
                    + eta * xi * (1 + eta) * (1 + xi) / 4 * L["G"]
                    - eta * xi * (1 - xi) * (1 + eta) / 4 * L["H"]
                    - eta * (1 - eta) / 2 * Lf[opp[al]]["O"])
    if wall == "bottom":
        if al == 2:
            return (Lf[2]["O"] + eta2**2 / 2 * (Lf[4]["O"] + Lf[2]["B"] - Lf[2]["O"])
                    + eta2 / 2 * (Lf[4]["O"] - Lf[2]["B"] - Lf[2]["O"]))
        if al in (5, 6):
            return (((1 - eta**2) * (1 - xi**2) - eta * (1 - eta) / 2) * L["O"]
                    + xi * (1 - eta**2) * (1 + xi) / 2 * L["C"]
                    - xi * (1 - xi) * (1 - eta**2) / 2 * L["A"]
                    - eta * (1 - eta) * (1 - xi**2) / 2 * L["B"]
                    - eta * xi * (1 + xi) * (1 - eta) / 4 * L["F"]
                    + eta * xi * (1 - xi) * (1 - eta) / 4 * L["E"]
                    + eta * (1 + eta) / 2 * Lf[opp[al]]["O"])
    return None


@pytest.mark.parametrize("wall", ["right", "left", "upper", "bottom"])
def test_wall_matches_paper_appendix_formulas(wall):
    """The eight wall formulas printed in Appendix A (right wall: alpha = 3 and
    alpha = 6, 7; left: 1 and 5, 8; upper: 4 and 7, 8; bottom: 2 and 5, 6).
    For the other directions at a wall node the interpolation simply loses its
    solid sources (Appendix A, the near-wall redistribution equation): the
    nine-point formula with the solid labels removed."""
    walls = (True, False, False) if wall in ("right", "left") else (False, True, False)
    m = _model("D2Q9", (6, 6, 1), masses=(1.0, 2.5, 9.0), walls=walls)
    ft = _rand(m, 3)
    out = evd.stream(m, ft)
    e = m.velocities()
    if wall == "right":
        nodes = [(m.nx - 1, y) for y in range(m.ny)]
        solid = {"A", "E", "H"}
    elif wall == "left":
        nodes = [(0, y) for y in range(m.ny)]
        solid = {"C", "F", "G"}
    elif wall == "upper":
        nodes = [(x, m.ny - 1) for x in range(m.nx)]
        solid = {"B", "E", "F"}
    else:
        nodes = [(x, 0) for x in range(m.nx)]
        solid = {"D", "G", "H"}
    checked = 0
    for s in range(m.N):
        ev = {al: (float(e[s, al, 0]), float(e[s, al, 1])) for al in range(9)}
        for (x, y) in nodes:
            # periodic neighbours along the wall: emulate by rolling the data
            roll = [0, 0]
            if walls[0]:
                roll[1] = (m.ny // 2) - y
            else:
                roll[0] = (m.nx // 2) - x
            ftr = torch.roll(ft, shifts=(roll[1], roll[0]), dims=(-2, -1))
            xr, yr = (x + roll[0]) % m.nx, (y + roll[1]) % m.ny
            Lf = {al: _labels(ftr, s, al, 0, yr, xr, m.nx, m.ny) for al in range(9)}
            for al in range(9):
                got = out[s, al, 0, y, x].item()
                want = _paper_wall(wall, al, ev, Lf)
                if want is None:
                    L = {k: (0.0 if k in solid else v) for k, v in Lf[al].items()}
                    want = _paper_interior(L, *ev[al])
                else:
                    checked += 1
                assert abs(got - want) < 1e-14, (wall, s, al, x, y, got, want)
    assert checked == m.N * len(nodes) * 3


# -------------------------------------------------------- exact properties
@pytest.mark.parametrize("lattice", ["D2Q9", "D3Q19"])
def test_interpolation_reproduces_quadratics(lattice):
    """Quadratic Lagrange interpolation is exact for quadratic data: away from
    the periodic seam, f(O) = p(O - e) for f~ = p quadratic."""
    shape = (8, 7, 1) if lattice == "D2Q9" else (6, 6, 6)
    m = _model(lattice, shape, masses=(1.0, 2.2, 7.0))
    z, y, x = torch.meshgrid(torch.arange(m.nz, dtype=DTYPE), torch.arange(m.ny, dtype=DTYPE),
                             torch.arange(m.nx, dtype=DTYPE), indexing="ij")

    def p(x, y, z):
        return 0.3 + 0.1 * x - 0.05 * y + 0.02 * z + 0.01 * x * x - 0.02 * x * y \
            + 0.015 * y * y + 0.01 * x * z - 0.004 * z * z + 0.003 * y * z

    ft = p(x, y, z)[None, None].expand(m.N, m.lat.Q, m.nz, m.ny, m.nx).clone()
    out = evd.stream(m, ft)
    e = m.velocities()
    lo = 1
    sl = (slice(lo, m.nz - 1) if m.nz > 1 else slice(None), slice(lo, m.ny - 1),
          slice(lo, m.nx - 1))
    for s in range(m.N):
        for al in range(m.lat.Q):
            ex, ey, ez = (float(v) for v in e[s, al])
            want = p(x - ex, y - ey, z - ez)
            assert torch.allclose(out[s, al][sl], want[sl], atol=1e-14, rtol=0)


def test_y_uniform_state_reduces_to_one_row():
    """Translation invariance: a state uniform along a periodic y axis stays
    uniform, and a one-row lattice (ny = 1, periodic) gives the same result.
    The long parity runs of the tube workloads rely on this."""
    D = torch.tensor([[0, .05, .08], [.05, 0, .03], [.08, .03, 0]], dtype=DTYPE)
    m4 = evd.Model("D2Q9", 12, 4, 1, [1.0, 6.0, 11.0], D, 1.0, g=[1e-4, 0, 0],
                   walls=(True, False, False))
    m1 = evd.Model("D2Q9", 12, 1, 1, [1.0, 6.0, 11.0], D, 1.0, g=[1e-4, 0, 0],
                   walls=(True, False, False))
    x = torch.rand(3, 1, 1, 12, dtype=DTYPE) + 0.1
    x = x / x.sum(0)
    f4 = evd.run(m4, evd.initial_populations(m4, x.expand(3, 1, 4, 12)), 30)
    f1 = evd.run(m1, evd.initial_populations(m1, x), 30)
    assert torch.allclose(f4, f1.expand_as(f4), atol=1e-15, rtol=0)
