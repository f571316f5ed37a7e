"""Pins of the oracle's wall rule where walls on several axes meet (reading
R11: edges and corners, which Appendix A, written for single walls, does not
cover).  What fixes it: every source keeps its whole weight (species mass is
exact in closed boxes for any state), at c = 1 the stream is a permutation
with halfway bounce-back into the corner, and a closed box at rest stays at
rest at c = 1.  The reduction to the single-wall formulas is pinned by the stream
tests, which run through the same rule."""
import pytest
import torch

from oracle import evd
from oracle.lattice import DTYPE


def _box(lattice, masses, shape, walls):
    D = torch.full((len(masses), len(masses)), 0.05, dtype=DTYPE)
    return evd.Model(lattice, *shape, masses, D, 1.0, walls=walls)


BOXES = [("D2Q9", (5, 4, 1), (True, True, False)),
         ("D2Q9", (2, 3, 1), (True, True, False)),
         ("D3Q19", (4, 3, 5), (True, True, True)),
         ("D3Q19", (3, 4, 3), (True, False, True)),
         ("D3Q19", (3, 3, 4), (False, True, True))]


@pytest.mark.parametrize("lattice,shape,walls", BOXES)
def test_stream_conserves_every_species_in_closed_boxes(lattice, shape, walls):
    m = _box(lattice, [1.0, 3.0, 7.0], shape, walls)
    gen = torch.Generator().manual_seed(1)
    for _ in range(3):
        ft = torch.rand(m.N, m.lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)
        out = evd.stream(m, ft)
        d = (out.sum(dim=(1, 2, 3, 4)) - ft.sum(dim=(1, 2, 3, 4))).abs()
        assert d.max() < 1e-13 * ft.sum()


@pytest.mark.parametrize("lattice,shape,walls", BOXES)
def test_unit_speed_stream_is_a_permutation_with_corner_bounce_back(lattice, shape, walls):
    """Equal masses: every species moves at c = 1, the stream is an exact
    shift plus halfway bounce-back, hence a permutation of the values."""
    m = _box(lattice, [1.0, 1.0], shape, walls)
    gen = torch.Generator().manual_seed(2)
    ft = torch.rand(m.N, m.lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)
    out = evd.stream(m, ft)
    for i in range(m.N):
        assert torch.equal(torch.sort(out[i].flatten()).values, torch.sort(ft[i].flatten()).values)
    # the population moving into the (0, 0, 0) corner comes back reversed
    lat = m.lat
    dvec = tuple(-1 if walls[a] else 0 for a in range(3))
    if lattice == "D2Q9":
        dvec = (dvec[0], dvec[1], 0)
    if dvec in lat.dirs and sum(abs(v) for v in dvec) > 1:
        b = lat.dirs.index(dvec)
        assert out[0, lat.opp[b], 0, 0, 0] == ft[0, b, 0, 0, 0]


@pytest.mark.parametrize("lattice,shape,walls", BOXES[:3])
def test_closed_box_at_rest_stays_at_rest_at_unit_speed(lattice, shape, walls):
    """Equal masses (c = 1: halfway bounce-back everywhere, corners included):
    a closed box at rest stays at rest.  (For c < 1 the Appendix A rule
    itself does not keep a rest state exactly in the wall layer, with one
    wall as with several.)"""
    m = _box(lattice, [1.0, 1.0], shape, walls)
    x = torch.tensor([0.4, 0.6], dtype=DTYPE)[:, None, None, None].expand(2, m.nz, m.ny, m.nx)
    f = evd.initial_populations(m, x.clone())
    g = evd.step(m, f)
    assert (g - f).abs().max() < 1e-15


@pytest.mark.parametrize("lattice,shape,walls", BOXES)
def test_per_direction_closed_form_equals_the_sum_over_crossed_wall_sets(lattice, shape, walls):
    """The kernel evaluates the rule per direction a in closed form: with
    n_away walls of the node that a points away from and n_tow that it points
    toward, f_a gains (1 - (1 - l+)^n_away)(1 - l-)^n_tow f~_a
    + (1 - (1 - l-)^n_away) f~_abar (l+- = lambda_{+-1}(c), the Lagrange weights
    of the node beyond and behind for Courant number c).  Checked here against
    the oracle's sum over the sets of crossed walls at every node of a box,
    for species of three speeds."""
    m = _box(lattice, [1.0, 3.0, 7.0], shape, walls)
    lat = m.lat
    e = m.velocities()
    lam = [[[evd.lagrange_weights(float(e[i, al, a])) for a in range(3)]
            for al in range(lat.Q)] for i in range(m.N)]
    walled = [a for a in range(3) if walls[a]]
    gen = torch.Generator().manual_seed(3)
    ft = torch.rand(m.N, lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)
    got = evd._wall_returns(m, ft, lam, walled)
    want = torch.zeros_like(ft)
    dims = (m.nx, m.ny, m.nz)
    for i in range(m.N):
        c = max(abs(float(v)) for v in e[i].flatten())
        lm, _, lp = evd.lagrange_weights(c)      # l- = lambda_-1(c), l+ = lambda_+1(c)
        for z in range(m.nz):
            for y in range(m.ny):
                for x in range(m.nx):
                    pos = (x, y, z)
                    side = [0, 0, 0]
                    for a in walled:
                        side[a] = -1 if pos[a] == 0 else (1 if pos[a] == dims[a] - 1 else 0)
                    for a in range(1, lat.Q):
                        na = sum(1 for k in range(3) if side[k] * lat.dirs[a][k] < 0)
                        nt = sum(1 for k in range(3) if side[k] * lat.dirs[a][k] > 0)
                        if na == 0:
                            continue
                        c1 = (1 - (1 - lp) ** na) * (1 - lm) ** nt
                        c2 = 1 - (1 - lm) ** na
                        want[i, a, z, y, x] = (c1 * ft[i, a, z, y, x]
                                               + c2 * ft[i, lat.opp[a], z, y, x])
    assert (got - want).abs().max() < 1e-15
