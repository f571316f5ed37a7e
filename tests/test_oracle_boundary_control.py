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


def _box(lattice, masses, shape, walls):
    D = torch.full((len(masses), len(masses)), 0.05, dtype=DTYPE)
    return evd.Model(lattice, *shape, masses, D, 1.0, walls=walls)


@pytest.mark.parametrize("lattice,shape,walls", [("D2Q9", (5, 4, 1), (True, True, False)),
                                                 ("D2Q9", (4, 3, 1), (False, True, False)),
                                                 ("D3Q19", (3, 4, 3), (True, False, True))])
def test_equilibrium_boundary_at_unit_speed_is_a_shift_from_equilibrium_solids(lattice, shape,
                                                                               walls):
    """Equal masses: every species moves at c = 1, so the stream is an exact
    shift, f_a(O) = f~_a(O - c_a), and a source beyond a wall gives
    w_a rho_s with rho_s the density of the node facing it (the source's
    coordinates clamped into the lattice)."""
    m = _box(lattice, [2.0, 2.0], shape, walls)
    lat = m.lat
    gen = torch.Generator().manual_seed(4)
    ft = torch.rand(m.N, lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)
    got = evd.stream_equilibrium_walls(m, ft)
    rho = ft.sum(dim=1)
    dims = (m.nx, m.ny, m.nz)
    for i in range(m.N):
        for a in range(lat.Q):
            for z in range(m.nz):
                for y in range(m.ny):
                    for x in range(m.nx):
                        src = [(x, y, z)[d] - lat.dirs[a][d] for d in range(3)]
                        solid = False
                        for d in range(3):
                            if walls[d] and not 0 <= src[d] < dims[d]:
                                solid = True
                                src[d] = min(max(src[d], 0), dims[d] - 1)
                            else:
                                src[d] %= dims[d]
                        sx, sy, sz = src
                        want = (lat.w[a] * rho[i, sz, sy, sx] if solid
                                else ft[i, a, sz, sy, sx])
                        assert abs(got[i, a, z, y, x] - want) < 1e-15


@pytest.mark.parametrize("lattice,shape,walls", [("D2Q9", (4, 5, 1), (True, True, False)),
                                                 ("D3Q19", (3, 3, 4), (False, True, True))])
def test_equilibrium_boundary_equals_brute_force_interpolation(lattice, shape, walls):
    """Species slower than c = 1, node by node: f_a(O) = sum over source
    offsets k in {-1,0,1}^d of prod_d lambda_{k_d}(c e_{a,d}) times f~_a(O+k),
    or w_a rho_s at a solid source, with lambda_-1(s) = s(1+s)/2,
    lambda_0(s) = 1 - s^2, lambda_+1(s) = -s(1-s)/2 (eq.
    Second_order_spatial_interpolation)."""
    m = _box(lattice, [1.0, 3.0, 7.0], shape, walls)
    lat = m.lat
    gen = torch.Generator().manual_seed(5)
    ft = torch.rand(m.N, lat.Q, m.nz, m.ny, m.nx, generator=gen, dtype=DTYPE)
    got = evd.stream_equilibrium_walls(m, ft)
    rho = ft.sum(dim=1)
    dims = (m.nx, m.ny, m.nz)
    offs = [-1, 0, 1]

    def lam(k, s):
        return {-1: s * (1 + s) / 2, 0: 1 - s * s, 1: -s * (1 - s) / 2}[k]

    for i in range(m.N):
        c = (1.0 / m.M[i]) ** 0.5
        for a in range(lat.Q):
            for z in range(m.nz):
                for y in range(m.ny):
                    for x in range(m.nx):
                        acc = 0.0
                        for kz in (offs if lat.dim == 3 else [0]):
                            for ky in offs:
                                for kx in offs:
                                    k = (kx, ky, kz)
                                    wgt = 1.0
                                    for d in range(3):
                                        wgt *= lam(k[d], c * lat.dirs[a][d])
                                    if wgt == 0.0:
                                        continue
                                    src = [(x, y, z)[d] + k[d] for d in range(3)]
                                    solid = False
                                    for d in range(3):
                                        if walls[d] and not 0 <= src[d] < dims[d]:
                                            solid = True
                                            src[d] = min(max(src[d], 0), dims[d] - 1)
                                        else:
                                            src[d] %= dims[d]
                                    sx, sy, sz = src
                                    v = (lat.w[a] * rho[i, sz, sy, sx] if solid
                                         else ft[i, a, sz, sy, sx])
                                    acc += wgt * float(v)
                        assert abs(float(got[i, a, z, y, x]) - acc) < 1e-14
