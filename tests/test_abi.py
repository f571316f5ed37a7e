"""CPU tests of the C-ABI library: it loads, exports every entry point the
header declares, its struct layout matches the C compiler's, and the host-side
validation and stability pre-check behave as documented.  No kernel runs."""
import ctypes
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import evd, stability

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm_mc.h")


def _lib():
    from paper_2504_07059_amd import _lib
    return _lib


def test_library_exports_every_declared_entry_point():
    """Every lbm_mc_* function declared in any header under include/."""
    import glob
    L = _lib()
    cdll = ctypes.CDLL(L.LIB_PATH)
    total = 0
    for h in sorted(glob.glob(os.path.join(ROOT, "include", "*.h"))):
        names = set(re.findall(r"\b(lbm_mc_[a-z_]+)\s*\(", open(h).read()))
        total += len(names)
        for n in sorted(names):
            assert hasattr(cdll, n), f"{n} declared in {os.path.basename(h)} but not exported"
    assert total >= 18


def test_params_struct_layout_matches_c():
    L = _lib()
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "lbm_mc.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(lbm_mc_params),
         offsetof(lbm_mc_params, molar_mass), offsetof(lbm_mc_params, diff),
         offsetof(lbm_mc_params, tau1), offsetof(lbm_mc_params, g),
         offsetof(lbm_mc_params, n0), offsetof(lbm_mc_params, forcing),
         offsetof(lbm_mc_params, wall_velocity));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                               check=True).stdout.split()]
    P = L.Params
    assert vals == [ctypes.sizeof(P), P.molar_mass.offset, P.diff.offset, P.tau1.offset,
                    P.g.offset, P.n0.offset, P.forcing.offset, P.wall_velocity.offset]


def _tube(nx=64, ny=4, N=3, **kw):
    from paper_2504_07059_amd.lbm import make_params
    masses = [2.0, 28.0, 44.0, 60.0][:N]
    acc = W.load_accepted()["ternary_gravity"]["pairs"]
    D = W.pairs_to_matrix(acc, 3) if N == 3 else [[0.05 * (i != j) for j in range(N)]
                                                  for i in range(N)]
    args = dict(lattice="D2Q9", nx=nx, ny=ny, nz=1, masses=masses, diff=D, tau1=1.0,
                g=(1e-6, 0, 0), walls=(True, False, False))
    args.update(kw)
    return make_params(**args)


def _x0(p, comp=W.GAS_B + (0.0,)):
    N = p.n_species
    nodes = p.nx * p.ny * p.nz
    x = np.zeros((N, nodes))
    c = np.array(comp[:N], dtype=float)
    c = c / c.sum()
    x[:] = c[:, None]
    return x


def test_check_accepts_valid_problem_and_layout():
    from paper_2504_07059_amd.lbm import check_problem, layout
    p = _tube()
    st, lam, msg = check_problem(p, _x0(p))
    assert st == 0, msg
    assert 0 < lam < 2
    total, offs, pitch, fields = layout(p)
    assert pitch == [64]
    assert total == 3 * 9 * 4 * 64
    assert offs == [0] and fields == [0]


@pytest.mark.parametrize("mutate,status", [
    (dict(tau1=0.5), 1),
    (dict(masses=[28.0, 2.0, 44.0]), 1),
    (dict(walls=(True, True, False), wall_velocity=[[0, 0.01, 0], [0, 0, 0]]), 2),
    (dict(lattice="D2Q9", nz=2), 1),
    (dict(nx=1), 1),
])
def test_check_rejects_invalid_problems(mutate, status):
    from paper_2504_07059_amd.lbm import check_problem
    p = _tube(**mutate)
    st, _, msg = check_problem(p, _x0(p))
    assert st == status, msg
    assert msg


def test_check_forcing_values():
    """forcing 0 (standard), 1 (plus S_diff) and 2 (the whole corrected
    forcing) are accepted, other values rejected; a batch must share one
    forcing."""
    from paper_2504_07059_amd.lbm import check_problem
    for forcing, status in ((0, 0), (1, 0), ("diff", 0), (2, 0), ("full", 0), (3, 1), (-1, 1)):
        p = _tube(forcing=forcing)
        st, _, msg = check_problem(p, _x0(p))
        assert st == status, (forcing, msg)
    a, b = _tube(forcing=0), _tube(forcing=1)
    st, _, msg = check_problem([a, b], np.concatenate([_x0(a), _x0(b)]))
    assert st == 1 and "forcing" in msg
    # the one-sided wall differences of forcing 2 need 3 nodes on the wall axis
    p = _tube(nx=2, forcing=2)
    st, _, msg = check_problem(p, _x0(p))
    assert st == 1 and "forcing 2" in msg
    p = _tube(nx=3, forcing=2)
    assert check_problem(p, _x0(p))[0] == 0


def test_check_rejects_bad_compositions_and_diffusivities():
    from paper_2504_07059_amd.lbm import check_problem
    p = _tube()
    x = _x0(p)
    x[0, 5] += 0.1
    st, _, msg = check_problem(p, x)
    assert st == 1 and "sum" in msg
    x = _x0(p)
    x[0, 3] = -1e-3
    x[1, 3] += 1e-3
    assert check_problem(p, x)[0] == 1
    p.diff[0][1] = 0.07          # not symmetric
    assert check_problem(p, _x0(p))[0] == 1
    p = _tube(N=2, masses=[1.0, 1.0], diff=[[0, -0.05], [-0.05, 0]])
    assert check_problem(p, _x0(p))[0] == 1


def test_stability_precheck_matches_oracle_and_rejects_unstable():
    """The library's eigenvalue of K agrees with the oracle's (independent
    implementations), and a draw with tiny D at composition A is UNSTABLE."""
    from paper_2504_07059_amd.lbm import check_problem, make_params
    D = [[0, 0.02, 0.011], [0.02, 0, 0.012], [0.011, 0.012, 0]]
    p = make_params("D2Q9", 8, 1, 1, [2.0, 28.0, 44.0], D, 1.0, walls=(True, False, False))
    x = np.array(W.GAS_A)[:, None].repeat(8, 1)
    st, lam, msg = check_problem(p, x)
    m = evd.Model("D2Q9", 4, 1, 1, [2.0, 28.0, 44.0], torch.tensor(D, dtype=torch.float64), 1.0)
    lo, hi = stability.eig_range(m, W.GAS_A)
    assert hi >= 2.0 and st == 4, (hi, st, msg)
    Dok = W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3)
    p = make_params("D2Q9", 8, 1, 1, [2.0, 28.0, 44.0], Dok, 1.0, walls=(True, False, False))
    x = np.array(W.GAS_B)[:, None].repeat(8, 1)
    st, lam, msg = check_problem(p, x)
    m = evd.Model("D2Q9", 4, 1, 1, [2.0, 28.0, 44.0], torch.tensor(Dok, dtype=torch.float64), 1.0)
    assert st == 0, msg
    # the library also samples towards the mean composition, which equals x here
    assert abs(lam - stability.eig_range(m, W.GAS_B)[1]) < 1e-12


def test_init_rejects_bad_buffers_before_touching_the_gpu():
    L = _lib()
    p = _tube()
    x = np.ascontiguousarray(_x0(p))
    arr = (L.Params * 1)(p)
    ctx = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    st = L.lib.lbm_mc_init(arr, 1, x.ctypes.data_as(dp), None, None, 10 ** 6, None,
                           ctypes.byref(ctx))
    assert st == 1 and not ctx.value
    st = L.lib.lbm_mc_init(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(4096),
                           ctypes.c_void_p(4096), 10 ** 6, None, ctypes.byref(ctx))
    assert st == 1 and b"distinct" in L.lib.lbm_mc_last_error()
    st = L.lib.lbm_mc_init(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(4096),
                           ctypes.c_void_p(8192), 10, None, ctypes.byref(ctx))
    assert st == 1 and b"floats" in L.lib.lbm_mc_last_error()
    assert L.lib.lbm_mc_step(None, 1) == 1
    assert L.lib.lbm_mc_prepare(None, 1) == 1
    assert L.lib.lbm_mc_destroy(None) == 0


def test_init_field_rejects_bad_arguments_before_touching_the_gpu():
    """lbm_mc_init_field: a NULL or misaligned force field, or a nonzero g
    beside it, is rejected before any device work."""
    L = _lib()
    dp = ctypes.POINTER(ctypes.c_double)
    ctx = ctypes.c_void_p()
    p = _tube(g=(0.0, 0.0, 0.0))
    x = np.ascontiguousarray(_x0(p))
    arr = (L.Params * 1)(p)
    st = L.lib.lbm_mc_init_field(arr, 1, x.ctypes.data_as(dp), None, ctypes.c_void_p(4096),
                                 ctypes.c_void_p(8192), 10 ** 6, None, ctypes.byref(ctx))
    assert st == 1 and b"accel" in L.lib.lbm_mc_last_error() and not ctx.value
    st = L.lib.lbm_mc_init_field(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(4098),
                                 ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10 ** 6, None,
                                 ctypes.byref(ctx))
    assert st == 1 and b"aligned" in L.lib.lbm_mc_last_error()
    q = _tube(g=(1e-6, 0.0, 0.0))
    arr = (L.Params * 1)(q)
    st = L.lib.lbm_mc_init_field(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(1 << 20),
                                 ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10 ** 6, None,
                                 ctypes.byref(ctx))
    assert st == 1 and b"g must be 0" in L.lib.lbm_mc_last_error()


def test_check_wall_velocities():
    """Wall velocities must be finite, tangential, on a lattice with a wall
    axis, with no z component in 2-D; a force field with moving walls is
    rejected before any device work."""
    from paper_2504_07059_amd.lbm import check_problem
    p = _tube(wall_velocity=[[0, 0.01, 0], [0, -0.02, 0]])
    assert check_problem(p, _x0(p))[0] == 0
    for uw, frag in (([[0.01, 0, 0], [0, 0, 0]], "tangential"),
                     ([[0, 0, 0.01], [0, 0, 0]], "z velocity"),
                     ([[0, float("nan"), 0], [0, 0, 0]], "finite")):
        p = _tube(wall_velocity=uw)
        st, _, msg = check_problem(p, _x0(p))
        assert st == 1 and frag in msg, (uw, msg)
    p = _tube(walls=(False, False, False), wall_velocity=[[0, 0.01, 0], [0, 0, 0]])
    st, _, msg = check_problem(p, _x0(p))
    assert st == 1 and "wall axis" in msg
    L = _lib()
    dp = ctypes.POINTER(ctypes.c_double)
    ctx = ctypes.c_void_p()
    p = _tube(g=(0.0, 0.0, 0.0), wall_velocity=[[0, 0.01, 0], [0, 0, 0]])
    x = np.ascontiguousarray(_x0(p))
    arr = (L.Params * 1)(p)
    st = L.lib.lbm_mc_init_field(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(1 << 20),
                                 ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10 ** 6, None,
                                 ctypes.byref(ctx))
    assert st == 2 and b"moving walls" in L.lib.lbm_mc_last_error()


def test_check_equilibrium_boundary_kind():
    """bc = WALL_EQ selects the equilibrium comparison boundary (Sec. 4.1):
    accepted on any wall axes with the standard forcing; mixing it with
    Appendix A walls in one lattice or across a batch, the corrected
    forcing, wall velocities and a force field are rejected (UNSUPPORTED),
    the last before any device work."""
    from paper_2504_07059_amd.lbm import check_problem
    for walls in ((True, False, False), (False, True, False), (True, True, False)):
        p = _tube(walls=walls, wall_kind="equilibrium")
        st, _, msg = check_problem(p, _x0(p))
        assert st == 0, (walls, msg)
        assert list(p.bc) == [2 if w else 0 for w in walls]
    p = _tube(walls=(True, True, False), wall_kind="equilibrium")
    p.bc[1] = 1
    st, _, msg = check_problem(p, _x0(p))
    assert st == 2 and "WALL_EQ" in msg
    a, b = _tube(wall_kind="equilibrium"), _tube()
    st, _, msg = check_problem([a, b], np.concatenate([_x0(a), _x0(b)]))
    assert st == 2 and "wall kind" in msg
    p = _tube(wall_kind="equilibrium", forcing=1)
    st, _, msg = check_problem(p, _x0(p))
    assert st == 2 and "forcing 0" in msg
    p = _tube(wall_kind="equilibrium", wall_velocity=[[0, 0.01, 0], [0, 0, 0]])
    st, _, msg = check_problem(p, _x0(p))
    assert st == 2 and "moving" in msg
    p.bc[0] = 3
    st, _, msg = check_problem(p, _x0(p))
    assert st == 1 and "WALL_EQ" in msg
    L = _lib()
    dp = ctypes.POINTER(ctypes.c_double)
    ctx = ctypes.c_void_p()
    q = _tube(g=(0.0, 0.0, 0.0), wall_kind="equilibrium")
    x = np.ascontiguousarray(_x0(q))
    arr = (L.Params * 1)(q)
    st = L.lib.lbm_mc_init_field(arr, 1, x.ctypes.data_as(dp), ctypes.c_void_p(1 << 20),
                                 ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10 ** 6, None,
                                 ctypes.byref(ctx))
    assert st == 2 and b"equilibrium" in L.lib.lbm_mc_last_error() and not ctx.value
