"""GPU test of lbm_mc_profile_static, the entry point that allocates nothing
(its FP64 partial sums live in the library's fixed device array), through the
C ABI, against lbm_mc_profile on the same states: bit-identical where it uses
the same row chunks, within FP64 rounding where the array forces fewer
chunks; two calls in a row, the second on a smaller lattice, and the first
again after it (the array keeps the last call's contents); sizes beyond the
array rejected before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import lbm_workloads as W

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


def _wk(name, lattice, shape, masses, walls, g, seed):
    N = len(masses)
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.05, 0.1, size=(N, N))
    return W.Workload(name, lattice, *shape, masses, ((d + d.T) / 2).tolist(), 1.0, list(g),
                      list(walls), 5, "random", seed=seed)


def _static(sim, state, out):
    """The entry point called through ctypes with raw device pointers."""
    from paper_2504_07059_amd import _lib
    st = _lib.lib.lbm_mc_profile_static(sim.ctx, ctypes.c_void_p(state.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()))
    return st


def test_static_profile_equals_profile_twice():
    lbm = _lbm()
    big = _wk("d2q9_n3_big", "D2Q9", (700, 90, 1), [2.0, 28.0, 44.0], (True, False, False),
              (1e-5, 0, 0), 3)
    small = _wk("d3q19_n4_small", "D3Q19", (40, 20, 12), [1.0, 2.0, 3.0, 4.0],
                (False, False, True), (0, 0, -1e-5), 4)
    _announce("profile_static: big then small then big")
    sims = []
    for w in (big, small):
        sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        sim.step(7)
        sims.append(sim)
    refs = [s.profile() for s in sims]
    for k in (0, 1, 0):
        sim = sims[k]
        out = torch.full_like(refs[k], float("nan"))
        assert _static(sim, sim.buffers()[0], out) == 0
        torch.cuda.synchronize()
        assert torch.equal(out, refs[k]), k
    for s in sims:
        s.sync()
        s.close()


def test_static_profile_with_fewer_chunks():
    """A lattice whose row chunks do not all fit the array (N nx = 400000 of
    524288 doubles): the entry point uses one chunk of all rows; the result
    agrees with lbm_mc_profile to FP64 rounding."""
    lbm = _lbm()
    w = _wk("d2q9_n4_wide", "D2Q9", (100000, 8, 1), [1.0, 2.0, 3.0, 4.0], (True, False, False),
            (1e-6, 0, 0), 5)
    _announce("profile_static: wide lattice, capped chunks")
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.step(3)
    ref = sim.profile()
    out = torch.full_like(ref, float("nan"))
    assert _static(sim, sim.buffers()[0], out) == 0
    torch.cuda.synchronize()
    assert (out - ref).abs().max().item() < 1e-13
    sim.sync()
    sim.close()


def test_static_profile_rejects_sizes_beyond_the_array():
    lbm = _lbm()
    w = _wk("d2q9_n4_too_wide", "D2Q9", (131073, 1, 1), [1.0, 2.0, 3.0, 4.0],
            (False, False, False), (0, 0, 0), 6)
    _announce("profile_static: rejected size")
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    out = torch.zeros((4, w.nx), dtype=torch.float64, device="cuda")
    assert _static(sim, sim.buffers()[0], out) == 1
    from paper_2504_07059_amd import _lib
    assert b"exceeds the fixed scratch" in _lib.lib.lbm_mc_last_error()
    assert bool((out == 0).all())
    sim.close()
