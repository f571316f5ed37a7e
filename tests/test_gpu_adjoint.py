"""GPU tests of the hand-written adjoint (through the C ABI) against the FP64
oracle's discrete adjoint (reverse mode through the oracle's steps).

Bars: one reverse step, every adjoint value within 2e-5 of the largest
(FP32 arithmetic of one step, O(1) adjoint fields); parameter gradients of
one step within 1e-4 relative (FP64 sums of FP32 node terms); gradients of a
misfit over hundreds to thousands of steps within 1e-3 relative (FP32 state
and adjoint along the whole trajectory).  The state sequence entry point is
bit-identical to single steps; the reverse sequence, where each reverse
step's transposed stream runs fused with the next one's collision VJP (the
adjoint staying in population space), agrees with single reverse steps to
FP32 rounding."""
import json
import os

import numpy as np
import pytest
import torch

import lbm_workloads as W
from oracle import adjoint as OA
from oracle import evd
from oracle.lattice import DTYPE

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LAM_TOL = 2e-5
GRAD1_RTOL = 1e-4
GRAD_RTOL = 1e-3
WEIGHTS = {9: [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4,
           19: [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12}


def _lbm():
    from paper_2504_07059_amd import lbm
    return lbm


def _adj():
    from paper_2504_07059_amd import adjoint
    return adjoint


def _announce(msg):
    print(f"\n[gpu case] {msg}", flush=True)


TUNING = {}


def _wk(name, lattice, shape, masses, walls, g, seed=11, diff=None, tuning=None):
    N = len(masses)
    if diff is None:
        rng = np.random.default_rng(seed)
        d = rng.uniform(0.06, 0.1, size=(N, N))
        diff = ((d + d.T) / 2).tolist()
    TUNING[name] = tuning
    return W.Workload(name, lattice, *shape, masses, diff, 1.0, list(g), list(walls), 5,
                      "random", seed=seed)


# several tiles per lattice (small work-groups, few layers per thread), ragged
# edges, every wall axis, 2-4 species
CASES = [
    _wk("d2q9_n3_xwall", "D2Q9", (70, 13, 1), [2.0, 28.0, 44.0], (True, False, False),
        (1e-5, 2e-6, 0), diff=W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3),
        tuning=dict(block_x=64, rows=4)),
    _wk("d2q9_n2_ywall", "D2Q9", (45, 14, 1), [1.0, 3.0], (False, True, False), (0, -2e-5, 0),
        tuning=dict(block_x=64, rows=3)),
    _wk("d2q9_n4_periodic", "D2Q9", (37, 11, 1), [1.0, 2.0, 3.0, 4.0], (False, False, False),
        (3e-6, 1e-6, 0), tuning=dict(block_x=64, rows=4)),
    _wk("d2q9_n2_equal", "D2Q9", (66, 5, 1), [1.0, 1.0], (True, False, False), (1e-5, 0, 0),
        tuning=dict(block_x=64, rows=2)),
    _wk("d3q19_n4_zwall", "D3Q19", (14, 9, 8), [1.0, 2.0, 3.0, 4.0], (False, False, True),
        (0, 0, -1e-5), tuning=dict(block_x=32, block_y=2, rows=3, variant=1)),
    _wk("d3q19_n2_xwall", "D3Q19", (11, 7, 6), [1.0, 5.0], (True, False, False), (2e-5, 0, 0),
        tuning=dict(block_x=32, block_y=2, rows=4)),
    _wk("d3q19_n3_ywall", "D3Q19", (9, 10, 5), [1.0, 2.0, 6.0], (False, True, False),
        (0, 1e-5, 0), tuning=dict(block_x=32, block_y=4, rows=2, variant=0)),
    # tiny axes: walls two nodes apart, one periodic row, one layer in 3-D
    _wk("d2q9_n2_two_columns", "D2Q9", (2, 6, 1), [1.0, 3.0], (True, False, False),
        (2e-5, 1e-5, 0), tuning=dict(block_x=64, rows=2)),
    _wk("d2q9_n3_one_row", "D2Q9", (40, 1, 1), [2.0, 28.0, 44.0], (True, False, False),
        (1e-5, 0, 0), diff=W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3),
        tuning=dict(block_x=64, rows=1)),
    _wk("d3q19_n2_one_layer", "D3Q19", (9, 3, 1), [1.0, 4.0], (False, True, False),
        (0, 1e-5, 0), tuning=dict(block_x=32, block_y=2, rows=1, variant=1)),
]


def _pairs(w):
    N = w.n_species
    return [w.diff[i][j] for i in range(N) for j in range(i + 1, N)]


def _sim(w):
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(**TUNING[w.name])
    return sim


def _pops(s, Q):
    """Populations f~ of a stored state [N, Q, ...] (float64)."""
    w = torch.tensor(WEIGHTS[Q], dtype=DTYPE)
    sh = (1, Q) + (1,) * (s.dim() - 2)
    f = (w / w[0]).view(sh) * s[:, :1] + s
    f[:, 0] = s[:, 0]
    return f


def _lam_f(lam_s, Q):
    """dL/df~ from dL/ds (transpose of the storage map s = T f~)."""
    wr = (torch.tensor(WEIGHTS[Q], dtype=DTYPE) / WEIGHTS[Q][0])[1:]
    out = lam_s.clone()
    out[:, 0] = lam_s[:, 0] - (wr.view(1, -1, *([1] * (lam_s.dim() - 2))) * lam_s[:, 1:]).sum(1)
    return out


def _lam_s(lam_f, Q):
    """dL/ds from dL/df~ (inverse transpose of the storage map)."""
    wr = (torch.tensor(WEIGHTS[Q], dtype=DTYPE) / WEIGHTS[Q][0])[1:]
    out = lam_f.clone()
    out[:, 0] = lam_f[:, 0] + (wr.view(1, -1, *([1] * (lam_f.dim() - 2))) * lam_f[:, 1:]).sum(1)
    return out


def _oracle_model(w, D, g):
    return evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, OA.pair_matrix(D, w.n_species),
                     w.tau1, g=g, walls=w.walls, n0=w.n0)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _check_grad(got, D_ref, g_ref, rtol, floor):
    """Per-component relative check; components whose reference is below
    `floor` times the largest (zero in exact arithmetic, e.g. dL/dD at t = 0
    where all species move alike) must stay below that floor: FP32 rounding
    of the other terms, not a signal."""
    ref = list(D_ref) + list(g_ref)
    scale = max(abs(v) for v in ref)
    for k, (u, v) in enumerate(zip(got, ref)):
        if abs(v) >= floor * scale:
            assert _rel(u, v) < rtol, (k, u, v)
        else:
            assert abs(u - v) < floor * scale, (k, u, v)


@pytest.mark.parametrize("w", CASES, ids=[w.name for w in CASES])
def test_adjoint_step_matches_oracle(w):
    """One reverse step at a non-trivial state (5 steps in) with a random
    adjoint field: lam(t-1) elementwise and the D_ij / g gradient terms
    against reverse mode through one oracle step (stream, walls, collide)."""
    _announce(f"adjoint step {w.name}")
    sim = _sim(w)
    sim.step(5)
    s_prev = sim.buffers()[0].clone()
    gen = torch.Generator().manual_seed(7)
    shape = tuple(sim.view(s_prev).shape)
    lam_in_h = torch.randn(shape, generator=gen, dtype=DTYPE)
    lam_in = torch.zeros_like(s_prev)
    sim.view(lam_in).copy_(lam_in_h.float())
    lam_out = torch.zeros_like(s_prev)
    npair = w.n_species * (w.n_species - 1) // 2
    grad = torch.zeros(npair + 3, dtype=torch.float64, device=s_prev.device)
    sim.adjoint_step(s_prev, lam_in, lam_out, grad)
    got_lam = sim.view(lam_out).double().cpu()
    got_grad = grad.cpu().tolist()
    state = sim.view(s_prev).double().cpu()
    sim.sync()
    sim.close()

    Q = shape[1]
    D = torch.tensor(_pairs(w), dtype=DTYPE, requires_grad=True)
    g = torch.tensor(w.g, dtype=DTYPE, requires_grad=True)
    m = _oracle_model(w, D, g)
    fprev = _pops(state, Q).requires_grad_()
    out = evd.collide(m, evd.stream(m, fprev))
    (out * _lam_f(lam_in_h.float().double(), Q)).sum().backward()
    ref_lam = _lam_s(fprev.grad, Q)
    err = ((got_lam - ref_lam).abs().max() / ref_lam.abs().max()).item()
    assert err < LAM_TOL, err
    _check_grad(got_grad, D.grad.tolist(), g.grad.tolist(), GRAD1_RTOL, 1e-6)


@pytest.mark.parametrize("w", CASES[::2], ids=[w.name for w in CASES[::2]])
def test_adjoint_init_matches_oracle(w):
    """Gradient terms of the initialisation s(0) = store(C(f(0; g))), with
    f(0) built at u_i0 = -g/2, against reverse mode through the oracle's
    initial populations and collision."""
    _announce(f"adjoint init {w.name}")
    sim = _sim(w)
    s0 = sim.buffers()[0]
    gen = torch.Generator().manual_seed(8)
    shape = tuple(sim.view(s0).shape)
    lam_h = torch.randn(shape, generator=gen, dtype=DTYPE)
    lam = torch.zeros_like(s0)
    sim.view(lam).copy_(lam_h.float())
    npair = w.n_species * (w.n_species - 1) // 2
    grad = torch.zeros(npair + 3, dtype=torch.float64, device=s0.device)
    sim.adjoint_init(lam, grad)
    got = grad.cpu().tolist()
    sim.sync()
    sim.close()

    Q = shape[1]
    D = torch.tensor(_pairs(w), dtype=DTYPE, requires_grad=True)
    g = torch.tensor(w.g, dtype=DTYPE, requires_grad=True)
    m = _oracle_model(w, D, g)
    f0 = evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE))
    (evd.collide(m, f0) * _lam_f(lam_h.float().double(), Q)).sum().backward()
    _check_grad(got, D.grad.tolist(), g.grad.tolist(), GRAD1_RTOL, 1e-6)


@pytest.mark.parametrize("case", [0, 6, 4], ids=["d2q9_n3", "d3q19_n3", "d3q19_n4"])
def test_sequence_entry_points_equal_single_steps(case):
    """replay == step bit for bit, and adjoint_run == repeated adjoint_step
    over a sequence with an odd number of steps: bit for bit for a one-step
    run; with fused reverse steps within 1e-5 of the largest
    adjoint value and of the largest gradient term (the fused pass skips the
    storage transform and its inverse between steps, each a few FP32
    roundings of O(1) values per step).  The sequence calls replay captured
    graphs from their second call on: each is called twice, with other work
    and a synchronisation in between, and both calls are checked against the
    single steps and against each other."""
    w = CASES[case]
    _announce(f"replay / adjoint_run {w.name}")
    sim = _sim(w)
    n = 7
    s0 = sim.buffers()[0].clone()
    stride = (sim.total + 63) // 64 * 64
    seq = torch.zeros((n + 1, stride), dtype=torch.float32, device=s0.device)
    sim.step(n)
    ref_state = sim.view(sim.buffers()[0]).clone()
    for rep in range(2):
        seq.zero_()
        seq[0, : sim.total].copy_(s0)
        sim.replay(seq[0], n, seq[1:])
        sim.sync()
        # node values only: the row padding is never written
        assert torch.equal(ref_state, sim.view(seq[n, : sim.total])), rep

    gen = torch.Generator().manual_seed(9)
    lam_T = torch.zeros_like(s0)
    sim.view(lam_T).copy_(torch.randn(tuple(sim.view(s0).shape), generator=gen))
    npair = w.n_species * (w.n_species - 1) // 2
    g_ref = torch.zeros(npair + 3, dtype=torch.float64, device=s0.device)
    a, b = lam_T.clone(), torch.zeros_like(s0)
    for k in range(n, 0, -1):
        sim.adjoint_step(seq[k - 1, : sim.total], a, b, g_ref)
        a, b = b, a
    runs = []
    for rep in range(2):
        g1 = torch.zeros_like(g_ref)
        out_run = torch.zeros_like(s0)
        sim.adjoint_run(seq, n, lam_T, out_run, g1)
        sim.step(3)                     # other work between the two calls
        sim.sync()
        got, ref = sim.view(out_run), sim.view(a)
        assert (got - ref).abs().max().item() <= 1e-5 * ref.abs().max().item(), rep
        assert (g1 - g_ref).abs().max().item() <= 1e-5 * g_ref.abs().max().item(), rep
        runs.append((got.clone(), g1.clone()))
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    # a one-step run is kernel A and kernel B, as adjoint_step
    g1 = torch.zeros_like(g_ref)
    g2 = torch.zeros_like(g_ref)
    out_run = torch.zeros_like(s0)
    out_step = torch.zeros_like(s0)
    sim.adjoint_run(seq, 1, lam_T, out_run, g1)
    sim.adjoint_step(seq[0, : sim.total], lam_T, out_step, g2)
    sim.sync()
    assert torch.equal(sim.view(out_run), sim.view(out_step))
    assert torch.equal(g1, g2)
    sim.close()


def test_sequence_beyond_the_cache_equals_single_steps():
    """A ternary tube of 1024x640 nodes, whose four population-sized buffers
    of the reverse step (283 MB) exceed the 256 MB last-level cache: the
    reverse kernels store non-temporally and the fused pass runs its build
    for three waves per SIMD (marching and gradient sums in LDS).  A
    sequence of 5 reverse steps against single reverse steps (kernels A and
    B): within 1e-5 of the largest adjoint value and of the largest gradient
    term, as for the cache-resident builds."""
    _, ev = W.adjoint_tube(nx=1024, ny=640, steps=5)
    _announce("adjoint_run 1024x640 (beyond the last-level cache)")
    lbm = _lbm()
    sim = lbm.LbmMc(lbm.params_from_workload(ev), ev.x0())
    n = 5
    s0 = sim.buffers()[0].clone()
    assert 4 * sim.total * 4 > (256 << 20)
    stride = (sim.total + 63) // 64 * 64
    seq = torch.zeros((n + 1, stride), dtype=torch.float32, device=s0.device)
    seq[0, : sim.total].copy_(s0)
    sim.replay(seq[0], n, seq[1:])
    gen = torch.Generator().manual_seed(5)
    lam_T = torch.zeros_like(s0)
    sim.view(lam_T).copy_(torch.randn(tuple(sim.view(s0).shape), generator=gen))
    g_ref = torch.zeros(3 + 3, dtype=torch.float64, device=s0.device)
    a, b = lam_T.clone(), torch.zeros_like(s0)
    for k in range(n, 0, -1):
        sim.adjoint_step(seq[k - 1, : sim.total], a, b, g_ref)
        a, b = b, a
    g1 = torch.zeros_like(g_ref)
    out_run = torch.zeros_like(s0)
    sim.adjoint_run(seq, n, lam_T, out_run, g1)
    sim.sync()
    got, ref = sim.view(out_run), sim.view(a)
    assert (got - ref).abs().max().item() <= 1e-5 * ref.abs().max().item()
    assert (g1 - g_ref).abs().max().item() <= 1e-5 * g_ref.abs().max().item()
    sim.close()


def _tube_problem(nx, ny, steps, K):
    adj = _adj()
    truth, ev = W.adjoint_tube(nx=nx, ny=ny, steps=steps)
    prob = adj.Problem("D2Q9", nx, ny, 1, ev.masses, ev.tau1, ev.walls, ev.x0(), steps,
                       checkpoint_every=K)
    return truth, ev, prob


def _gpu_gradient(ev, prob, target):
    adj = _adj()
    pairs = torch.tensor(_pairs(ev), dtype=torch.float64, requires_grad=True)
    g = torch.tensor(ev.g, dtype=torch.float64, requires_grad=True)
    xbar = adj.evolve(pairs, g, prob)
    L = adj.profile_misfit(xbar, torch.as_tensor(target, device=xbar.device))
    L.backward()
    return L.item(), pairs.grad.tolist(), g.grad.tolist()


def test_misfit_gradient_small_tube_matches_oracle():
    """Checkpointed forward + reverse sweep (K = 64, 400 steps: a partial last
    segment) of the profile misfit on a 96x4 tube against reverse mode through
    the FP64 oracle (one row: the tube is y-uniform)."""
    _announce("misfit gradient 96x4, 400 steps")
    truth, ev, prob = _tube_problem(96, 4, 400, 64)
    tube = OA.Tube("D2Q9", 96, 1, 1, ev.masses, ev.tau1, ev.walls,
                   torch.tensor(ev.x0()[:, :, :1, :], dtype=DTYPE))
    with torch.no_grad():
        target = OA.profile(tube, torch.tensor(_pairs(truth), dtype=DTYPE),
                            torch.tensor(truth.g, dtype=DTYPE), 400)
    L_ref, dp_ref, dg_ref = OA.gradient(tube, _pairs(ev), ev.g, target, 400, segment=100)
    L, dp, dg = _gpu_gradient(ev, prob, target)
    assert _rel(L, L_ref) < 1e-3, (L, L_ref)
    for u, v in zip(dp + dg[:1], dp_ref + dg_ref[:1]):
        assert _rel(u, v) < GRAD_RTOL, (u, v)
    assert abs(dg[1]) <= 1e-6 * abs(dg_ref[0]) and dg[2] == 0.0


def test_recorded_states_give_the_checkpointed_gradient():
    """checkpoint_every = 0 records every state in the forward and recomputes
    nothing; the reverse steps then run on the same states as with
    checkpoints (the recomputation is bitwise the forward step): the loss is
    identical.  The gradient agrees to FP32 rounding: with checkpoints the
    adjoint passes through its storage form at each segment boundary, while
    the recorded run's fused reverse steps keep it in population space, and
    the FP64 sums are grouped per segment instead of once over the run.  A
    run of one step (no boundary) agrees to the last digits."""
    import dataclasses
    for steps in (400, 1):
        _announce(f"recorded states 96x4, {steps} steps")
        truth, ev, prob = _tube_problem(96, 4, steps, 64)
        target = np.full((ev.n_species, 96), 1.0 / ev.n_species)
        L_ref, dp_ref, dg_ref = _gpu_gradient(ev, prob, target)
        scale = max(abs(v) for v in dp_ref + dg_ref)
        # recorded explicitly, and by the automatic choice (a small problem
        # fits in memory)
        for K in (0, None):
            L, dp, dg = _gpu_gradient(ev, dataclasses.replace(prob, checkpoint_every=K), target)
            assert L == L_ref
            tol = 1e-12 if steps == 1 else 1e-5
            for u, v in zip(dp + dg, dp_ref + dg_ref):
                assert abs(u - v) <= tol * scale, (K, u, v)


def test_misfit_gradient_full_tube_matches_stored_oracle():
    """The full adjoint workload: 512x64 tube, 4000 steps, checkpoints every
    100 steps; gradient with respect to the three D_ij and g_x against the
    stored FP64 oracle reverse-mode gradient (itself pinned by central
    differences)."""
    with open(os.path.join(GOLDEN, "adjoint_tube.json")) as fh:
        G = json.load(fh)
    _announce("misfit gradient 512x64, 4000 steps")
    truth, ev, prob = _tube_problem(512, 64, 4000, 100)
    assert _pairs(ev) == G["pairs_eval"] and list(ev.g) == G["g_eval"]
    L, dp, dg = _gpu_gradient(ev, prob, np.asarray(G["target"]))
    assert _rel(L, G["loss"]) < 1e-3, (L, G["loss"])
    for u, v in zip(dp + dg[:1], G["grad_pairs"] + G["grad_g"][:1]):
        assert _rel(u, v) < GRAD_RTOL, (u, v)


def test_adjoint_rejects_the_diffusion_forcing():
    """The reverse step differentiates the standard forcing only: a context
    with forcing 1 gets UNSUPPORTED from the adjoint entry points, and its
    forward stepping is unaffected."""
    import dataclasses
    lbm = _lbm()
    w = dataclasses.replace(CASES[0], forcing="diff")
    _announce(f"adjoint rejects forcing 1 {w.name}")
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.step(2)
    s_prev = sim.buffers()[0].clone()
    lam_in = torch.zeros_like(s_prev)
    lam_out = torch.zeros_like(s_prev)
    grad = torch.zeros(w.n_species * (w.n_species - 1) // 2 + 3, dtype=torch.float64,
                       device=s_prev.device)
    from paper_2504_07059_amd._lib import LbmError
    with pytest.raises(LbmError) as e:
        sim.adjoint_step(s_prev, lam_in, lam_out, grad)
    assert e.value.status == 2 and "forcing" in str(e.value)
    with pytest.raises(LbmError) as e:
        sim.adjoint_init(lam_in, grad)
    assert e.value.status == 2
    sim.step(2)
    sim.sync()
    sim.close()


def test_adjoint_rejects_walls_on_several_axes():
    """Boxes with walls on two axes step forward (edges and corners are
    handled), but the reverse step covers walls on one axis only: the adjoint
    entry points return UNSUPPORTED."""
    import dataclasses
    lbm = _lbm()
    w = dataclasses.replace(CASES[0], walls=[True, True, False])
    _announce(f"adjoint rejects walls on two axes {w.name}")
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.step(2)
    s_prev = sim.buffers()[0].clone()
    lam_in = torch.zeros_like(s_prev)
    lam_out = torch.zeros_like(s_prev)
    grad = torch.zeros(w.n_species * (w.n_species - 1) // 2 + 3, dtype=torch.float64,
                       device=s_prev.device)
    from paper_2504_07059_amd._lib import LbmError
    with pytest.raises(LbmError) as e:
        sim.adjoint_step(s_prev, lam_in, lam_out, grad)
    assert e.value.status == 2 and "several axes" in str(e.value)
    sim.step(2)
    sim.sync()
    sim.close()
