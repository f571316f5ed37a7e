"""Benchmark of the EVD multicomponent LBM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only LEG]

Headline workload: the batched form, 512 independent D2Q9 ternary tubes of
uneven sizes (nx in 128..2048, ny in 16..64; 22.76 M nodes, 2.46 GB per
population buffer), each with its own seeded pair diffusivities, gravity and
molar masses, walls at the x ends, halves of two uniform compositions
(synthetic stand-ins for the paper's Case I tube).  One step advances every
tube by one fused time step (stream with the second-order interpolation and
the impermeable walls, moments, cross-relaxation solve, collision with
forcing, store) in one persistent launch.  The value is MLUPS x species =
nodes * species * steps / microseconds over K timed steps, with the state
resident in HBM before the timed region.

The JSON line carries, besides the contract's keys:
  roofline      the fused step kernel against the HBM roofline: algorithmic
                bytes per launch (72 B per species-node for D2Q9, one FP32
                read and one FP32 write of 9 populations; 152 B for D3Q19)
                divided by the average launch duration, timed with HIP events
                on the launch stream over the timed region, against 8 TB/s;
                `traffic` is the counted HBM bytes per launch (FETCH_SIZE +
                WRITE_SIZE, copy-calibrated) from the committed profile of the
                same kernel sources and shape, else null; `ceiling` is the
                same rate against the library's streaming copy
                (lbm_mc_stream_copy), the practical read-write ceiling.
  accuracy      the paired accuracy gate: the same batch run for its
                configured 10,000 steps at the timed shape, sampled tubes
                against the stored FP64 oracle result (max |dx|), and the
                FP64 mass drift of every tube.
  cpu_baseline  the FP64 oracle, as it stands, on this host's cores, on a
                bounded sample of the same workload (whole tubes of the
                batch), with all threads and with one.
  sub           the other forms of the metric, each with its roofline and
                its paired accuracy: the batch launched tube by tube; the
                ternary tube at 16384 x 1024 (HBM scale) and its physics
                variants; the 1024 x 64 tube (last-level-cache resident); the
                3-D layer (D3Q19, 4 species, 256 x 128 x 128); the adjoint
                (gradient of a profile misfit, checkpointed) on the 512 x 64
                tube and at HBM scale; the streaming copy sweep.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS x species + % HBM roofline (fwd, batched, adjoint) at 1e-5 mole-frac error"
UNIT = "MLUPS x species"
PEAK_HBM_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")


def bytes_per_species_node(lattice):
    return 2 * 4 * (9 if lattice == "D2Q9" else 19)


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _timed_steps(sim, steps, warmup):
    """Warm up, capture the step graphs outside the timed region, then time
    exactly `steps` steps with events on the context's stream."""
    import torch
    sim.step(warmup)
    sim.prepare(steps)
    sim.sync()
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    sim.sync()
    return e0.elapsed_time(e1)


# ------------------------------------------------------------------ roofline
KERNEL_SOURCES = ("step_impl.hpp", "kernels.hpp", "collide.hpp", "lattice.hpp", "common.hpp",
                  "host.hip")
# the reverse step's kernels (the fused pass) read the forward gather as well
ADJOINT_SOURCES = KERNEL_SOURCES + ("adjoint.hip", "adjoint.hpp")


def kernel_sources_sha(sources=KERNEL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2504_07059_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, tuning, sources=KERNEL_SOURCES):
    """HBM bytes per launch of the dominant kernel (the fused step; the fused
    reverse pass for an adjoint workload, tuning "reverse") from the committed
    counter summaries (FETCH_SIZE + WRITE_SIZE, copy-calibrated), if one was
    taken for this workload and execution shape from the current kernel
    sources; else None."""
    import glob
    sha = kernel_sources_sha(sources)
    want = ",".join(str(v) for v in tuning)
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                rec = dict(kv.split("=", 1) for kv in line.split()[1:])
                if (rec.get("workload") == workload_name and rec.get("tuning") == want
                        and rec.get("kernel_sources_sha256_16") == sha):
                    return float(rec["bytes_per_launch"])
    return None


def roofline(name, per_launch_bytes, ms, steps, tuning=None, ceiling=None, bound="hbm",
             sources=KERNEL_SOURCES):
    avg_s = ms * 1e-3 / steps
    achieved = per_launch_bytes / avg_s / 1e9
    out = {"bound": bound, "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": achieved / PEAK_HBM_GBS,
           "traffic": measured_traffic(name, tuning, sources) if tuning is not None else None,
           "bytes_per_launch": per_launch_bytes, "avg_launch_us": avg_s * 1e6}
    if ceiling:
        out["ceiling"] = {"kernel": "lbm_mc_stream_copy", "GBs": ceiling,
                          "frac": achieved / ceiling}
    return out


# ------------------------------------------------------------ streaming copy
def copy_sweep(sizes_gib=(1, 2, 4), blocks_per_cu=(1, 2, 4, 8), reps=5):
    """The library's streaming copy over buffer sizes and grid sizes: the
    best read+write rate over buffers of 2 GiB and more (well beyond the
    256 MB last-level cache) is the practical ceiling of a read-one-write-one
    kernel."""
    import ctypes
    import torch
    from paper_2504_07059_amd._lib import lib
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    rows = []
    best = 0.0
    for gib in sizes_gib:
        n = (gib << 30) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for bpc in blocks_per_cu:
            blocks = cus * bpc
            args = (ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n, blocks, sp)
            for _ in range(2):
                assert lib.lbm_mc_stream_copy(*args) == 0
            e0, e1 = _events()
            e0.record(stream)
            for _ in range(reps):
                lib.lbm_mc_stream_copy(*args)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = 2 * n * 4 / (ms * 1e-3) / 1e9
            rows.append({"GiB": gib, "blocks": blocks, "us": ms * 1e3, "GBs": gbs})
            if gib >= 2:
                best = max(best, gbs)
        assert torch.equal(a[:1024], b[:1024]) and torch.equal(a[-1024:], b[-1024:])
        del a, b
        torch.cuda.empty_cache()
    return {"best_GBs": best, "frac_of_peak": best / PEAK_HBM_GBS, "sweep": rows}


# ------------------------------------------------------------------- batched
def batch_workload():
    import lbm_workloads as W
    from paper_2504_07059_amd import lbm
    tubes = W.batched_tubes()
    params = [lbm.params_from_workload(w) for w in tubes]
    return tubes, params, W.concat_x0(tubes)


def time_batched(steps, warmup, modes=(1,), autotune=True, tuning=None):
    """The 512-tube batch, one persistent launch per step (mode 1) and, for
    comparison, one launch per tube per step (mode 0), both under captured
    graphs, at the autotuned shape of the one-launch form."""
    import numpy as np
    from paper_2504_07059_amd import lbm
    tubes, params, x0 = batch_workload()
    nodes = sum(w.nodes for w in tubes)
    if autotune and tuning is None:
        tmp = lbm.LbmMc(params, x0)
        tmp.autotune(reps=3)
        tuning = tmp.get_tuning()
        tmp.close()
    sim = lbm.LbmMc(params, x0)
    if tuning is not None:
        sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"].copy()
    res = {}
    for mode in modes:
        sim.set_batched_mode(mode)
        res[mode] = _timed_steps(sim, steps, warmup)
    drift = float(np.abs(sim.moments(fields=False)["mass"] / m0 - 1).max())
    tune = sim.get_tuning()
    sim.close()
    return {"nodes": nodes, "lattices": len(tubes), "ms": res, "tuning": list(tune),
            "mass_drift_timed_run": drift}


def batched_accuracy(tuning, steps=10000):
    """Paired accuracy gate of the batch: the configured 10,000 steps at the
    timed shape; the stored oracle profiles of six sampled tubes (one row
    each: the tubes are uniform along y) against every row of those tubes,
    and the FP64 mass drift of all 512 tubes."""
    import numpy as np
    from paper_2504_07059_amd import lbm
    path = os.path.join(GOLDEN, "batched_sample.json")
    tubes, params, x0 = batch_workload()
    sim = lbm.LbmMc(params, x0)
    sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"].copy()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.sync()
    run_s = time.perf_counter() - t0
    out = sim.moments()
    sim.sync()
    drift = float(np.abs(out["mass"] / m0 - 1).max())
    dx = None
    if os.path.exists(path):
        G = json.load(open(path))["tubes"]
        dx = 0.0
        for k, rec in G.items():
            ref = np.array(rec[str(steps)]["x"])                        # [N, nx]
            x = sim.field(out, "x", lattice=int(k)).double().cpu().numpy()[:, 0]
            dx = max(dx, float(np.abs(x - ref[:, None, :]).max()))
    sim.close()
    return {"steps": steps, "max_dx_vs_oracle": dx, "sampled_tubes": 6,
            "mass_drift": drift, "run_s": run_s}


# --------------------------------------------------------------- one lattice
def time_lattice(w, steps, warmup, autotune=True, tuning=None, accel=None):
    import numpy as np
    from paper_2504_07059_amd import lbm
    p = lbm.params_from_workload(w)
    x0 = w.x0()
    if autotune and tuning is None:
        tmp = lbm.LbmMc(p, x0, accel=accel)
        tmp.autotune(reps=5)
        tuning = tmp.get_tuning()
        tmp.close()
    sim = lbm.LbmMc(p, x0, accel=accel)
    if tuning is not None:
        sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"][0].copy()
    ms = _timed_steps(sim, steps, warmup)
    drift = float(np.abs(sim.moments(fields=False)["mass"][0] / m0 - 1).max())
    tune = sim.get_tuning()
    sim.close()
    return ms, drift, list(tune)


def tube_accuracy_vs_oracle(w, tuning, steps):
    """A tube uniform along y against the FP64 oracle run on one row for the
    same steps (every row compared)."""
    import numpy as np
    import torch
    from oracle import evd
    from oracle.lattice import DTYPE
    from paper_2504_07059_amd import lbm
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(steps)
    out = sim.moments()
    sim.sync()
    x = sim.field(out, "x").double().cpu().numpy()[:, 0]               # [N, ny, nx]
    drift = float(np.abs(out["mass"][0] / m0 - 1).max())
    sim.close()
    m = evd.Model(w.lattice, w.nx, 1, 1, w.masses, torch.tensor(w.diff, dtype=DTYPE), w.tau1,
                  g=w.g, walls=w.walls, n0=w.n0, forcing=w.forcing)
    f = evd.initial_populations(m, torch.tensor(w.x0()[:, :, :1, :], dtype=DTYPE))
    with torch.no_grad():
        f = evd.run(m, f, steps)
    ref = evd.observables(m, f)["x"][:, 0, 0, :].numpy()
    return {"steps": steps, "max_dx_vs_oracle": float(np.abs(x - ref[:, None, :]).max()),
            "mass_drift": drift}


def tube_accuracy_vs_golden(w, tuning, t=20000):
    """The 1024x64 tube at step t against the stored oracle result."""
    import numpy as np
    from paper_2504_07059_amd import lbm
    g = json.load(open(os.path.join(GOLDEN, "ternary_gravity.json")))["checkpoints"][str(t)]
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(t)
    out = sim.moments()
    sim.sync()
    x = sim.field(out, "x").double().cpu().numpy()
    dx = float(np.abs(x[:, 0] - np.array(g["x"])[:, None, :]).max())
    drift = float(np.abs(out["mass"][0] / m0 - 1).max())
    sim.close()
    return {"steps": t, "max_dx_vs_oracle": dx, "mass_drift": drift}


def layer_accuracy_crops(w, tuning, steps=8, samples=((5, 7, 0), (100, 64, 63), (255, 127, 127),
                                                     (64, 0, 96))):
    """The 3-D layer at full size after a few steps, at sampled nodes (on both
    z walls, at the interface and on the periodic seams), against the oracle
    run on a crop around each (after s steps a node depends only on its
    radius-s neighbourhood; the crop keeps the real walls and is periodic
    elsewhere, exact at its centre)."""
    import numpy as np
    import torch
    from oracle import evd
    from oracle.lattice import DTYPE
    from paper_2504_07059_amd import lbm
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    sim.set_tuning(*tuning)
    sim.step(steps)
    out = sim.moments()
    sim.sync()
    x = sim.field(out, "x").double().cpu().numpy()                      # [N, nz, ny, nx]
    sim.close()
    x0 = w.x0()
    r = steps + 1
    dx = 0.0
    for (cx, cy, cz) in samples:
        ix = [(cx + k) % w.nx for k in range(-r, r + 1)]
        iy = [(cy + k) % w.ny for k in range(-r, r + 1)]
        z0, z1 = max(0, cz - r), min(w.nz, cz + r + 1)
        sub = x0[:, z0:z1][:, :, iy][:, :, :, ix]
        # a crop touching a z wall keeps walls on both of its z ends (the far
        # end is beyond the centre's reach); an interior crop is periodic
        m = evd.Model(w.lattice, len(ix), len(iy), z1 - z0, w.masses,
                      torch.tensor(w.diff, dtype=DTYPE), w.tau1, g=w.g,
                      walls=(False, False, w.walls[2] and (z0 == 0 or z1 == w.nz)),
                      n0=w.n0)
        f = evd.initial_populations(m, torch.tensor(np.ascontiguousarray(sub), dtype=DTYPE))
        with torch.no_grad():
            f = evd.run(m, f, steps)
        ref = evd.observables(m, f)["x"][:, cz - z0, r, r].numpy()
        dx = max(dx, float(np.abs(x[:, cz, cy, cx] - ref).max()))
    return {"steps": steps, "max_dx_vs_oracle_sampled": dx, "samples": len(samples)}


# ------------------------------------------------------------------- adjoint
def time_adjoint(nx=512, ny=64, steps=4000, K=100, fwd_bwd=True):
    """Gradient of the profile misfit with respect to the three pair
    diffusivities and g through the checkpointed adjoint: time per forward +
    backward step against a plain forward step on the same lattice, and the
    reverse step alone."""
    import dataclasses
    import torch
    import lbm_workloads as W
    from paper_2504_07059_amd import adjoint as A
    from paper_2504_07059_amd import lbm
    truth, ev = W.adjoint_tube(nx=nx, ny=ny, steps=steps)
    N = ev.n_species
    pairs = lambda w: [w.diff[i][j] for i in range(N) for j in range(i + 1, N)]
    prob = A.Problem("D2Q9", ev.nx, ev.ny, 1, ev.masses, ev.tau1, ev.walls, ev.x0(), steps,
                     checkpoint_every=K)
    f64 = torch.float64
    species_nodes = ev.nodes * N
    sim = lbm.LbmMc(lbm.params_from_workload(ev), ev.x0())
    ms_fwd = _timed_steps(sim, min(steps, 2000), 100)
    fwd_us = ms_fwd * 1e3 / min(steps, 2000)
    # one checkpoint segment: recomputation and the reverse steps
    stride = (sim.total + 63) // 64 * 64
    seg = torch.empty((K, stride), dtype=torch.float32, device=sim.fa.device)
    seg[0, : sim.total].copy_(sim.buffers()[0])
    sim.replay(seg[0], K - 1, seg[1:])               # warm (captures its graph)
    e0, e1 = _events()
    e0.record(sim.stream)
    sim.replay(seg[0], K - 1, seg[1:])
    e1.record(sim.stream)
    lam_a = torch.zeros(sim.total, dtype=torch.float32, device=seg.device)
    lam_b = torch.zeros_like(lam_a)
    sim.view(lam_a).fill_(1e-3)
    grad = torch.zeros(N * (N - 1) // 2 + 3, dtype=f64, device=seg.device)
    sim.adjoint_run(seg, K, lam_a, lam_b, grad)      # warm
    e2, e3 = _events()
    e2.record(sim.stream)
    sim.adjoint_run(seg, K, lam_a, lam_b, grad)
    e3.record(sim.stream)
    torch.cuda.synchronize()
    replay_us = e0.elapsed_time(e1) * 1e3 / (K - 1)
    reverse_us = e2.elapsed_time(e3) * 1e3 / K
    sim_total = sim.total
    sim.close()
    del seg
    out = {"workload": f"adjoint_tube_{nx}x{ny}", "steps": steps, "checkpoint_every": K,
           "species_nodes": species_nodes, "forward_us_per_step": fwd_us,
           "replay_us_per_step": replay_us, "reverse_us_per_step": reverse_us,
           # one forward step of the gradient: forward, recomputation, reverse
           "fwd_bwd_kernel_us_per_step": fwd_us + replay_us + reverse_us,
           "reverse_roofline": roofline(f"adjoint_tube_{nx}x{ny}", 108 * species_nodes,
                                        reverse_us * 1e-3, 1, tuning=("reverse",),
                                        sources=ADJOINT_SOURCES),
           "fwd_bwd_roofline": roofline(None, 252 * species_nodes,
                                        (fwd_us + replay_us + reverse_us) * 1e-3, 1)}
    out["fwd_bwd_kernel_over_forward"] = out["fwd_bwd_kernel_us_per_step"] / fwd_us
    # every state recorded in the forward (checkpoint_every = 0, memory
    # permitting): the forward is the recording replay, nothing is recomputed
    out["recorded_fwd_bwd_kernel_us_per_step"] = replay_us + reverse_us
    out["recorded_fwd_bwd_kernel_over_forward"] = (replay_us + reverse_us) / fwd_us
    out["recorded_state_bytes"] = 4 * sim_total * (steps + 1)
    if not fwd_bwd:
        return out
    with torch.no_grad():
        target = A.evolve(torch.tensor(pairs(truth), dtype=f64),
                          torch.tensor(truth.g, dtype=f64), prob)

    def run():
        p_t = torch.tensor(pairs(ev), dtype=f64, requires_grad=True)
        g_t = torch.tensor(ev.g, dtype=f64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = A.profile_misfit(A.evolve(p_t, g_t, prob), target)
        L.backward()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, L, p_t, g_t

    wall_cold = run()[0]
    wall, L, p_t, g_t = run()
    out.update({"fwd_bwd_wall_ms_per_step": wall * 1e3 / steps,
                "fwd_bwd_wall_over_forward": wall * 1e6 / steps / fwd_us,
                "fwd_bwd_first_call_ms_per_step": wall_cold * 1e3 / steps,
                "loss": L.item(), "grad_pairs": p_t.grad.tolist(),
                "grad_g": g_t.grad.tolist()})
    # the same gradient with every state recorded in the forward
    prob_k, prob = prob, dataclasses.replace(prob, checkpoint_every=0)
    run()
    wall_r, L_r, p_r, g_r = run()
    prob = prob_k
    out.update({"recorded_fwd_bwd_wall_ms_per_step": wall_r * 1e3 / steps,
                "recorded_fwd_bwd_wall_over_forward": wall_r * 1e6 / steps / fwd_us,
                "recorded_loss_equals_checkpointed": L_r.item() == L.item(),
                "recorded_grad_max_rel_diff": max(
                    abs(u - v) / max(abs(v), 1e-300)
                    for u, v in zip(p_r.grad.tolist() + g_r.grad.tolist()[:1],
                                    p_t.grad.tolist() + g_t.grad.tolist()[:1]))})
    gpath = os.path.join(GOLDEN, "adjoint_tube.json")
    if (nx, ny, steps, K) == (512, 64, 4000, 100) and os.path.exists(gpath):
        G = json.load(open(gpath))
        ref = G["grad_pairs"] + G["grad_g"][:1]
        got = out["grad_pairs"] + out["grad_g"][:1]
        out["accuracy"] = {"max_rel_grad_err_vs_oracle": max(abs(u - v) / abs(v)
                                                             for u, v in zip(got, ref)),
                           "rel_loss_err_vs_oracle": abs(L.item() - G["loss"]) / G["loss"]}
    return out


def time_adjoint_3d(K=20):
    """Reverse sweeps of D3Q19 lattices: a ternary box 256x128x64 with z
    walls (the adjoint tube's gases) and the 3-D layer workload (four
    species, 256x128x128): K recorded states, then K reverse steps through
    lbm_mc_adjoint_run (fused passes), against a forward step."""
    import torch
    import lbm_workloads as W
    from paper_2504_07059_amd import lbm
    cases = [("adjoint_d3q19_ternary_256x128x64",
              W.Workload("adjoint_d3q19_ternary", "D3Q19", 256, 128, 64, [2.0, 28.0, 44.0],
                         W.pairs_to_matrix(W.load_accepted()["ternary_gravity"]["pairs"], 3),
                         1.0, [0.0, 0.0, -1e-6], [False, False, True], K, "halves")),
             ("adjoint_layer_mixing_3d_256x128x128", workload("c2"))]
    out = {}
    for name, w in cases:
        sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
        stride = (sim.total + 63) // 64 * 64
        seq = torch.zeros((K + 1, stride), dtype=torch.float32, device="cuda")
        seq[0, : sim.total].copy_(sim.buffers()[0])
        sim.replay(seq[0], K, seq[1:])
        lam_a = torch.zeros(sim.total, dtype=torch.float32, device="cuda")
        sim.view(lam_a).fill_(1e-3)
        lam_b = torch.zeros_like(lam_a)
        N = w.n_species
        grad = torch.zeros(N * (N - 1) // 2 + 3, dtype=torch.float64, device="cuda")
        sim.adjoint_run(seq, K, lam_a, lam_b, grad)      # warm (captures its graph)
        e0, e1 = _events()
        torch.cuda.synchronize()
        e0.record(sim.stream)
        sim.adjoint_run(seq, K, lam_a, lam_b, grad)
        e1.record(sim.stream)
        torch.cuda.synchronize()
        reverse_us = e0.elapsed_time(e1) * 1e3 / K
        fwd_us = _timed_steps(sim, 50, 5) * 1e3 / 50
        species_nodes = w.nx * w.ny * w.nz * N
        sim.close()
        del seq
        torch.cuda.empty_cache()
        # a D3Q19 reverse step reads f~(t-1) and mu, writes mu: 3 x 19 floats
        out[name] = {"steps": K, "species_nodes": species_nodes, "reverse_us_per_step": reverse_us,
                     "forward_us_per_step": fwd_us, "reverse_over_forward": reverse_us / fwd_us,
                     "reverse_roofline": roofline(None, 228 * species_nodes, reverse_us * 1e-3, 1)}
    return out


# -------------------------------------------------------------- CPU baseline
def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _oracle_rate(tubes, budget_s):
    """MLUPS x species of the oracle over whole tubes of the batch (all rows),
    a bounded number of steps each."""
    import torch
    from oracle import evd
    from oracle.lattice import DTYPE
    total_nodes, total_steps, total_s = 0, 0, 0.0
    for w in tubes:
        m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                      w.tau1, g=w.g, walls=w.walls, n0=w.n0)
        with torch.no_grad():
            f = evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE))
            f = evd.step(m, f)                    # warm (thread pool, allocator)
            t0 = time.perf_counter()
            f = evd.run(m, f, 2)
            per = (time.perf_counter() - t0) / 2
            n = max(1, int(budget_s / len(tubes) / max(per, 1e-6)))
            t0 = time.perf_counter()
            f = evd.run(m, f, n)
            dt = time.perf_counter() - t0
        total_nodes += w.nodes * w.n_species * n
        total_steps += n
        total_s += dt
    return total_nodes / (total_s * 1e6), total_steps, total_s


def cpu_baseline(budget_s=12.0):
    """The FP64 oracle, as it stands, on this host: three whole tubes of the
    batch (the first, a short and a long one), with every thread torch uses
    and with one thread."""
    import torch
    import lbm_workloads as W
    tubes = W.batched_tubes()
    sample = [tubes[0], tubes[206], tubes[168]]
    threads = torch.get_num_threads()
    v, n, s = _oracle_rate(sample, budget_s)
    torch.set_num_threads(1)
    v1, n1, s1 = _oracle_rate(sample, budget_s)
    torch.set_num_threads(threads)
    names = ", ".join(f"tube {k} ({w.nx}x{w.ny})" for k, w in zip((0, 206, 168), sample))
    return {"value": v, "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"{names} of the 512-tube batch, whole tubes, FP64: {n} steps in "
                      f"{s:.1f} s with {threads} threads; {n1} steps in {s1:.1f} s with 1",
            "single_thread_value": v1, "cpu_model": cpu_model(), "nproc": os.cpu_count()}


# ---------------------------------------------------------------------- main
def workload(name):
    import lbm_workloads as W
    if name == "c1":
        return W.ternary_gravity()
    if name == "c1_hbm":
        return W.ternary_gravity(16384, 1024, 500, name="ternary_gravity_16384x1024")
    if name == "c2":
        return W.layer_mixing_3d()
    raise SystemExit(f"unknown workload {name}")


def sub_tube_hbm(copy_best, variants=True, tuning=None):
    import dataclasses
    import torch
    w = workload("c1_hbm")
    steps = 500
    ms, drift, tune = time_lattice(w, steps, 20, tuning=tuning)
    per = bytes_per_species_node(w.lattice) * w.nodes * w.n_species
    rec = {"workload": w.name, "steps": steps, "tuning": tune,
           "value": w.nodes * w.n_species * steps / (ms * 1e3), "unit": UNIT,
           "ms_per_step": ms / steps, "mass_drift_timed_run": drift,
           "roofline": roofline(w.name, per, ms, steps, tune, copy_best),
           "accuracy": tube_accuracy_vs_oracle(w, tune, 100)}
    if variants:
        res = {}
        for name, wv, accel in (
                ("forcing_1", dataclasses.replace(w, forcing="diff"), None),
                ("forcing_2", dataclasses.replace(w, forcing="full"), None),
                ("force_field", dataclasses.replace(w, g=[0.0, 0.0, 0.0]), "field"),
                ("equilibrium_boundary", dataclasses.replace(w, wall_kind="equilibrium"), None)):
            tun = None
            if wv.wall_kind == "equilibrium":
                tun = tune if tune[4] == 0 else (256, 1, 32, 0, 0)
            if accel == "field":
                accel = torch.empty((2, w.nz, w.ny, w.nx), dtype=torch.float32, device="cuda")
                accel[0] = w.g[0]
                accel[1] = w.g[1]
            msv, dv, tv = time_lattice(wv, 100, 10, tuning=tun, accel=accel)
            res[name] = {"value": w.nodes * w.n_species * 100 / (msv * 1e3), "unit": UNIT,
                         "ms_per_step": msv / 100, "steps": 100, "mass_drift": dv,
                         "tuning": tv}
            del accel
        rec["variants"] = res
    return rec


def sub_tube_llc(tuning=None):
    w = workload("c1")
    steps = 2000
    ms, drift, tune = time_lattice(w, steps, 200, tuning=tuning)
    per = bytes_per_species_node(w.lattice) * w.nodes * w.n_species
    return {"workload": w.name, "steps": steps, "tuning": tune,
            "value": w.nodes * w.n_species * steps / (ms * 1e3), "unit": UNIT,
            "ms_per_step": ms / steps, "mass_drift_timed_run": drift,
            "roofline": roofline(w.name, per, ms, steps, tune, bound="llc"),
            "note": "both population buffers (7.1 MB each) stay in the 256 MB last-level "
                    "cache: the rate is against the HBM peak for reference only",
            "accuracy": tube_accuracy_vs_golden(w, tune)}


def sub_layer_3d(copy_best, tuning=None):
    w = workload("c2")
    steps = 200
    ms, drift, tune = time_lattice(w, steps, 20, tuning=tuning)
    per = bytes_per_species_node(w.lattice) * w.nodes * w.n_species
    return {"workload": w.name, "steps": steps, "tuning": tune,
            "value": w.nodes * w.n_species * steps / (ms * 1e3), "unit": UNIT,
            "ms_per_step": ms / steps, "mass_drift_timed_run": drift,
            "roofline": roofline(w.name, per, ms, steps, tune, copy_best),
            "accuracy": layer_accuracy_crops(w, tune)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-sub", action="store_true", help="headline only (no sub-records)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the 10,000-step gate")
    ap.add_argument("--tuning", help="fixed execution shape bx,by,rows,persistent,variant")
    ap.add_argument("--only", choices=["batched", "batched_per_lattice", "tube_hbm", "tube_llc",
                                       "layer_3d", "adjoint", "adjoint_hbm", "adjoint_3d",
                                       "copy"],
                    help="run one leg alone and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    fixed = [int(v) for v in args.tuning.split(",")] if args.tuning else None

    if args.only:
        if args.only == "copy":
            res = copy_sweep()
        elif args.only in ("batched", "batched_per_lattice"):
            mode = 1 if args.only == "batched" else 0
            res = time_batched(args.steps, args.warmup, modes=(mode,), tuning=fixed)
        elif args.only == "tube_hbm":
            res = sub_tube_hbm(None, variants=False, tuning=fixed)
        elif args.only == "tube_llc":
            res = sub_tube_llc(tuning=fixed)
        elif args.only == "layer_3d":
            res = sub_layer_3d(None, tuning=fixed)
        elif args.only == "adjoint_3d":
            res = time_adjoint_3d()
        elif args.only == "adjoint":
            res = time_adjoint()
        else:
            res = time_adjoint(4096, 1024, 200, 100, fwd_bwd=False)
        print(json.dumps(res), flush=True)
        return

    t_start = time.perf_counter()
    copy = copy_sweep()
    bt = time_batched(args.steps, args.warmup, modes=(1,), tuning=fixed)
    ms = bt["ms"][1]
    tune = bt["tuning"]
    nodes, N = bt["nodes"], 3
    per = bytes_per_species_node("D2Q9") * nodes * N
    line = {
        "metric": METRIC,
        "value": nodes * N * args.steps / (ms * 1e3),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched_512_ternary_tubes", "lattice": "D2Q9",
                   "lattices": bt["lattices"], "nodes": nodes, "species": N,
                   "launch": "one persistent launch per step", "tuning": tune,
                   "parallelism": "single GPU"},
        "roofline": roofline("batched_512_ternary_tubes", per, ms, args.steps, tune,
                             copy["best_GBs"]),
    }
    if not args.no_accuracy:
        line["accuracy"] = batched_accuracy(tune)
    if not args.no_sub:
        sub = {}
        pl = time_batched(min(args.steps, 100), 5, modes=(0,), tuning=tune)
        msl = pl["ms"][0]
        nst = min(args.steps, 100)
        sub["batched_launch_per_lattice"] = {
            "value": nodes * N * nst / (msl * 1e3), "unit": UNIT, "steps": nst,
            "ms_per_step": msl / nst, "tuning": tune,
            "roofline": roofline(None, per, msl, nst)}
        sub["tube_16384x1024"] = sub_tube_hbm(copy["best_GBs"])
        sub["tube_1024x64"] = sub_tube_llc()
        sub["layer_3d_256x128x128"] = sub_layer_3d(copy["best_GBs"])
        sub["adjoint_512x64"] = time_adjoint()
        sub["adjoint_4096x1024"] = time_adjoint(4096, 1024, 200, 100, fwd_bwd=False)
        sub["adjoint_d3q19"] = time_adjoint_3d()
        sub["stream_copy"] = copy
        line["sub"] = sub
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline()
    line["bench_wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
