"""Benchmark of the fused EVD multicomponent LBM step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: the ternary ideal-gas tube with gravity, D2Q9, molar masses
2:28:44, 1024 x 64 nodes, walls at the x ends, periodic in y, g = 1e-6 along x,
seeded pair diffusivities, halves of two uniform compositions (synthetic input
of the paper's Case I structure).  One step is one fused pass (stream with the
second-order interpolation + impermeable walls + moments + tau solve +
collision with forcing) over the whole lattice.  The metric is
MLUPS x species = nodes * species * steps / microseconds, with the state
resident in HBM before the timed region.

The JSON line also carries
  roofline:     HBM roofline of the fused step kernel: algorithmic bytes per
                launch (72 B per species-node for D2Q9: one FP32 read and one
                FP32 write of 9 populations; 152 B for D3Q19) divided by the
                average launch time measured with HIP events on the launch
                stream over the timed region, against 8 TB/s;
  cpu_baseline: the FP64 oracle timed on this host's CPU cores on a bounded
                sample of the same workload;
  accuracy:     max |x_s - x_s(oracle)| of the timed run when the oracle result
                for that step count is stored, and the FP64 mass drift;
  hbm_scale:    the same physics on a 16384 x 1024 tube (3.6 GB per step), where
                the lattice no longer fits the 256 MB last-level cache; its
                "variants" time the same tube with the diffusion-driven
                forcing term (forcing 1), the whole corrected forcing
                (forcing 2) and a per-node force field;
  batched:      512 independent ternary tubes of uneven sizes (22.8 M nodes),
                one persistent launch per step against one launch per tube;
  d3q19:        the 3-D layer workload (D3Q19, 4 species, 256 x 128 x 128,
                152 B per species-node), 200 steps at the autotuned shape;
  adjoint:      gradient of a mole-fraction profile misfit with respect to the
                three pair diffusivities and g on a 512 x 64 ternary tube over
                4000 steps (checkpoints every 100 steps, recomputation, the
                hand-written reverse kernels): time per forward+backward step
                against a plain forward step, and the reverse step's own HBM
                rate (180 B per species-node: kernel A reads the state and the
                adjoint and writes the scratch, kernel B reads the scratch and
                writes the adjoint, 9 floats each).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def bytes_per_species_node(lattice):
    return 2 * 4 * (9 if lattice == "D2Q9" else 19)


def workload(name):
    import lbm_workloads as W
    if name in ("ternary_gravity_1024x64", "c1"):
        return W.ternary_gravity()
    if name in ("ternary_gravity_16384x1024", "c1_hbm"):
        return W.ternary_gravity(16384, 1024, 500, name="ternary_gravity_16384x1024")
    if name in ("layer_mixing_3d_256x128x128", "c2", "3d"):
        return W.layer_mixing_3d()
    if name in ("binary_erf_200x4", "c0"):
        return W.binary_erf()
    raise SystemExit(f"unknown workload {name}")


def time_gpu(w, steps, warmup, autotune=False, tuning=None, accel=None):
    import numpy as np
    import torch
    from paper_2504_07059_amd import lbm

    p = lbm.params_from_workload(w)
    x0 = w.x0()
    if autotune and tuning is None:
        tmp = lbm.LbmMc(p, x0, accel=accel)
        tmp.autotune(reps=5)
        tmp.close()
    sim = lbm.LbmMc(p, x0, accel=accel)
    if tuning is not None:
        sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(warmup)
    sim.prepare(steps)   # graph capture is host work: keep it out of the timed region
    sim.sync()
    stream = sim.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    sim.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    ms = ev0.elapsed_time(ev1)
    out = sim.moments()
    drift = float(np.abs(out["mass"][0] / m0 - 1).max())
    return sim, out, ms, wall, drift


def time_variants(wh, tuning, steps=100, warmup=10):
    """The HBM-scale workload under the optional physics of the library, each
    at the execution shape the autotuner picks for it (the best shape differs
    between them): the diffusion-driven forcing term (forcing 1), the whole
    corrected forcing (forcing 2: a density pre-pass plus gradients), a force
    field k(x) read at every node in place of g (the same values as g, so the
    physics is the plain step's), and the equilibrium comparison boundary in
    place of the Appendix A walls (one thread per column: the plain step's
    shape when that is one, else 256-column tiles of 32 layers)."""
    import dataclasses
    import torch
    res = {}
    for name, w, accel in (
            ("forcing_1", dataclasses.replace(wh, forcing="diff"), None),
            ("forcing_2", dataclasses.replace(wh, forcing="full"), None),
            ("force_field", dataclasses.replace(wh, g=[0.0, 0.0, 0.0]), "field"),
            ("equilibrium_boundary", dataclasses.replace(wh, wall_kind="equilibrium"), None)):
        tun = None
        if w.wall_kind == "equilibrium":
            tun = tuning if tuning is not None and tuning[4] == 0 else (256, 1, 32, 0, 0)
        if accel == "field":
            accel = torch.empty((2, wh.nz, wh.ny, wh.nx), dtype=torch.float32, device="cuda")
            accel[0] = wh.g[0]
            accel[1] = wh.g[1]
        sim, out, ms, wall, drift = time_gpu(w, steps, warmup, autotune=tun is None,
                                             tuning=tun, accel=accel)
        used = list(sim.get_tuning())
        sim.close()
        res[name] = {"value": wh.nodes * wh.n_species * steps / (ms * 1e3),
                     "unit": "MLUPS x species", "ms_per_step": ms / steps, "steps": steps,
                     "mass_drift": drift, "tuning": used}
        del accel
    return res


def accuracy_vs_golden(w, t=20000, tuning=None):
    """Paired accuracy gate: a fresh run of the same workload to step t (at the
    same execution shape) against the stored FP64 oracle result."""
    import numpy as np
    from paper_2504_07059_amd import lbm
    path = os.path.join(ROOT, "tests", "golden", "ternary_gravity.json")
    if w.name != "ternary_gravity_1024x64" or not os.path.exists(path):
        return None, None
    g = json.load(open(path))["checkpoints"][str(t)]
    sim = lbm.LbmMc(lbm.params_from_workload(w), w.x0())
    if tuning is not None:
        sim.set_tuning(*tuning)
    m0 = sim.moments(fields=False)["mass"][0].copy()
    sim.step(t)
    out = sim.moments()
    sim.sync()
    x = sim.field(out, "x").double().cpu().numpy()
    dx = float(np.abs(x[:, 0] - np.array(g["x"])[:, None, :]).max())
    drift = float(np.abs(out["mass"][0] / m0 - 1).max())
    sim.close()
    return dx, drift


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle, as it stands, on this host's cores: a bounded number of
    steps of the same workload (initial state included in the setup, not in
    the timing)."""
    import torch
    from oracle import evd
    from oracle.lattice import DTYPE
    m = evd.Model(w.lattice, w.nx, w.ny, w.nz, w.masses, torch.tensor(w.diff, dtype=DTYPE),
                  w.tau1, g=w.g, walls=w.walls, n0=w.n0)
    f = evd.initial_populations(m, torch.tensor(w.x0(), dtype=DTYPE))
    f = evd.step(m, f)                       # warm (thread pool, allocator)
    t0 = time.perf_counter()
    f = evd.run(m, f, 3)
    per = (time.perf_counter() - t0) / 3
    n = max(1, int(budget_s / max(per, 1e-6)))
    t0 = time.perf_counter()
    f = evd.run(m, f, n)
    dt = time.perf_counter() - t0
    value = w.nodes * w.n_species * n / (dt * 1e6)
    return {"value": value, "unit": "MLUPS x species", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{w.name}: {n} full-lattice FP64 steps in {dt:.1f} s "
                      f"({torch.get_num_threads()} threads)"}


def time_batched(steps, warmup):
    """The 512-tube batch: one persistent launch per step (autotuned shape) and,
    for comparison, one launch per tube per step, both under captured graphs."""
    import numpy as np
    import torch
    import lbm_workloads as W
    from paper_2504_07059_amd import lbm
    tubes = W.batched_tubes()
    params = [lbm.params_from_workload(w) for w in tubes]
    x0 = W.concat_x0(tubes)
    nodes = sum(w.nodes for w in tubes)
    tmp = lbm.LbmMc(params, x0)
    tmp.autotune(reps=3)
    tmp.close()
    sim = lbm.LbmMc(params, x0)
    m0 = sim.moments(fields=False)["mass"].copy()
    res = {}
    for mode in (1, 0):
        sim.set_batched_mode(mode)
        sim.step(warmup)
        sim.prepare(steps)
        sim.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(sim.stream)
        sim.step(steps)
        ev1.record(sim.stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        res[mode] = ms
    drift = float(np.abs(sim.moments(fields=False)["mass"] / m0 - 1).max())
    tune = sim.get_tuning()
    sim.close()
    per_launch = bytes_per_species_node("D2Q9") * nodes * 3
    out = {"workload": "batched_512_ternary_tubes", "lattices": len(tubes), "nodes": nodes,
           "steps": steps, "tuning": list(tune), "mass_drift": drift}
    for mode, key in ((1, "one_launch"), (0, "launch_per_lattice")):
        ms = res[mode]
        out[key] = {"value": nodes * 3 * steps / (ms * 1e3), "unit": "MLUPS x species",
                    "ms_per_step": ms / steps,
                    "achieved_GBs": per_launch / (ms * 1e-3 / steps) / 1e9}
    return out


def time_adjoint(steps=4000, K=100):
    import torch
    import lbm_workloads as W
    from paper_2504_07059_amd import adjoint as A
    from paper_2504_07059_amd import lbm
    truth, ev = W.adjoint_tube(steps=steps)
    N = ev.n_species
    pairs = lambda w: [w.diff[i][j] for i in range(N) for j in range(i + 1, N)]
    prob = A.Problem("D2Q9", ev.nx, ev.ny, 1, ev.masses, ev.tau1, ev.walls, ev.x0(), steps,
                     checkpoint_every=K)
    f64 = torch.float64
    with torch.no_grad():
        target = A.evolve(torch.tensor(pairs(truth), dtype=f64),
                          torch.tensor(truth.g, dtype=f64), prob)

    def events():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # plain forward on the same lattice
    sim = lbm.LbmMc(lbm.params_from_workload(ev), ev.x0())
    sim.step(200)
    sim.prepare(steps)
    sim.sync()
    e0, e1 = events()
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1)
    # reverse kernels alone: one segment of K steps from a recomputed sequence
    stride = (sim.total + 63) // 64 * 64
    seg = torch.empty((K, stride), dtype=torch.float32, device=sim.fa.device)
    seg[0, : sim.total].copy_(sim.buffers()[0])
    sim.replay(seg[0], K - 1, seg[1:])               # warm (captures its graph)
    e0, e1 = events()
    e0.record(sim.stream)
    sim.replay(seg[0], K - 1, seg[1:])
    e1.record(sim.stream)
    lam_a = torch.zeros(sim.total, dtype=torch.float32, device=seg.device)
    lam_b = torch.zeros_like(lam_a)
    sim.view(lam_a).fill_(1e-3)
    grad = torch.zeros(N * (N - 1) // 2 + 3, dtype=f64, device=seg.device)
    sim.adjoint_run(seg, K, lam_a, lam_b, grad)      # warm
    e2, e3 = events()
    e2.record(sim.stream)
    sim.adjoint_run(seg, K, lam_a, lam_b, grad)
    e3.record(sim.stream)
    torch.cuda.synchronize()
    replay_us = e0.elapsed_time(e1) * 1e3 / (K - 1)
    reverse_us = e2.elapsed_time(e3) * 1e3 / K
    sim.close()
    # whole forward + backward of the misfit: one untimed pass (first use of
    # the adjoint kernels and of autograd), then the timed one
    def fwd_bwd():
        p_t = torch.tensor(pairs(ev), dtype=f64, requires_grad=True)
        g_t = torch.tensor(ev.g, dtype=f64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = A.profile_misfit(A.evolve(p_t, g_t, prob), target)
        L.backward()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, L, p_t, g_t

    wall_cold = fwd_bwd()[0]
    wall_fb, L, p_t, g_t = fwd_bwd()
    species_nodes = ev.nodes * N
    return {"workload": f"adjoint_tube_{ev.nx}x{ev.ny}", "steps": steps, "checkpoint_every": K,
            "forward_ms_per_step": ms_fwd / steps,
            "fwd_bwd_ms_per_step": wall_fb * 1e3 / steps,
            "fwd_bwd_over_forward": wall_fb * 1e3 / ms_fwd,
            "fwd_bwd_first_call_ms_per_step": wall_cold * 1e3 / steps,
            "reverse_step_us": reverse_us, "replay_step_us": replay_us,
            "reverse_GBs": 180 * species_nodes / (reverse_us * 1e-6) / 1e9,
            "loss": L.item(), "grad_pairs": p_t.grad.tolist(), "grad_g": g_t.grad.tolist()}


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device-to-device copy of known size (reads and writes nbytes per
    launch): the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"copy_bytes": nbytes, "reps": reps}


KERNEL_SOURCES = ("step.hip", "kernels.hpp", "collide.hpp", "lattice.hpp", "common.hpp")


def measured_traffic(workload_name, tuning):
    """HBM bytes per launch of the fused step from the committed counter
    summaries (FETCH_SIZE + WRITE_SIZE, copy-calibrated), if one was taken for
    this workload and execution shape from the current kernel sources; else
    None."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_07059_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()[:16]
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


def roofline(w, ms, steps, tuning=None):
    per_launch = bytes_per_species_node(w.lattice) * w.nodes * w.n_species
    avg_s = ms * 1e-3 / steps
    achieved = per_launch / avg_s / 1e9
    traffic = measured_traffic(w.name, tuning) if tuning is not None else None
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
            "bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--workload", default="ternary_gravity_1024x64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-hbm", action="store_true", help="skip the HBM-scale companion run")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-tube batch")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-3d", action="store_true", help="skip the D3Q19 layer workload")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the library's default execution shape instead of the autotuned one")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the paired accuracy run against the stored oracle result")
    ap.add_argument("--tuning", help="fixed execution shape bx,by,rows,persistent (no autotune)")
    ap.add_argument("--only", choices=["batched", "adjoint", "copy"],
                    help="run one companion leg alone and print its JSON (for profiling)")
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
    if args.only:
        if args.only == "copy":
            res = copy_calibration()
        else:
            res = time_batched(args.steps, args.warmup) if args.only == "batched" else time_adjoint()
        print(json.dumps(res), flush=True)
        return

    w = workload(args.workload)
    fixed = [int(v) for v in args.tuning.split(",")] if args.tuning else None
    sim, out, ms, wall, drift = time_gpu(w, args.steps, args.warmup, not args.no_autotune, fixed)
    tune = sim.get_tuning()
    sim.close()
    acc_dx, acc_drift = (None, None) if args.no_accuracy else accuracy_vs_golden(w, tuning=tune)
    value = w.nodes * w.n_species * args.steps / (ms * 1e3)
    line = {
        "metric": "MLUPS x species (fused EVD-LBM step, FP32 state)",
        "value": value,
        "unit": "MLUPS x species",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": w.lattice, "nx": w.nx, "ny": w.ny,
                   "nz": w.nz, "species": w.n_species, "masses": w.masses,
                   "walls": w.walls, "g": w.g, "tuning": list(tune),
                   "parallelism": "single GPU"},
        "roofline": roofline(w, ms, args.steps, tune),
        "accuracy": {"max_dx_vs_oracle_t20000": acc_dx, "mass_drift_t20000": acc_drift,
                     "mass_drift_timed_run": drift},
        "wall_s": wall,
    }
    if not args.no_hbm and w.name.startswith("ternary_gravity_1024"):
        wh = workload("c1_hbm")
        s2, o2, ms2, wall2, drift2 = time_gpu(wh, wh.steps, 20, autotune=True)
        t2 = s2.get_tuning()
        s2.close()
        line["hbm_scale"] = {
            "workload": wh.name, "steps": wh.steps,
            "value": wh.nodes * wh.n_species * wh.steps / (ms2 * 1e3),
            "unit": "MLUPS x species", "ms_per_step": ms2 / wh.steps,
            "roofline": roofline(wh, ms2, wh.steps, t2), "mass_drift": drift2,
            "tuning": list(t2), "variants": time_variants(wh, t2)}
    if not args.no_batched and w.name.startswith("ternary_gravity_1024"):
        line["batched"] = time_batched(200, 20)
    if not args.no_3d and w.name.startswith("ternary_gravity_1024"):
        w3 = workload("c2")
        s3, o3, ms3, wall3, drift3 = time_gpu(w3, 200, 20, autotune=True)
        t3 = s3.get_tuning()
        s3.close()
        line["d3q19"] = {
            "workload": w3.name, "steps": 200,
            "value": w3.nodes * w3.n_species * 200 / (ms3 * 1e3),
            "unit": "MLUPS x species", "ms_per_step": ms3 / 200,
            "roofline": roofline(w3, ms3, 200, t3), "mass_drift": drift3, "tuning": list(t3)}
    if not args.no_adjoint and w.name.startswith("ternary_gravity_1024"):
        line["adjoint"] = time_adjoint()
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
