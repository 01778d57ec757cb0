#!/usr/bin/env python3
"""Throughput of the coupled GP phase-field / lattice-Boltzmann step on one
MI355X, in MLUPS (million lattice-cell updates per second; one update = one
cell through one whole coupled step), FP32 and FP64 side by side, with the
HBM roofline of the dominant kernel and the FP64 CPU oracle as a baseline.

Workload: the 3D binary-alloy dendrite with natural convection, 256^3 cells,
D3Q19, two phases, one solute, FP32 storage and arithmetic (the
configuration the HBM-roofline target is stated on); the same grid in FP64
is timed beside it.  Inputs are synthetic (seed + noise from a fixed seed)
and resident in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]
                    [--no-adjoint] [--no-drift]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def bytes_per_lup(cfg, s):
    """Algorithmic bytes per lattice update: the state read once and written
    once, phi counted N-1 times (sum phi = 1), U and T derived:
    2 (N - 1 + nc + Q) s."""
    Q = 9 if cfg["dim"] == 2 else (27 if cfg.get("lattice") == "D3Q27" else 19)
    return 2 * (cfg["N"] - 1 + cfg["nc"] + Q) * s


def prewarm(sim, min_ms=100.0):
    """Untimed steps until at least min_ms of device work has run, so that
    the clocks have left their idle state before the timed window; returns
    the steps run."""
    import torch
    n, done = 1, 0
    t0 = time.perf_counter()
    while True:
        sim.step(n)
        torch.cuda.synchronize()
        done += n
        if (time.perf_counter() - t0) * 1e3 >= min_ms:
            return done
        n *= 2


def run_gpu(cfg, precision, steps, warmup, kernel_steps=50, advance=0):
    """Throughput over `steps` steps launched back to back (no host
    synchronisation inside the timed region), then the mean duration of each
    kernel over `kernel_steps` more steps, every launch bracketed by HIP events
    on the library's stream (torch's current stream).  Before the timed
    window: `advance` steps (to time a grown microstructure), `warmup` steps
    and an untimed run of at least 100 ms (clock warm-up)."""
    import torch
    from paper_2608_26908_amd.gpf import Sim
    sim = Sim(cfg, precision=precision)
    if advance:
        sim.step(advance)
    sim.step(warmup)
    torch.cuda.synchronize()
    pre = prewarm(sim)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    t0 = time.perf_counter()
    sim.step(steps)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    ks = max(1, min(kernel_steps, steps))
    k_phi_ms, k_mulbm_ms = sim.step_timed(ks)
    cells = sim.cells
    sol = sim.reduce("solute")
    sim.close()
    return dict(ms_per_step=ms / steps, wall_s=wall, cells=cells,
                k_phi_ms=k_phi_ms / ks, k_mulbm_ms=k_mulbm_ms / ks, prewarm_steps=pre,
                mlups=cells * steps / (ms * 1e-3) / 1e6, solute=[float(v) for v in sol])


def copy_bandwidth(mib=1024, reps=20):
    """Read + write GB/s of a plain device-to-device copy of `mib` MiB: the
    bandwidth a streaming kernel can reach on this device, beside the
    published peak."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        b.copy_(a)
    stop.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / reps
    del a, b
    return 2 * mib * (1 << 20) / (ms * 1e-3) / 1e9


def run_adjoint(cfg, precision, steps, K, names, target_changes):
    """Wall time of the forward run and of the reverse sweep (segment
    recompute + adjoint kernels), same stream, for the loss L = 1/2 sum (phi -
    phi_t)^2 against a target run with other parameters: the library forms L
    (GPF_LOSS) and its seed dL/dphi on the device.  The timed sweep is the
    second one of the same recording: the first allocates the tapes and the
    adjoint buffers, which later sweeps (an inversion loop) reuse."""
    import torch
    from paper_2608_26908_amd.gpf import Sim
    t = Sim(dict(cfg, **target_changes), precision=precision)
    t.step(steps)
    target = t.read_device("phi").double()
    t.close()
    sim = Sim(cfg, precision=precision)
    sim.set_target(target)
    sim.step(2)  # warm-up of every kernel
    torch.cuda.synchronize()
    ck = sim.checkpoint()
    prewarm(sim)
    sim.restore(ck)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    sim.restore(ck)
    sim.record(K)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    loss = sim.reduce("loss")
    seed = sim.loss_seed()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint(seed, names)
    t_cold = time.perf_counter() - t0
    t0 = time.perf_counter()
    grads = sim.adjoint(seed, names)
    t_adj = time.perf_counter() - t0
    sim.close()
    return dict(forward_ms=round(t_plain * 1e3, 2), forward_recording_ms=round(t_fwd * 1e3, 2),
                adjoint_ms=round(t_adj * 1e3, 2), ratio=round(t_adj / t_plain, 3),
                first_sweep_ms=round(t_cold * 1e3, 2),
                timed="second reverse sweep of the recording (the first allocated tapes and adjoint buffers)",
                loss=loss, grads=dict(zip(names, [float(g) for g in grads])))


def solute_drift(cfg, precision, steps=10000):
    """Relative change of the FP64 solute total over `steps` steps (walls and
    periodic axes conserve it exactly in exact arithmetic)."""
    import numpy as np
    from paper_2608_26908_amd.gpf import Sim
    sim = Sim(cfg, precision=precision)
    s0 = sim.reduce("solute")
    sim.step(steps)
    s1 = sim.reduce("solute")
    sim.close()
    return float(np.max(np.abs(s1 - s0) / np.abs(s0)))


def cpu_model():
    """The host CPU's model name (lscpu), or the platform's processor string."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(cfg, steps=7):
    """The FP64 oracle as it stands, on this host's cores, on bounded samples
    of the same workload: all cores on the full grid (one untimed step, then
    `steps` timed steps), and one thread on a 128^3 block of it (same
    parameters, seed at the same relative place; one untimed step, two timed)."""
    from oracle import pyoracle
    from paper_2608_26908_amd.workloads import cells as ncells, scaled
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sim = pyoracle.OracleSim(cfg, threads=threads)
    sim.step(1)
    t0 = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t0
    sub = scaled(cfg["name"], [128] * cfg["dim"])
    one = pyoracle.OracleSim(sub, threads=1)
    one.step(1)
    t1 = time.perf_counter()
    one.step(2)
    dt1 = time.perf_counter() - t1
    return {"value": round(ncells(cfg) * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu": cpu_model(),
            "sample": f"full {cfg['n']} grid, FP64 oracle, {steps} timed steps after 1 untimed step "
                      f"({dt:.1f} s)",
            "one_thread": {"value": round(ncells(sub) * 2 / dt1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                           "sample": f"{sub['n']} block of the workload, 2 timed steps after 1 untimed "
                                     f"({dt1:.1f} s)"}}


def traffic_record(name, precision):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_mulbm_{name}_{precision}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2608_26908_amd.build import source_digest
        if rec.get("source_digest") != source_digest():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="dendrite3d")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-drift", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the shrinkage, D3Q27, moving-frame and four-phase lines (profiling runs)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a device-to-device copy of this many MiB (a kernel of known "
                         "traffic to calibrate the HBM byte counters of a profiler run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the single-GPU throughput is the figure reported)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2608_26908_amd.workloads import workload
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = workload(args.workload)
    if args.copy_calib_mib:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(f"# copy calibration: 3 copies of {args.copy_calib_mib} MiB", file=sys.stderr, flush=True)
        del a, b
    r32 = run_gpu(cfg, "fp32", args.steps, args.warmup)
    print(f"# fp32: {r32['mlups']:.1f} MLUPS, {r32['ms_per_step']:.3f} ms/step "
          f"(k_phi {r32['k_phi_ms']:.3f} ms, k_mulbm {r32['k_mulbm_ms']:.3f} ms)", file=sys.stderr,
          flush=True)
    # the same workload grown: the dendrite after its 5000 configured steps
    late = None
    if not args.no_extra:
        late = run_gpu(cfg, "fp32", args.steps, args.warmup, advance=cfg.get("steps", 5000))
        print(f"# fp32 after {cfg.get('steps', 5000)} steps: {late['mlups']:.1f} MLUPS, "
              f"{late['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        r64 = run_gpu(cfg, "fp64", args.steps, args.warmup)
        print(f"# fp64: {r64['mlups']:.1f} MLUPS, {r64['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)

    rs = r27 = rf0 = rf1 = r4 = None
    c27 = workload(args.workload, lattice="D3Q27")
    c4 = workload("eutectic4_3d")
    if not args.no_extra:
        # the shrinkage force of Eq. (shrinkage) on (rho_s / rho_l = 1.2): the same
        # workload, extra arithmetic on values the kernel already holds
        rs = run_gpu(workload(args.workload, eta=[0.2, 0.0, 0.0]), "fp32", min(args.steps, 100),
                     args.warmup)
        print(f"# fp32 with shrinkage: {rs['mlups']:.1f} MLUPS, {rs['ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)
        # the paper's own 3D lattice, D3Q27 (Table LBM_Schemes), on the same workload
        r27 = run_gpu(c27, "fp32", min(args.steps, 100), args.warmup)
        print(f"# fp32 D3Q27: {r27['mlups']:.1f} MLUPS, {r27['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
        # the moving frame of Case 2 on the eutectic (1024 x 512): a front search
        # every 100 steps (one synchronisation) and the shifts it triggers
        e2 = workload("eutectic2d")
        rf0 = run_gpu(e2, "fp32", 1000, 50)
        rf1 = run_gpu(dict(e2, frame_every=100, frame_front=16), "fp32", 1000, 50)
        print(f"# eutectic2d fp32: {rf0['mlups']:.1f} MLUPS, with the moving frame {rf1['mlups']:.1f}",
              file=sys.stderr, flush=True)
        # four phases (three solids and the liquid, Case 3), 192 x 192 x 384 D3Q19
        r4 = run_gpu(c4, "fp32", min(args.steps, 100), args.warmup)
        print(f"# fp32 four phases: {r4['mlups']:.1f} MLUPS, {r4['ms_per_step']:.3f} ms/step", file=sys.stderr,
              flush=True)
    copy_gbs = copy_bandwidth()
    print(f"# device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    # the achievable side of the roofline: the population update's access
    # patterns without its arithmetic, on the same grid (library kernels)
    from paper_2608_26908_amd.gpf import bandwidth_probe
    ceil, bufs = {}, None
    for pat in ("copy19", "pull19", "pull19_zmarch"):
        ceil[pat], a, b = bandwidth_probe(pat, cfg["n"], reps=20, buffers=bufs)
        bufs = (a, b)
    del bufs, a, b
    print(f"# access-pattern ceilings (GB/s): " + ", ".join(f"{k} {v:.0f}" for k, v in ceil.items()),
          file=sys.stderr, flush=True)
    b32 = bytes_per_lup(cfg, 4)
    cells = r32["cells"]
    achieved = b32 * cells / (r32["k_mulbm_ms"] * 1e-3) / 1e9
    traffic = traffic_record(args.workload, "fp32")
    line = {
        "metric": "MLUPS of coupled PF+LBM step (FP32 vs FP64) + % HBM roofline; adjoint/forward cost",
        "value": round(r32["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: 3D binary-alloy dendrite with natural convection, "
                               f"{'x'.join(str(v) for v in cfg['n'])} cells, D3Q19, 2 phases, 1 solute, "
                               "FP32 storage (f as f - w rho0)",
                   "grid": cfg["n"], "lattice": "D3Q19", "phases": cfg["N"], "solutes": cfg["nc"],
                   "precision": "fp32"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": "k_mulbm_z (chemical potential + LBM collide/stream, z-marching)",
                     "bytes_per_lup": b32,
                     "step_frac": round(b32 * cells / (r32["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "copy_GBps": round(copy_gbs, 1),
                     "pattern_ceilings_GBps": {k: round(v, 1) for k, v in ceil.items()}},
        "kernels_ms": {"k_phi": round(r32["k_phi_ms"], 4), "k_mulbm": round(r32["k_mulbm_ms"], 4)},
        "timing": f"{args.warmup} warm-up steps, then an untimed run of {r32['prewarm_steps']} steps "
                  "(>= 100 ms of device work) before the timed window",
    }
    if late:
        line["grown"] = {"workload": f"{args.workload} after its {cfg.get('steps', 5000)} configured steps "
                                     "(grown dendrite)", "value": round(late["mlups"], 2), "unit": "MLUPS",
                         "ms_per_step": round(late["ms_per_step"], 4),
                         "k_phi_ms": round(late["k_phi_ms"], 4), "k_mulbm_ms": round(late["k_mulbm_ms"], 4),
                         "roofline_frac": round(b32 * cells / (late["k_mulbm_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "step_frac": round(b32 * cells / (late["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if not args.no_extra:
        line["shrinkage"] = {"value": round(rs["mlups"], 2), "unit": "MLUPS", "eta": [0.2, 0.0, 0.0],
                             "ms_per_step": round(rs["ms_per_step"], 4),
                             "k_phi_ms": round(rs["k_phi_ms"], 4), "k_mulbm_ms": round(rs["k_mulbm_ms"], 4)}
        line["moving_frame"] = {"workload": "eutectic2d 1024x512 FP32, front search every 100 steps, front kept at 16",
                                "value": round(rf1["mlups"], 2), "unit": "MLUPS",
                                "without_frame": round(rf0["mlups"], 2)}
        b4 = bytes_per_lup(c4, 4)
        line["four_phase"] = {"workload": "eutectic4_3d: 192x192x384 D3Q19, 4 phases, 2 solutes, FP32",
                              "value": round(r4["mlups"], 2), "unit": "MLUPS",
                              "ms_per_step": round(r4["ms_per_step"], 4), "k_phi_ms": round(r4["k_phi_ms"], 4),
                              "k_mulbm_ms": round(r4["k_mulbm_ms"], 4), "bytes_per_lup": b4,
                              "roofline_frac": round(b4 * r4["cells"] / (r4["k_mulbm_ms"] * 1e-3) / 1e9
                                                     / HBM_PEAK_GBS, 4)}
        b27 = bytes_per_lup(c27, 4)
        line["d3q27"] = {"value": round(r27["mlups"], 2), "unit": "MLUPS", "ms_per_step": round(r27["ms_per_step"], 4),
                         "k_phi_ms": round(r27["k_phi_ms"], 4), "k_mulbm_ms": round(r27["k_mulbm_ms"], 4),
                         "bytes_per_lup": b27,
                         "roofline_frac": round(b27 * cells / (r27["k_mulbm_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "step_frac": round(b27 * cells / (r27["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if r64:
        b64 = bytes_per_lup(cfg, 8)
        line["fp64"] = {"value": round(r64["mlups"], 2), "unit": "MLUPS",
                        "ms_per_step": round(r64["ms_per_step"], 4),
                        "k_phi_ms": round(r64["k_phi_ms"], 4), "k_mulbm_ms": round(r64["k_mulbm_ms"], 4),
                        "roofline_frac": round(b64 * cells / (r64["k_mulbm_ms"] * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4)}
    if not args.no_adjoint:
        a2 = workload("adjoint2d")
        line["adjoint"] = dict(
            workload="adjoint2d: 256x256 D2Q9 dendrite, FP32 forward, FP64 gradients, 2000 steps, "
                     "checkpoint every 100",
            **run_adjoint(a2, "fp32", 2000, 100, ["delta", "tau_pf", "D", "gbeta"],
                          dict(delta=[[0, 0.025], [0.025, 0]], tau_pf=1.2, gbeta=[2e-5])))
        print(f"# adjoint2d: ratio {line['adjoint']['ratio']}", file=sys.stderr, flush=True)
        e3 = workload("eutectic3d")
        line["adjoint3d"] = dict(
            workload="eutectic3d: 192x192x384 D3Q19, 3 phases, 2 solutes, FP32 forward, 1000 steps (a tenth "
                     "of the 10^4-step run), checkpoint every 100 (the interval that fits the whole run's "
                     "checkpoints and two tapes in 288 GB)",
            **run_adjoint(e3, "fp32", 1000, 100, ["D", "D1"],
                          dict(D=[[0.0, 0.0], [0.0, 0.0], [1.2, 0.8]])))
        print(f"# adjoint3d: ratio {line['adjoint3d']['ratio']}", file=sys.stderr, flush=True)
    if not args.no_extra:
        # every workload of the paper's configurations, FP32 and FP64 side by
        # side: MLUPS and the step's fraction of the HBM roofline at its own
        # algorithmic bytes per LUP
        per = {}
        for name, steps in (("dendrite2d", 2000), ("eutectic2d", 1000), ("dendrite3d", 50),
                            ("adjoint2d", 2000), ("eutectic3d", 50)):
            wc = workload(name)
            row = {"grid": wc["n"], "phases": wc["N"], "solutes": wc["nc"]}
            for prec, s in (("fp32", 4), ("fp64", 8)):
                r = run_gpu(wc, prec, steps, max(10, steps // 10))
                row[prec] = {"MLUPS": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                             "step_frac": round(bytes_per_lup(wc, s) * r["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
            per[name] = row
            print(f"# {name}: fp32 {row['fp32']['MLUPS']} MLUPS, fp64 {row['fp64']['MLUPS']} MLUPS",
                  file=sys.stderr, flush=True)
        line["configs"] = per
    if not args.no_drift:
        drift = {"dendrite3d_fp32": solute_drift(cfg, "fp32")}
        e2 = workload("eutectic2d")
        for prec in ("fp32", "fp64"):
            drift[f"eutectic2d_{prec}"] = solute_drift(e2, prec)
        line["solute_drift_per_1e4_steps"] = {k: float(f"{v:.3g}") for k, v in drift.items()}
        print(f"# solute drift per 1e4 steps: {line['solute_drift_per_1e4_steps']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
