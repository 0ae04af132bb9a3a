"""Throughput of the dense-suspension time step on one MI355X.

Workload: N = 100 000 bidisperse spheres (radii 1 and 1.4, equal volumes), phi = 0.55, simple
shear rate 1 under Lees-Edwards boundaries, mu = 1, dt = 1e-4, stress sampled every 10 steps,
timed after a pre-shear of one strain unit (10 000 steps) so that the contact network and the
contact history are those of a sheared suspension.  Inputs are seeded synthetic packings
already resident in device memory when timing starts.

Prints one JSON line: particle-steps/s of the graph-replayed step (wall clock between device
synchronisations), the roofline of the dominant kernel (k_pairs) from HIP events recorded on
the library's stream around its launches in a second pass over as many steps, the per-kernel
table, the mixed-precision, batched-sweep and adjoint modes on the same GPU (``modes``), and
the FP64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def pairs_kernel_bytes(N: int, ncell: int, contacts: int, capacity: int) -> float:
    """Algorithmic bytes of one pair-kernel launch (FP64), the per-unit figures of the step's
    compulsory traffic times the units of one launch:
    per particle: the sorted record read (x, u_half, w_half 3 x 24 B, radius 8 B, id 4 B = 84 B),
    F and T written (48 B), its history row count and slot (8 B);
    per contact (each stored once): the old key + stretch read (4 + 24 B) and the new one
    written (4 + 24 B).  ncell and capacity do not enter (kept for the callers)."""
    return N * (84 + 48 + 8) + contacts * (28 + 28)


def cpu_baseline(w, seconds: float = 10.0, label: str = "the same"):
    import oracle
    p = w.params
    threads = oracle.num_threads()
    st, F, T, S = oracle.init_state(p, w.x, w.rad, use_cells=True)
    t0 = time.perf_counter()
    steps = 0
    while True:
        st, *_ = oracle.step(p, st, use_cells=True)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds or steps >= 200:
            break
    N = len(w.rad)
    return {"value": N * steps / el, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} FP64 oracle steps (cell-list pair search, OpenMP) of {label} workload "
                      f"(N={N}), {el:.1f} s"}


def maybe_tune(sim, args):
    """Autotune the launch (its trial steps are ordinary steps, before the warm-up)."""
    if not args.tune:
        return None
    import tempfile

    from paper_2108_01013_amd import tune
    path = args.tune_cache or os.path.join(tempfile.gettempdir(), "dss_tuning_bench.json")
    rec = tune.autotune(sim, trial_steps=args.tune_steps, cache_path=path,
                        log=lambda m: print("# " + m, file=sys.stderr, flush=True))
    return {"choice": rec["tuning"], "ms_per_step": round(rec["ms_per_step"], 5), "cached": rec["cached"],
            "trials": [{"tuning": t["tuning"], "ms_per_step": round(t["ms_per_step"], 5)}
                       for t in rec.get("trials", [])]}


def timed_run(sim, N, args, stress_every, kernels=("k_pairs",), steps=None, warmup=None):
    """Warm-up, then the timed region: `steps` graph-replayed steps between two device
    synchronisations (kernel timing off).  Then, from where that left off, as many steps with HIP
    events around the pair kernel(s) (direct launches: the events are recorded by the launches
    themselves), and a per-kernel breakdown over at most 50 steps.
    Returns (seconds of the timed region, pair-kernel timing, breakdown)."""
    import torch
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    sim.set_timing(False)
    # the host's garbage is collected before the warm-up, and no collection runs from there to
    # the end of the timed region: a collection takes ≈ 50 ms, and the device left idle that
    # long ran the timed steps that followed 3-4 % slower
    gc.collect()
    gc.disable()
    try:
        sim.step(warmup, stress_every=stress_every, sync=True)
        # the graphs of the timed call are captured now, so that it replays them only
        sim.prepare_steps(steps, stress_every=stress_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps, stress_every=stress_every, sync=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    finally:
        gc.enable()
    sim.set_timing(True, kernels=list(kernels))
    sim.step(steps, stress_every=stress_every, sync=True)
    timing = sim.timing()
    sim.set_timing(True)
    sim.step(min(steps, 50), stress_every=stress_every, sync=True)
    breakdown = sim.timing()
    sim.set_timing(False)
    return el, timing, breakdown


def preshear(sim, steps: int, chunk: int = 1000):
    """Shear the box for `steps` steps before timing, in chunks that each end with a check of the
    device error flags (the run stops at the first one)."""
    from paper_2108_01013_amd.dss import DssError
    done = 0
    t0 = time.perf_counter()
    try:
        while done < steps:
            k = min(chunk, steps - done)
            sim.step(k, stress_every=0, sync=True)
            done += k
    except DssError as e:
        print(f"# pre-shear stopped after {done} steps: {e}", file=sys.stderr, flush=True)
        sys.exit(1)
    print(f"# pre-shear: {done} steps in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return done


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pairs_fp64_N100k_hbm_traffic.txt")


def measured_traffic():
    """HBM bytes per k_pairs<double> launch from the committed counter summary, or None once the
    kernel source has changed since the counters were taken."""
    import hashlib
    try:
        vals = {}
        for line in open(TRAFFIC_FILE):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
        src = open(os.path.join(ROOT, "paper_2108_01013_amd", "csrc", "dss_kernels.hpp"), "rb").read()
        if hashlib.sha256(src).hexdigest() != vals.get("kernel_source_sha256"):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def roofline(timing, N, ncell, contacts, capacity, traffic=None):
    ms_pairs, n_pairs_launch = timing["k_pairs"]
    name = timing.get("name", "k_pairs")
    if name != "k_pairs":
        traffic = None      # the counters were taken on the row-tile kernel
    avg_pairs_s = ms_pairs / max(n_pairs_launch, 1) * 1e-3
    bytes_launch = pairs_kernel_bytes(N, ncell, contacts, capacity)
    achieved = bytes_launch / avg_pairs_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None if traffic is None else int(traffic),
            "kernel": name, "avg_launch_us": round(avg_pairs_s * 1e6, 3),
            "bytes_per_launch": int(bytes_launch)}


def kernel_table(breakdown):
    return {k: {"avg_us": round(v[0] / max(v[1], 1) * 1e3, 3), "launches": v[1]} for k, v in breakdown.items()
            if v[1] > 0}


def cached_workload(args, make):
    """The seeded workload, or its copy saved by an earlier run of the same command (profiling
    passes re-run the benchmark; --workload-cache keeps them from regenerating it)."""
    import numpy as np
    if args.workload_cache and os.path.exists(args.workload_cache):
        from paper_2108_01013_amd import synth
        z = np.load(args.workload_cache)
        L = float(z["L"])
        return synth.Workload(str(z["name"]), z["x"], z["rad"], L, synth.default_params([L, L, L]))
    w = make()
    if args.workload_cache:
        np.savez(args.workload_cache, x=w.x, rad=w.rad, L=w.L, name=w.name)
    return w


def copy_probe(nbytes: int = 1 << 28, reps: int = 3):
    """A plain device copy of known size (calibration of the HBM byte counters)."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"# copy probe: {reps} copies of {nbytes} bytes", file=sys.stderr, flush=True)


def run_single(args):
    from paper_2108_01013_amd import synth

    t_gen = time.perf_counter()
    w = cached_workload(args, lambda: synth.config_single_box(N=args.N or 100_000))
    print(f"# workload generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    import torch

    from paper_2108_01013_amd.dss import DSS_FP64, DSS_MIXED, Simulation
    prec = DSS_FP64 if args.precision == "fp64" else DSS_MIXED
    torch.cuda.set_device(0)
    p = dict(w.params)
    physics = []
    if args.rolling:
        p.update(kr=0.05 * p["kn"], mu_r=0.1)
        physics.append("rolling resistance k_r=0.05 k_n mu_r=0.1")
    if args.ec_ranges:
        p.update(ec_ranges=True, hamaker=1e-3)
        physics.append("electro-chemical ranges (repulsion < 20 lambda_D, attraction A=1e-3 < 4 a0)")
    sim = Simulation(p, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    if args.sized:
        sim.set_tuning(sized=True, cell_scale=args.cell_scale or 1.0, wave_class=args.wave_class)
        physics.append(f"size-class stencils (cell scale {args.cell_scale or 1.0}, wavefronts from class {args.wave_class})")
    sim.set_particles(w.x, w.rad)
    N = len(w.rad)
    tuned = maybe_tune(sim, args)
    if args.state_cache and os.path.exists(args.state_cache):
        # the pre-sheared state of an earlier run of the same command (profiling passes)
        sim.load_state(open(args.state_cache, "rb").read())
        sheared = int(sim.info()["step"])
        print(f"# pre-sheared state loaded (time index {sheared})", file=sys.stderr, flush=True)
    else:
        sheared = preshear(sim, args.preshear)
        if args.state_cache:
            with open(args.state_cache, "wb") as f:
                f.write(sim.save_state())
    el, timing, breakdown = timed_run(sim, N, args, 10)
    # the mixed mode continues from here (a host snapshot taken before the timed run would
    # leave its copy in the device's caches and slow the first timed steps)
    blob = sim.save_state() if args.modes else None
    info = sim.info()
    _, sigma_mean, nsamp = sim.read_stress()
    obs = observables_timing(sim) if args.observables else None
    if info["error_flags"]:
        print(f"# device error flags {info['error_flags']}", file=sys.stderr)
        sys.exit(1)
    ncell = int(info["cells"][0] * info["cells"][1] * info["cells"][2])
    ncell *= sim.box_info(0)["size_classes"]
    roof = roofline(timing, N, ncell, info["n_contacts"], info["capacity"],
                    measured_traffic() if args.precision == "fp64" and N == 100_000 and not physics else None)
    if args.sized and roof["kernel"] == "k_pairs":
        roof["kernel"] = "k_pairs_sized"
        roof["traffic"] = None
    table = kernel_table(breakdown)
    sim.close()
    modes = None
    # the inputs of the mode comparison are made after the timed run (their worker processes
    # start afresh, since this process already uses the GPU), so that nothing of them runs
    # before or beside it
    mode_inputs = mode_workloads(args, start_method="spawn") if args.modes else None
    if mode_inputs:
        modes = {"fp64": {"value": round(N * args.steps / el, 1), "ms_per_step": round(el / args.steps * 1e3, 5),
                          "roofline_frac": roof["frac"], "kernel": roof["kernel"]}}
        modes["mixed"] = mode_mixed(w, p, blob, args)
        modes["sweep"] = mode_sweep(*mode_inputs[0], args)
        modes["adjoint"] = mode_adjoint(mode_inputs[1], args)
        base = modes["fp64"]["ms_per_step"] / N
        for k in ("mixed", "sweep", "adjoint"):
            modes[k]["per_particle_step_vs_fp64"] = round(base / (modes[k]["ms_per_step"] / modes[k]["N"]), 4)
    cpu = None if args.no_cpu_baseline else cpu_baseline(w, args.cpu_seconds, "the same N=100k phi=0.55")
    return {
        "metric": "particle-steps/s at N=100k phi=0.55; mixed/batched/adjoint vs plain FP64",
        "value": round(N * args.steps / el, 1), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"single box N={N} bidisperse 1:1.4 equal volume, phi=0.55, LE shear rate 1, "
                               f"mu=1, dt=1e-4, stress every 10 steps, {args.precision}, timed after "
                               f"{sheared} steps of pre-shear, graph-replayed steps"
                               + "".join(", " + x for x in physics),
                   "N": N, "phi": 0.55, "precision": args.precision, "preshear_steps": sheared},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": table,
        "modes": modes,
        "observables_ms": obs,
        "tuning": tuned or None,
        "diagnostics": {"n_pairs": info["n_pairs"], "n_contacts": info["n_contacts"],
                        "contacts_per_particle": round(info["n_contacts"] / N, 4),
                        "max_row_fill": info["max_row_fill"], "capacity": info["capacity"],
                        "cells": info["cells"], "stress_samples": nsamp,
                        "eta_r_mean": float(sigma_mean[0, 1] / (p["eta0"] * p["shear_rate"]))},
    }


def mode_workloads(args, start_method="fork"):
    """Inputs of the mode comparison: the 64-box sweep and the N = 50k adjoint box (the
    sweep's boxes are relaxed in worker processes: forked before the GPU is touched, else
    spawned)."""
    from paper_2108_01013_amd import synth
    t0 = time.perf_counter()
    sweep = synth.config_sweep(B=args.boxes, workers=args.workers, start_method=start_method)
    wa = synth.bidisperse_box(50_000, 0.56, seed=5)
    print(f"# mode workloads generated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return sweep, wa


def mode_mixed(w, p, blob, args):
    """Mixed precision from the sheared state the FP64 run ended in (its snapshot), after at
    least 20 warm-up steps (the snapshot's upload passes through the device's caches)."""
    import torch

    from paper_2108_01013_amd.dss import DSS_MIXED, Simulation
    sim = Simulation(p, precision=DSS_MIXED, stream=torch.cuda.current_stream().cuda_stream)
    sim.set_particles(w.x, w.rad)
    sim.load_state(blob)
    N = len(w.rad)
    el, timing, breakdown = timed_run(sim, N, args, 10, warmup=max(args.warmup, 20))
    info = sim.info()
    ncell = int(info["cells"][0] * info["cells"][1] * info["cells"][2])
    roof = roofline(timing, N, ncell, info["n_contacts"], info["capacity"])
    sim.close()
    return {"value": round(N * args.steps / el, 1), "ms_per_step": round(el / args.steps * 1e3, 5), "N": N,
            "workload": "the FP64 box's pre-sheared state, FP32 pair arithmetic with FP64 gap and sums",
            "roofline": roof, "contacts_per_particle": round(info["n_contacts"] / N, 4)}


def measure_sweep(ws, gds, args, tune: bool, preshear_steps: int):
    import numpy as np
    import torch

    from paper_2108_01013_amd.dss import DSS_FP64, DSS_MIXED, Batch
    prec = DSS_FP64 if args.precision == "fp64" else DSS_MIXED
    params = [dict(w.params, shear_rate=g) for w, g in zip(ws, gds)]
    sim = Batch(params, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    sim.set_particles([w.x for w in ws], [w.rad for w in ws])
    N = sim.N
    tuned = maybe_tune(sim, args) if tune else None
    sheared = preshear(sim, preshear_steps)
    el, timing, breakdown = timed_run(sim, N, args, 10)
    info = sim.info()
    _, sigma_mean, nsamp = sim.read_stress()
    if info["error_flags"]:
        print(f"# device error flags {info['error_flags']}", file=sys.stderr)
        sys.exit(1)
    boxes = [sim.box_info(b) for b in range(sim.B)]
    ncell = int(sum(np.prod(b["cells"]) for b in boxes))
    eta = [float(sigma_mean[b, 0, 1] / (params[b]["eta0"] * gds[b])) for b in range(sim.B)]
    res = dict(N=N, B=sim.B, el=el, sheared=sheared, info=info, nsamp=nsamp, eta=eta, ncell=ncell,
               roof=roofline(timing, N, ncell, info["n_contacts"], info["capacity"]),
               table=kernel_table(breakdown), tuning=tuned or sim.tuning())
    sim.close()
    return res


def mode_sweep(ws, gds, args):
    r = measure_sweep(ws, gds, args, tune=False, preshear_steps=args.sweep_preshear)
    return {"value": round(r["N"] * args.steps / r["el"], 1), "ms_per_step": round(r["el"] / args.steps * 1e3, 5),
            "N": r["N"], "workload": f"{r['B']} boxes, N_b uniform on 2000..50000, phi 0.40..0.58, shear rate "
                                     f"1e-2..1e1, one graph per step, after {r['sheared']} steps of pre-shear",
            "roofline": r["roof"], "contacts_per_particle": round(r["info"]["n_contacts"] / r["N"], 4)}


def observables_timing(sim):
    """Wall time of each observable call after the timed region (each synchronises)."""
    out = {}
    t0 = time.perf_counter()
    sim.observe_start()
    out["observe_start"] = (time.perf_counter() - t0) * 1e3
    sim.step(10, sync=True)
    t0 = time.perf_counter()
    ob = sim.observe()
    out["observe"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    sim.phi_profile(64, 1.2)
    out["phi_profile_64"] = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    h = sim.contact_clusters()
    out["contact_clusters"] = (time.perf_counter() - t0) * 1e3
    out = {k: round(v, 3) for k, v in out.items()}
    nz = [i + 1 for i in range(len(h)) if h[i]]
    out.update(D_y=ob["D_y"], C_v=ob["C_v"], largest_cluster=max(nz) if nz else 0)
    return out


def run_poly(args):
    """High size ratio: N = 500k, lognormal radii on [1, 10], phi = 0.55, mixed precision by
    default, on the size-class stencils (autotuned over cell spacings unless --tune 0)."""
    from paper_2108_01013_amd import synth

    N = args.N or 500_000
    t_gen = time.perf_counter()
    w = cached_workload(args, lambda: synth.config_high_ratio(N=N))
    print(f"# workload generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    import torch

    from paper_2108_01013_amd.dss import DSS_FP64, DSS_MIXED, Simulation
    prec = DSS_FP64 if args.precision == "fp64" else DSS_MIXED
    torch.cuda.set_device(0)
    p = w.params
    sim = Simulation(p, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    sim.set_tuning(sized=True, cell_scale=args.cell_scale or 1.5, wave_class=args.wave_class)
    sim.set_particles(w.x, w.rad)
    N = len(w.rad)
    tuned = maybe_tune(sim, args)
    el, timing, breakdown = timed_run(sim, N, args, 10)
    info = sim.info()
    _, sigma_mean, nsamp = sim.read_stress()
    if info["error_flags"]:
        print(f"# device error flags {info['error_flags']}", file=sys.stderr)
        sys.exit(1)
    tun = sim.tuning()
    sized = tun["sized"]
    names = {"k_pairs": "k_pairs_sized"} if sized else {}
    box = sim.box_info(0)
    ncell = int(info["cells"][0] * info["cells"][1] * info["cells"][2]) * int(box["size_classes"])
    roof = roofline(timing, N, ncell, info["n_contacts"], info["capacity"])
    roof["kernel"] = names.get("k_pairs", "k_pairs")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds, "the same N=500k lognormal")
    table = {names.get(k, k): v for k, v in kernel_table(breakdown).items()}
    return {
        "metric": "particle-steps/s, high size ratio (size-class stencils)",
        "value": round(N * args.steps / el, 1), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"single box N={N}, ln a ~ Normal(ln 1.5, 0.5) truncated to [1, 10], phi=0.55, "
                               f"LE shear rate 1, mu=1, dt=1e-4, stress every 10 steps, {args.precision}",
                   "N": N, "phi": 0.55, "size_ratio": round(float(w.rad.max() / w.rad.min()), 3),
                   "precision": args.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": table,
        "tuning": tuned or tun,
        "diagnostics": {"n_pairs": info["n_pairs"], "n_contacts": info["n_contacts"],
                        "max_row_fill": info["max_row_fill"], "capacity": info["capacity"],
                        "cells": info["cells"], "size_classes": box["size_classes"], "stress_samples": nsamp,
                        "eta_r_mean": float(sigma_mean[0, 1] / (p["eta0"] * p["shear_rate"]))},
    }


def run_sweep(args):
    from paper_2108_01013_amd import synth

    # the boxes are relaxed in a process pool, before anything loads the HIP runtime
    t_gen = time.perf_counter()
    ws, gds = synth.config_sweep(B=args.boxes, workers=args.workers)
    print(f"# {len(ws)} boxes generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    import torch
    torch.cuda.set_device(0)
    r = measure_sweep(ws, gds, args, tune=bool(args.tune), preshear_steps=args.sweep_preshear)
    N, info = r["N"], r["info"]
    mid = min(range(len(ws)), key=lambda b: abs(len(ws[b].rad) - 20_000))
    cpu = None if args.no_cpu_baseline else cpu_baseline(ws[mid], args.cpu_seconds,
                                                         f"box {mid} of the sweep (phi={synth.SWEEP_PHI[mid % 5]})")
    return {
        "metric": "particle-steps/s, batched flow-curve sweep",
        "value": round(N * args.steps / r["el"], 1), "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["el"] / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{r['B']} boxes, N_b uniform on 2000..50000 (sum {N}), phi_b in "
                               f"{list(synth.SWEEP_PHI)}, shear rate 1e-2..1e1, bidisperse 1:1.4, mu=1, "
                               f"dt=1e-4, stress every 10 steps, {args.precision}, after {r['sheared']} steps "
                               f"of pre-shear",
                   "boxes": r["B"], "N": N, "precision": args.precision},
        "roofline": r["roof"],
        "cpu_baseline": cpu,
        "kernels": r["table"],
        "tuning": r["tuning"],
        "diagnostics": {"n_pairs": info["n_pairs"], "n_contacts": info["n_contacts"],
                        "contacts_per_particle": round(info["n_contacts"] / N, 4),
                        "max_row_fill": info["max_row_fill"], "capacity": info["capacity"],
                        "cells_total": r["ncell"], "stress_samples": r["nsamp"],
                        "eta_r_mean": [round(e, 4) for e in r["eta"]]},
    }


def vjp_kernel_bytes(N: int, pairs: int, contacts: int) -> float:
    """Compulsory bytes of one k_pairs_vjp launch: per particle x, u, w, radius read (80 B),
    force / torque cotangents read (48 B), x, u, w adjoints added (72 B read + 72 B written);
    per pair its two ids (8 B); per contact the old and new stretch with their keys
    (2 x 28 B) and the old-stretch adjoint written and the new one read (2 x 24 B)."""
    return N * (80 + 48 + 144) + pairs * 8 + contacts * (56 + 48)


def measure_adjoint(w, args, precision: str, K: int, C: int, warmup: int):
    """Adjoint of the mean Sigma_xy over K steps from w's packing: returns the wall time of the
    adjoint call, the forward-only wall time of K steps, the VJP kernel's roofline and the result."""
    import numpy as np
    import torch

    from paper_2108_01013_amd.dss import DSS_FP64, DSS_MIXED, Simulation
    p = w.params
    N = len(w.rad)
    prec = DSS_FP64 if precision == "fp64" else DSS_MIXED
    se = 10
    Wt = np.zeros((3, 3))
    Wt[0, 1] = 1.0
    sim = Simulation(p, precision=prec, stream=torch.cuda.current_stream().cuda_stream)
    sim.set_particles(w.x, w.rad)
    # warm-up: a short adjoint (allocations, first launches), then back to a state at u^n
    sim.adjoint(min(warmup, K) or 1, 1, C, Wt)
    sim.compute_forces()
    torch.cuda.synchronize()
    # forward only, for the ratio
    sim.prepare_steps(K, stress_every=se)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(K, stress_every=se, sync=True)
    fwd = time.perf_counter() - t0
    sim.compute_forces()
    sim.set_timing(True, kernels=["k_pairs_vjp"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = sim.adjoint(K, se, C, Wt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = sim.timing()
    sim.set_timing(False)
    info = sim.info()
    sim.close()
    ms, nl = tm["k_pairs_vjp"]
    avg = ms / max(nl, 1) * 1e-3
    bytes_launch = vjp_kernel_bytes(N, info["n_pairs"], info["n_contacts"])
    ach = bytes_launch / avg / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": "k_pairs_vjp",
            "avg_launch_us": round(avg * 1e6, 3), "bytes_per_launch": int(bytes_launch)}
    return dict(N=N, K=K, C=C, se=se, el=el, fwd=fwd, roof=roof, r=r, info=info)


def mode_adjoint(w, args):
    a = measure_adjoint(w, args, "mixed", 200, 20, args.warmup)
    return {"value": round(a["N"] * a["K"] / a["el"], 1), "ms_per_step": round(a["el"] / a["K"] * 1e3, 5),
            "N": a["N"], "workload": "gradient of mean Sigma_xy over 200 steps, N=50k bidisperse phi=0.56, "
                                     "mixed-precision forward, FP64 reverse, checkpoints every 20 steps; "
                                     "value counts forward, recompute and reverse",
            "roofline": a["roof"], "adjoint_over_forward": round(a["el"] / a["fwd"], 3)}


def run_adjoint(args):
    import numpy as np

    from paper_2108_01013_amd import synth

    t_gen = time.perf_counter()
    N = args.N or 50_000
    w = synth.bidisperse_box(N, 0.56, seed=5)
    print(f"# workload generated in {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    import torch
    torch.cuda.set_device(0)
    K, C = args.steps, args.ckpt
    a = measure_adjoint(w, args, args.precision, K, C, args.warmup)
    r, info = a["r"], a["info"]
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's forward objective on a bounded window; its gradient would be 2 runs per
        # component by finite differences
        import oracle
        Wt = np.zeros((3, 3))
        Wt[0, 1] = 1.0
        small = synth.bidisperse_box(2000, 0.56, seed=5)
        u0 = oracle.ambient_velocity(small.params, small.x)
        w0 = oracle.ambient_rotation(small.params, len(small.rad))
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < args.cpu_seconds and k < 500:
            oracle.stress_objective(small.params, small.x, small.rad, u0, w0, 20, 10, Wt, use_cells=True)
            k += 1
        ec = time.perf_counter() - t0
        cpu = {"value": 2000 * 20 * k / ec, "unit": "particle-steps/s (forward objective only)",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"{k} oracle runs of the stress objective, N=2000 phi=0.56, 20 steps each, {ec:.1f} s; "
                         "a finite-difference gradient costs 2 such runs per component"}
    el = a["el"]
    return {
        "metric": "adjoint particle-steps/s (forward + checkpointed recompute + reverse)",
        "value": round(N * K / el, 1), "unit": "particle-steps/s", "n_gpus": 1, "steps": K,
        "warmup": args.warmup, "ms_per_step": round(el / K * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"adjoint of mean Sigma_xy over {K} steps, N={N} bidisperse 1:1.4, phi=0.56, "
                               f"stress every {a['se']}, checkpoints every {C}, gradients w.r.t. x0, u0, w0, mu, "
                               f"F_ER, forward in {args.precision}, reverse in FP64",
                   "N": N, "ckpt_every": C, "precision": args.precision},
        "roofline": a["roof"],
        "cpu_baseline": cpu,
        "forward_only_ms_per_step": round(a["fwd"] / K * 1e3, 5),
        "adjoint_over_forward": round(el / a["fwd"], 3),
        "diagnostics": {"J": r["J"], "dJ_dmu": r["dmu"], "dJ_dF_ER": r["dF_ER"],
                        "grad_x_norm": float(np.linalg.norm(r["dx"])), "n_pairs": info["n_pairs"],
                        "n_contacts": info["n_contacts"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--mode", choices=["single", "sweep", "adjoint", "poly"], default="single",
                    help="single: one box of N particles; sweep: the batched flow-curve sweep; "
                         "adjoint: gradient of the mean shear stress (N=50k); poly: size ratio 10 "
                         "(N=500k, size-class stencils)")
    ap.add_argument("--ckpt", type=int, default=20, help="adjoint checkpoint spacing")
    ap.add_argument("--N", type=int, default=None, help="particles (default per mode)")
    ap.add_argument("--boxes", type=int, default=64)
    ap.add_argument("--workers", type=int, default=16, help="processes generating the sweep's boxes")
    ap.add_argument("--tune", type=int, default=None,
                    help="1: autotune the launch first (default: on for the sweep, off for one box)")
    ap.add_argument("--tune-steps", type=int, default=20)
    ap.add_argument("--tune-cache", default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload-cache", default=None, help="npz file to reuse the single-box workload")
    ap.add_argument("--state-cache", default=None,
                    help="single: file holding the pre-sheared state (written by the first run, loaded by later ones)")
    ap.add_argument("--copy-probe", action="store_true", help="end with plain 256 MiB device copies")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--rolling", action="store_true", help="single: with rolling resistance")
    ap.add_argument("--ec-ranges", action="store_true",
                    help="single: electro-chemical forces over their own ranges (with attraction)")
    ap.add_argument("--observables", action="store_true", help="single: time the observables after the run")
    ap.add_argument("--sized", action="store_true", help="single: size-class stencils instead of the row tiles")
    ap.add_argument("--cell-scale", type=float, default=None, help="poly: lattice spacing over 2 c a_min (1.5)")
    ap.add_argument("--wave-class", type=int, default=2, help="poly: first size class on a wavefront (2)")
    ap.add_argument("--preshear", type=int, default=10_000,
                    help="single: steps sheared before timing (10000 = one strain unit at dt = 1e-4)")
    ap.add_argument("--sweep-preshear", type=int, default=1000, help="sweep: steps sheared before timing")
    ap.add_argument("--modes", type=int, default=1,
                    help="single: 1 = also time mixed precision, the 64-box sweep and the adjoint (N=50k)")
    args = ap.parse_args()
    if args.tune is None:
        args.tune = 1 if args.mode == "sweep" else 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    out = {"single": run_single, "sweep": run_sweep, "adjoint": run_adjoint, "poly": run_poly}[args.mode](args)
    if args.copy_probe:
        copy_probe()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
