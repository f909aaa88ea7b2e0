"""Throughput of the moving-grid split-operator step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4]

A step is one composition step (all stages, every kinetic and potential substep
with its FFT sweeps, Ehrenfest reductions and grid moves) over the workload's
whole grid.  value = grid points x K / wall seconds of the K timed steps, with the
state resident in HBM.  Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

METRIC = "grid-point-steps/sec, c64 vs FP64 at <=1e-6 err; % HBM roofline"
HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1909_06412_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
POT_KIND = {"free": 0, "harmonic": 1, "morse_repulsion": 2, "henon_heiles": 3, "quadratic": 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    if name == "c1":
        return W.harmonic_1d()
    if name == "c2":
        return W.harmonic_3d(seed=0, order=4, dt=0.01, precision="c64")
    if name == "c3":
        return W.morse_repulsion_2d()
    if name == "c4":
        return W.henon_heiles_8d()
    if name == "c5":
        return W.morse_batch()
    raise SystemExit(f"unknown workload {name}")


def cpu_sample(name):
    """A bounded sample of the workload for the oracle timing (10-30 s of CPU)."""
    if name == "c4":
        w = W.henon_heiles_8d(n=8, dq=1.25, precision="c128")   # the paper's 8^8 grid, same span
        return w, 1, "one Suzuki-4 step of the 8-D Henon-Heiles model on an 8^8 grid (16.8M points)"
    if name == "c3":
        return W.morse_repulsion_2d(precision="c128"), 200, "200 Strang steps of the 256^2 Morse model"
    if name == "c2":
        return W.harmonic_3d(seed=0, order=4, dt=0.01), 20, "20 Suzuki-4 steps of the 32^3 harmonic model"
    if name == "c5":
        return W.morse_batch(precision="c128")[:8], 20, "20 Strang steps of 8 of the 256 packets"
    return W.harmonic_1d(), 1000, "1000 Strang steps of the 64-point oscillator"


def run_cpu_baseline(name):
    import oracle as O
    w, nsteps, desc = cpu_sample(name)
    if isinstance(w, list):
        t0 = time.perf_counter()
        pts = 0
        for wi in w:
            g = O.Grid(wi["N"], wi["dq"], wi["hbar"])
            wp = O.gaussian(g, wi["q0"], wi["p0"], wi["sigma"])
            pot = O.potentials.from_spec(*wi["potential"], wi["D"])
            O.run(wp, wi["dt"], nsteps, O.composition(wi["comp"], wi["order"]), pot, wi["inv_mass"],
                  wi["split"])
            pts += int(np.prod(wi["N"]))
        dt = time.perf_counter() - t0
        return {"value": pts * nsteps / dt, "unit": "grid-point-steps/s", "cores": 1, "kind": "oracle",
                "sample": f"{desc}, FP64 NumPy, {dt:.1f} s"}
    g = O.Grid(w["N"], w["dq"], w["hbar"])
    wp = O.gaussian(g, w["q0"], w["p0"], w["sigma"])
    pot = O.potentials.from_spec(*w["potential"], w["D"])
    gam = O.composition(w["comp"], w["order"])
    t0 = time.perf_counter()
    O.run(wp, w["dt"], nsteps, gam, pot, w["inv_mass"], w["split"])
    dt = time.perf_counter() - t0
    pts = int(np.prod(w["N"]))
    return {"value": pts * nsteps / dt, "unit": "grid-point-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{desc}, FP64 NumPy, {dt:.1f} s"}


# Sources the single-grid sweep kernels and their launches are built from (the
# batch, streaming and adjoint engines live in the .inc files and do not enter them).
GRID_SOURCES = ("mgso.hip", "mgso_common.h", "mgso_kernels.h", "mgso_split.h", "mgso_sweep.h", "mgso_sweep16.h")


def kernel_source_hash() -> str:
    """sha256 over the sources of the single-grid kernels (sorted by name):
    counters measured on other sources no longer describe the kernels."""
    import hashlib
    h = hashlib.sha256()
    for f in sorted(GRID_SOURCES):
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def kernel_label(w, precision, cls):
    """Kernel template name of a profiled sweep class (sweep, dir, epi, group axes, mode)."""
    si, d, epi, k, mode = cls
    t = "float" if precision == "c64" else "double"
    if mode >= 3:
        # passes of the three-pass 16^8 plan: B forward 0, B inverse 1, C moments 2, C round trip 3
        return f"k_split<{t}, {2 if mode == 4 else (d if si == 1 else 3)}>"
    fast16 = w["D"] >= 3 and all(n == 16 for n in w["N"]) and w["potential"][0] != "morse_repulsion"
    if not fast16:
        return f"k_sweep<{t}>"
    pk = POT_KIND[w["potential"][0]] if epi == 4 else -1
    return f"k_sweep16<{t}, {k}, {'true' if d else 'false'}, {epi}, {pk}, {mode}>"


def measured_traffic(w, precision, label):
    """HBM bytes per launch of `label` from the committed rocprofv3 counter summary
    of this workload (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter
    reads for a plain device copy of known size), or None when there is none or it
    was taken on other kernel sources."""
    path = os.path.join(PROFILES, f"pmc_traffic_{w['name'].replace('^', 'e')}_{precision}.txt")
    if not os.path.exists(path):
        return None
    src, table = None, {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("source_sha256"):
                src = line.split()[1]
            elif line.startswith("kernel "):
                parts = [x.strip() for x in line[len("kernel "):].split("|")]
                vals = dict(x.split(None, 1) for x in parts[1:])
                table[parts[0]] = float(vals["traffic_bytes"])
    if src != kernel_source_hash():
        return None
    return table.get(label)


def timed_run(w, precision, steps, warmup, profile):
    import paper_1909_06412_amd as mg
    import torch
    m = mg.from_workload(w, precision=precision)
    log(f"{w['name']} {precision}: state {m.h and mg.L.lib().mg_state_bytes(m.h) / 2**30:.2f} GiB, "
        f"warmup {warmup}")
    if warmup:
        m.step(w["dt"], warmup)
    if profile:
        m.set_option(mg.MG_OPT_PROFILE, 1)
        m.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.step(w["dt"], steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = (m.profile_class(), *m.profile_read(reset=True)) if profile else None
    m.set_option(mg.MG_OPT_PROFILE, 0)
    obs = m.observables()
    log(f"{w['name']} {precision}: {steps} steps in {el:.3f} s; norm {obs['norm']:.15f}")
    return m, el, prof, obs


def batch_run(ws, precision, steps, warmup, autotune=True):
    import paper_1909_06412_amd as mg
    import torch
    b = mg.batch_from_workloads(ws, precision=precision)
    tuned = None
    if autotune:
        # the batch's own autotuner picks the launch shape (outside the timed region)
        k, ms = b.autotune(ws[0]["dt"], 10)
        tuned = {"shape": int(k), "threads": b.config(k)[0], "tile": b.config(k)[1],
                 "streaming": bool(k == b.N_CONFIGS - 1),
                 "probe_ms_per_step": {f"{i}:{b.config(i)[0]}x{b.config(i)[1]}": round(float(x), 4)
                                       for i, x in enumerate(ms)}}
        log(f"autotune: {tuned}")
    log(f"batch of {b.B} packets, {b.points} points, {precision}; warmup {warmup}")
    if warmup:
        b.step(ws[0]["dt"], warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(ws[0]["dt"], steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    obs = b.observables()
    log(f"batch {precision}: {steps} steps in {el:.3f} s; norms {min(o['norm'] for o in obs):.12f}"
        f"..{max(o['norm'] for o in obs):.12f}")
    pts = b.points
    b.close()
    return el, pts, obs, tuned


def main_batch(args):
    ws = W.morse_batch(precision="c64")
    el, pts, obs, tuned = batch_run(ws, "c64", args.steps, args.warmup)
    value = pts * args.steps / el
    out = {
        "metric": METRIC, "value": value, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": "morse_batch_256_packets", "packets": len(ws), "points": pts,
                   "potential": "morse_repulsion", "composition": "strang", "order": 2, "split": "TVT",
                   "dt": ws[0]["dt"], "precision": "c64",
                   "launch": "autotuned shape: one persistent kernel per call, or one launch per sweep",
                   "launch_shape": tuned},
    }
    if not args.no_fp64:
        el2, _, obs2, _ = batch_run(W.morse_batch(precision="c128"), "c128", args.steps, args.warmup)
        d = max(abs(a["norm"] - b_["norm"]) for a, b_ in zip(obs, obs2))
        d = max(d, max(float(np.max(np.abs(a["q"] - b_["q"]))) for a, b_ in zip(obs, obs2)))
        out["fp64"] = {"value": pts * args.steps / el2, "ms_per_step": el2 / args.steps * 1e3,
                       "c64_speedup": el2 / el, "c64_vs_fp64_observable_maxdiff": d}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = run_cpu_baseline("c5")
    print(json.dumps(out), flush=True)


def calibrate_copy():
    """A plain device copy of known size (4 GiB read + 4 GiB written per copy): the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes, and the
    streaming bandwidth this device reaches with a simple kernel."""
    import torch
    n = 1 << 29
    x = torch.ones(n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    best = None
    for i in range(4):
        t0 = time.perf_counter()
        y.copy_(x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        best = el if best is None else min(best, el)
        log(f"copy {i}: {el * 1e3:.3f} ms")
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                      "best_ms": best * 1e3, "GB_s": 2 * n * 8 / best / 1e9}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # default steps: the unmerged end of a call (one extra kinetic half-substep) is
    # spread over 20 steps of the 16^8 grid (about 12 s) and 200 steps of the batch
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="time a plain 4 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.steps is None:
        args.steps = 200 if args.workload == "c5" else 20
    if args.workload == "c5":
        return main_batch(args)
    w = workload(args.workload)
    prec = w["precision"]
    pts = int(np.prod(w["N"]))
    m, el, prof, obs = timed_run(w, prec, args.steps, args.warmup, profile=True)
    m.close()
    del m
    torch.cuda.empty_cache()
    value = pts * args.steps / el
    cls, launches, total_ms, bytes_per = prof
    avg_ms = total_ms / max(launches, 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    label = kernel_label(w, prec, cls)
    traffic = measured_traffic(w, prec, label)
    out = {
        "metric": METRIC, "value": value, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64" if prec == "c64" else "c128", "data": "synthetic",
        "config": {"workload": w["name"], "grid": "x".join(map(str, w["N"])), "points": pts,
                   "potential": w["potential"][0], "composition": w["comp"], "order": w["order"],
                   "split": w["split"], "dt": w["dt"], "precision": prec},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": label, "sweep": cls[0], "avg_ms": avg_ms,
                     "launches": launches, "bytes_per_launch": bytes_per},
    }
    if not args.no_fp64 and prec == "c64":
        m2, el2, _, obs2 = timed_run(w, "c128", args.steps, args.warmup, profile=False)
        m2.close()
        del m2
        torch.cuda.empty_cache()
        d = max(abs(obs[k] - obs2[k]) for k in ("norm", "Ekin", "Epot"))
        d = max(d, float(np.max(np.abs(obs["q"] - obs2["q"]))), float(np.max(np.abs(obs["p"] - obs2["p"]))))
        out["fp64"] = {"value": pts * args.steps / el2, "ms_per_step": el2 / args.steps * 1e3,
                       "c64_speedup": el2 / el, "c64_vs_fp64_observable_maxdiff": d}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = run_cpu_baseline(args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
