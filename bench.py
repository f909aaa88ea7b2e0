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


def run_cpu_baseline(name, workers=1):
    """The oracle as it stands, timed on a bounded sample of the workload.  workers:
    threads of its FFT library primitive (the pointwise NumPy work stays on one)."""
    import oracle as O
    O.grid.set_fft_workers(workers)
    try:
        w, nsteps, desc = cpu_sample(name)
        ws = w if isinstance(w, list) else [w]
        t0 = time.perf_counter()
        pts = 0
        for wi in ws:
            g = O.Grid(wi["N"], wi["dq"], wi["hbar"])
            wp = O.gaussian(g, wi["q0"], wi["p0"], wi["sigma"])
            pot = O.potentials.from_spec(*wi["potential"], wi["D"])
            gam = O.composition(wi["comp"], wi["order"])
            if len(ws) == 1:
                t0 = time.perf_counter()       # a single grid: time the propagation only
            O.run(wp, wi["dt"], nsteps, gam, pot, wi["inv_mass"], wi["split"])
            pts += int(np.prod(wi["N"]))
        dt = time.perf_counter() - t0
    finally:
        O.grid.set_fft_workers(1)
    return {"value": pts * nsteps / dt, "unit": "grid-point-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{desc}, FP64 NumPy/SciPy (FFT on {workers} thread{'s' if workers > 1 else ''}), "
                      f"{dt:.1f} s"}


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
    # the 8-D Henon-Heiles potential sweep on the contiguous tile has its dimension fixed
    dt = 8 if (epi == 4 and pk == 3 and k == 3 and w["D"] == 8) else 0
    return f"k_sweep16<{t}, {k}, {'true' if d else 'false'}, {epi}, {pk}, {mode}, {dt}>"


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
    if not args.no_c64:
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


def stream_ceiling(m, reps=3):
    """Streaming reference on the state's own memory: torch's in-place x *= 1.0 over the
    whole state buffer (every byte read once and written once, the state left bit for bit
    as it was), best of `reps` by events on torch's stream.  The same physical pages as
    the sweeps, so it is the bandwidth a plain streaming kernel reaches there."""
    import torch
    buf = m._bufs[0]
    x = buf.view(torch.float64)
    nbytes = buf.numel()
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        x.mul_(1.0)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return {"kernel": "torch in-place x *= 1.0 over the state buffer", "bytes": 2 * nbytes, "ms": best,
            "GB_s": 2 * nbytes / best / 1e6}


def roofline_of(w, precision, prof):
    """Roofline entry of the kernel class with the largest total time: algorithmic
    bytes per launch / its average launch time from HIP events over the timed steps."""
    cls, launches, total_ms, bytes_per = prof
    avg_ms = total_ms / max(launches, 1)
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    label = kernel_label(w, precision, cls)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(w, precision, label),
            "kernel": label, "sweep": cls[0], "avg_ms": avg_ms, "launches": launches,
            "bytes_per_launch": bytes_per}


SAMPLE_POINTS = 1 << 16


def sampled_state(m, idx):
    """The device state at flat indices idx, as complex128 on the host."""
    import torch
    v = m.state_view()
    return v.index_select(0, torch.from_numpy(idx).to(v.device)).to(torch.complex128).cpu().numpy()


C2_SCHEMES = (("strang", 2), ("suzuki", 4), ("triple_jump", 4), ("triple_jump", 6), ("suzuki", 6),
              ("triple_jump", 8), ("triple_jump", 10))


def c2_gate(tol=1e-6, max_stages=20000):
    """"c64 vs FP64 at <= 1e-6 error" on the 3-D harmonic model (32^3, seed 0, t_f = 5).
    Every listed scheme (order 2-10, dt 0.1 ... 0.001, runs up to max_stages stages) in
    both precisions, timed as whole mg_step calls; error = relative l2 distance at t_f
    from a converged FP64 run on the same grid (10th-order triple jump, dt = 0.005),
    interpolated onto each run's final grid with mg_regrid.  Reports per precision the
    fastest run within tol (or, if none, the most accurate one)."""
    import paper_1909_06412_amd as mg
    import torch
    t_f = 5.0
    base = W.harmonic_3d(seed=0, order=10, dt=0.005, t_final=t_f)
    ref = mg.from_workload(base, precision="c128")
    ref.step(base["dt"], base["steps"])
    runs = []
    for prec in ("c128", "c64"):
        for comp, order in C2_SCHEMES:
            stages_per_step = {"strang": 1, "suzuki": 5 ** (order // 2 - 1),
                               "triple_jump": 3 ** (order // 2 - 1)}[comp]
            w = W.harmonic_3d(seed=0, order=order, dt=0.1, t_final=t_f, precision=prec)
            w["comp"] = comp
            m = mg.from_workload(w, precision=prec)
            for dt in W.HARMONIC_3D_DTS:
                n = int(round(t_f / dt))
                if n * stages_per_step > max_stages:
                    continue
                m.set_gaussian(w["q0"], w["p0"], w["sigma"])
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                m.step(dt, n)
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                psi, q, _, _ = m.get_state()
                ref.regrid(q)
                r_psi = ref.get_state()[0]
                err = float(np.linalg.norm(psi - r_psi) / np.linalg.norm(r_psi))
                runs.append({"precision": prec, "comp": comp, "order": order, "dt": dt,
                             "stages": n * stages_per_step, "ms": round(el * 1e3, 3), "err": err})
            m.close()
    ref.close()
    out = {"workload": "harmonic_3d_32^3_seed0", "t_final": t_f, "tolerance": tol,
           "reference": "FP64, 10th-order triple jump, dt 0.005", "error": "relative l2 at t_final"}
    for prec in ("c128", "c64"):
        ok = [r for r in runs if r["precision"] == prec and r["err"] <= tol]
        best = min(ok, key=lambda r: r["ms"]) if ok else min(
            (r for r in runs if r["precision"] == prec), key=lambda r: r["err"])
        out[prec] = dict(best, within_tolerance=bool(ok))
    if out["c128"]["within_tolerance"] and out["c64"]["within_tolerance"]:
        out["c64_speedup_at_tolerance"] = out["c128"]["ms"] / out["c64"]["ms"]
    out["runs"] = [[r["precision"], r["comp"], r["order"], r["dt"], r["stages"], r["ms"], float(f"{r['err']:.3e}")]
                   for r in runs]
    return out


def c1_extra():
    """The 64-point oscillator: its whole 1000-step Strang run, complex128."""
    w = W.harmonic_1d()
    m, el, _, obs = timed_run(w, "c128", w["steps"], 0, profile=False)
    m.close()
    return {"workload": w["name"], "steps": w["steps"], "value": 64 * w["steps"] / el,
            "ms_per_step": el / w["steps"] * 1e3, "norm_minus_1": obs["norm"] - 1.0}


def c3_extra(steps=2000):
    """The 256^2 atom-diatom model: whole-call throughput in both precisions."""
    out = {"workload": "morse_repulsion_256x256", "steps": steps}
    for prec in ("c64", "c128"):
        w = W.morse_repulsion_2d(precision=prec)
        m, el, _, obs = timed_run(w, prec, steps, 10, profile=False)
        m.close()
        out[prec] = {"value": int(np.prod(w["N"])) * steps / el, "ms_per_step": el / steps * 1e3,
                     "norm_minus_1": obs["norm"] - 1.0}
    return out


def c5_extra(steps=200):
    """The 256 uneven atom-diatom packets, autotuned launch shape, both precisions."""
    out = {"workload": "morse_batch_256_packets", "steps": steps}
    for prec in ("c64", "c128"):
        ws = W.morse_batch(precision=prec)
        el, pts, obs, tuned = batch_run(ws, prec, steps, 10)
        out[prec] = {"value": pts * steps / el, "ms_per_step": el / steps * 1e3, "points": pts,
                     "launch_shape": tuned["shape"],
                     "norm_minus_1_max": max(abs(o["norm"] - 1.0) for o in obs)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # default steps: the unmerged end of a call (one extra kinetic half-substep) is
    # spread over 20 steps of the 16^8 grid and 200 steps of the batch
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--no-c64", action="store_true", help="skip the complex64 leg")
    ap.add_argument("--no-extras", action="store_true", help="skip the C2 gate and the C3 / C5 keys")
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
    pts = int(np.prod(w["N"]))
    idx = np.random.default_rng(7).integers(0, pts, size=min(SAMPLE_POINTS, pts))
    # the paper's precision (FP64) is the headline; complex64 is reported beside it
    m, el, prof, obs = timed_run(w, "c128", args.steps, args.warmup, profile=True)
    s128 = sampled_state(m, idx)
    ceil128 = stream_ceiling(m)
    m.close()
    del m
    torch.cuda.empty_cache()
    value = pts * args.steps / el
    out = {
        "metric": METRIC, "value": value, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": "x".join(map(str, w["N"])), "points": pts,
                   "potential": w["potential"][0], "composition": w["comp"], "order": w["order"],
                   "split": w["split"], "dt": w["dt"], "precision": "c128"},
        "roofline": roofline_of(w, "c128", prof),
    }
    ceil128["roofline_kernel_frac"] = out["roofline"]["achieved"] / ceil128["GB_s"]
    out["stream_ceiling"] = {"c128": ceil128}
    if not args.no_c64:
        m2, el2, prof2, obs2 = timed_run(w, "c64", args.steps, args.warmup, profile=True)
        s64 = sampled_state(m2, idx)
        ceil64 = stream_ceiling(m2)
        m2.close()
        del m2
        torch.cuda.empty_cache()
        d = max(abs(obs[k] - obs2[k]) for k in ("norm", "Ekin", "Epot"))
        d = max(d, float(np.max(np.abs(obs["q"] - obs2["q"]))), float(np.max(np.abs(obs["p"] - obs2["p"]))))
        out["c64"] = {"value": pts * args.steps / el2, "ms_per_step": el2 / args.steps * 1e3,
                      "speedup_vs_fp64": el / el2, "roofline": roofline_of(w, "c64", prof2),
                      "vs_fp64": {"sampled_points": int(idx.size),
                                  "rel_l2": float(np.linalg.norm(s64 - s128) / np.linalg.norm(s128)),
                                  "max_rel": float(np.max(np.abs(s64 - s128)) / np.max(np.abs(s128))),
                                  "observable_maxdiff": d,
                                  "norm_minus_1": obs2["norm"] - 1.0, "fp64_norm_minus_1": obs["norm"] - 1.0}}
        ceil64["roofline_kernel_frac"] = out["c64"]["roofline"]["achieved"] / ceil64["GB_s"]
        out["stream_ceiling"]["c64"] = ceil64
    if not args.no_extras and args.workload == "c4":
        log("C1 ...")
        out["c1"] = c1_extra()
        log("C2 accuracy gate ...")
        out["c2_gate"] = c2_gate()
        log("C3 ...")
        out["c3"] = c3_extra()
        log("C5 ...")
        out["c5"] = c5_extra()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = run_cpu_baseline(args.workload)
        ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        out["cpu_baseline_all_cores"] = run_cpu_baseline(args.workload, workers=min(ncpu, 16))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
