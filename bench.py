#!/usr/bin/env python3
"""Benchmark of the FDTD-Bath time step on one MI355X.

Default workload: the large 3D grid, 512 x 512 x 512 cells (134 M), periodic in x and y, CPML in z,
a 205-cell Lorentz-Bath slab (40 % of z) with N_b = 16 explicit bath modes per cell and E component,
a Gaussian-profile plane source and a 256-frequency FP64 z-flux DFT plane; FP32 state, FP64 register
arithmetic, FP64 DFT accumulators.

One step = the whole time step: clock/source, every region's E and material update (bath force,
polarization and bath modes), every region's H update (CPML included), DFT staging and the blocked
DFT flush.  The flush runs once per 64 steps, so the warm-up and the timed region are both whole
64-step periods (a request for K steps times 64 * ceil(K / 64)), and every timed step carries its
share of the flush.

Prints one JSON line.  `value` is cell-updates per second (Gcell-updates/s) over the timed steps with
all state resident in HBM.  `roofline` is the dominant kernel's algorithmic HBM bytes per launch over
its average launch time, from HIP events recorded around each launch on the library's stream;
`step_roofline` is the whole step's algorithmic bytes over the step time.  `cpu_baseline` times the
FP64 CPU oracle on crops of the same layout (one thread, and every thread the host gives it) and
states the GPU's error against it on that crop (`parity`).  `learned` compares the K = 4 learned
closure in place of the explicit bath.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s & % HBM roofline; learned vs explicit bath at <=1e-3 error"
HBM_PEAK_GBS = 8000.0
KIND = {0: "background", 1: "drude", 2: "lorentz_bath", 3: "closure", 4: "multi_term"}


# the functions each counted kernel consists of (its own code and the helpers it calls)
KERNEL_CODE = {
    "E_lorentz_bath_nb8": ("__device__ __forceinline__ double ldd(", "__device__ __forceinline__ double at_minus(",
                           "__device__ __forceinline__ double source_term(", "__device__ __forceinline__ int xcd_block(",
                           "__device__ __forceinline__ void unflatten(", "__device__ __forceinline__ double z_minus_lane(",
                           "__device__ __forceinline__ double minus_lane_pairs(",
                           "__host__ __device__ inline long long pair_threads(", "void k_update_e_bath(const EArgs a"),
    "E_lorentz_bath_nb16": ("__device__ __forceinline__ double ldd(", "__device__ __forceinline__ double at_minus(",
                            "__device__ __forceinline__ double source_term(", "__device__ __forceinline__ int xcd_block(",
                            "__device__ __forceinline__ void unflatten(", "__device__ __forceinline__ void bath_component(",
                            "void k_update_e_bath_c(const EArgs a"),
}
# rocprofv3 kernel-name patterns of the counted kernels
KERNEL_NAMES = {"k_update_e_bath<3, float, 2,": "E_lorentz_bath_nb8", "k_update_e_bath_c<float, 4, false>": "E_lorentz_bath_nb16"}


def source_hash(tag: str = "E_lorentz_bath_nb16", src: str = None) -> str:
    """Hash of a counted kernel's code (its function and the helpers it calls, with comments and
    whitespace removed), so that counters taken on it stay valid while other kernels or comments
    change."""
    if src is None:
        src = open(os.path.join(ROOT, "paper_2505_23963_amd", "csrc", "fdtdb_kernels.hip")).read()
    h = hashlib.sha256()
    for start in KERNEL_CODE[tag]:
        s = src.find(start)
        e = src.find("\n}\n", s)
        body = src[s:e] if s >= 0 else start
        code = " ".join(re.sub(r"//[^\n]*", "", body).split())
        h.update(code.encode())
    return h.hexdigest()[:16]


def traffic_from_rocprof(pmc_dir: str):
    """Write profiles/traffic_counters.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE csv runs of
    this benchmark (pmc_<workload>_FETCH_SIZE/, pmc_<workload>_WRITE_SIZE/) and of the copy calibration
    (pmccopy_FETCH_SIZE/, pmccopy_WRITE_SIZE/) under pmc_dir.  Counter KiB per dispatch are scaled
    by what the same counter reads for a device copy of known size."""
    import csv

    def per_kernel(path):
        d = {}
        for row in csv.DictReader(open(path)):
            d.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in d.items()}

    out = {"kernels": {}, "calibration": {}}
    cal = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cp = per_kernel(os.path.join(pmc_dir, f"pmccopy_{c}", "run_counter_collection.csv"))
        kib = max(v for k, v in cp.items() if "copyBuffer" in k)
        cal[c] = (1 << 30) / (kib * 1024.0)          # the calibration copies 1 GiB
        out["calibration"][c] = {"copy_bytes": 1 << 30, "counter_kib": kib, "scale": cal[c]}
    for wl in sorted(glob.glob(os.path.join(pmc_dir, "pmc_*_FETCH_SIZE"))):
        f = per_kernel(os.path.join(wl, "run_counter_collection.csv"))
        w = per_kernel(os.path.join(wl.replace("FETCH_SIZE", "WRITE_SIZE"), "run_counter_collection.csv"))
        for name, kib in f.items():
            for pat, tag in KERNEL_NAMES.items():
                if pat in name and name in w:
                    rd = kib * 1024.0 * cal["FETCH_SIZE"]
                    wr = w[name] * 1024.0 * cal["WRITE_SIZE"]
                    out["kernels"][tag] = {"kernel": name, "source_hash": source_hash(tag), "fetch_kib": kib,
                                           "write_kib": w[name], "read_bytes": rd, "write_bytes": wr,
                                           "hbm_bytes_per_launch": rd + wr}
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out, indent=1))


def traffic_from_profiles(kernel_tag: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the current
    code of the kernel."""
    path = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(path):
        return None
    try:
        k = json.load(open(path)).get("kernels", {}).get(kernel_tag)
    except ValueError:
        return None
    if not k or k.get("source_hash") != source_hash(kernel_tag):
        return None
    return k.get("hbm_bytes_per_launch")


def _oracle_rate(p, threads: int, seconds_target: float):
    """Cell-updates/s of the oracle as it stands on problem p with the given thread count: whole runs of
    5 steps from rest until about seconds_target have passed.  Returns (rate, steps, seconds, threads,
    oracle)."""
    import oracle
    oracle.build(force=False)
    used = oracle.set_threads(threads)
    o = oracle.Oracle(p)
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds_target:
        o.step(5)
        steps += 5
    dt = time.perf_counter() - t0
    return p.cells * steps / dt, steps, dt, used, o


def _crop_parity(p, o, steps, stream):
    """The GPU's errors against the oracle o after the same `steps` on crop p: relative L2 of E, H, and
    the bath layer's P and Y (all components)."""
    import numpy as np
    from paper_2505_23963_amd import Grid
    g = Grid(p, stream=stream)
    g.step(steps)
    g.synchronize()
    out = {}
    groups = {"E": [(lambda x, c=c: x.field(c)) for c in range(3)],
              "H": [(lambda x, c=c: x.field(c)) for c in range(3, 6)]}
    mi = next(i for i, m in enumerate(p.materials) if type(m).__name__ == "LorentzBath")
    groups["P"] = [(lambda x, c=c: x.polarization(mi, c, 0)) for c in range(3)]
    groups["Y"] = [(lambda x, c=c: x.bath(mi, c, 0)) for c in range(3)]
    for k, gets in groups.items():
        d = sum(float(np.linalg.norm(f(g) - f(o))) ** 2 for f in gets)
        n = sum(float(np.linalg.norm(f(o))) ** 2 for f in gets)
        out[k] = float("%.3e" % (np.sqrt(d / n) if n > 0 else 0.0))
    return out


def cpu_baseline(make_crop, crop_one: str, crop_all: str, seconds_target: float = 12.0, stream=None):
    """The FP64 oracle as it stands, timed on crops of the workload: one thread on the smaller crop and every
    thread the host gives it (OMP_NUM_THREADS, else all cores) on the larger one; then the GPU on the small
    crop for the same steps, and its error against the oracle there."""
    import os as _os
    n_all = int(_os.environ.get("OMP_NUM_THREADS", "0") or 0) or (_os.cpu_count() or 1)
    p1 = make_crop(crop_one)
    r1, st1, dt1, _, o1 = _oracle_rate(p1, 1, seconds_target)
    pa = make_crop(crop_all)
    ra, sta, dta, used, oa = _oracle_rate(pa, n_all, seconds_target)
    del oa
    parity = _crop_parity(p1, o1, st1, stream)
    return {"value": round(ra / 1e9, 6), "unit": "Gcell-updates/s", "cores": used, "kind": "oracle",
            "sample": f"FP64 oracle, {used} threads, {crop_all} crop of the same layout, {sta} steps from rest in "
                      f"{dta:.1f} s",
            "one_core": {"value": round(r1 / 1e9, 6), "unit": "Gcell-updates/s", "cores": 1,
                         "sample": f"{crop_one} crop, {st1} steps from rest in {dt1:.1f} s"},
            "parity": {"crop": crop_one, "steps": st1, "rel_l2": parity,
                       "measure": "relative L2 over all components of each field after the same steps, GPU FP32 "
                                  "state against the FP64 oracle"}}


def copy_calibration(gib: float = 1.0, reps: int = 5):
    """A plain device-to-device copy of known size (for scaling rocprofv3 byte counters)."""
    import torch
    n = int(gib * (1 << 30) // 4)
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "ms": dt * 1e3,
                      "GBps": 8 * n / dt / 1e9}), flush=True)


def bench_cavities(args):
    """64 1D cavities (L ~ U[1500, 4000], N_b = 32, FP32 state) in the on-chip batched launch."""
    import torch
    from fdtdb_inputs import configs
    from paper_2505_23963_amd import Batch
    torch.cuda.init()
    stream = torch.cuda.Stream()
    ps = configs.config3_cavities()
    steps = args.steps if args.steps != 64 else 50000
    b = Batch(ps, stream=stream.cuda_stream)
    b.step(args.warmup)
    b.synchronize()
    cells = sum(int(p.n[0]) for p in ps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    dt = time.perf_counter() - t0
    # bytes one step would move through HBM in the grid formulation (state read and written once)
    lb = sum(int(p.materials[1].box[1][0] - p.materials[1].box[0][0]) for p in ps)
    dr = sum(40 for _ in ps)
    vac = cells - lb - dr
    w = 4
    per_step = lb * (3 * w + w + 3 * w + 3 * 32 * w + 3 * w) + dr * (7 * w) + vac * (6 * w) + 2 * 32 * len(ps) * 8 * w
    print(json.dumps({
        "metric": METRIC, "value": round(cells * steps / dt / 1e9, 3), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(dt / steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "64 batched 1D cavities, L ~ U[1500,4000], N_b=32, FP32 state, per-cavity 512-frequency "
                               "DFT and bath energy every 10 steps", "cells": cells, "tiling": list(b.tiling)},
        "hbm_equivalent_GBps": round(per_step / (dt / steps) / 1e9, 1),
    }), flush=True)


def bench_fp1d(args):
    """The 1D Fabry-Perot workload (2048 cells, N_b = 16, FP64, 20000 steps): the grid path with graph replay
    and the on-chip batched path with one cavity."""
    import torch
    from fdtdb_inputs import configs
    from paper_2505_23963_amd import Batch, Grid
    torch.cuda.init()
    stream = torch.cuda.Stream()
    s = stream.cuda_stream
    p = configs.config1_1d()
    steps = args.steps if args.steps != 64 else p.steps
    out = {}
    g = Grid(p, stream=s, graph_chunk=128)
    g.step(args.warmup)
    g.synchronize()
    t0 = time.perf_counter()
    g.step(steps)
    g.synchronize()
    out["grid_graph"] = p.cells * steps / (time.perf_counter() - t0) / 1e9
    import copy
    pb = copy.deepcopy(p)
    pb.dfts = pb.dfts[:1]          # the batched path keeps one DFT point per cavity (the inside monitor)
    b = Batch([pb], stream=s)
    b.step(args.warmup)
    b.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.synchronize()
    dt = time.perf_counter() - t0
    out["batched_on_chip"] = p.cells * steps / dt / 1e9
    best = max(out.values())
    print(json.dumps({
        "metric": METRIC, "value": round(best, 4), "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(p.cells / best / 1e9 * 1e3, 6), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "1D Fabry-Perot 2048 cells (PML 64, Drude mirrors, 1800-cell Lorentz-Bath, N_b=16), "
                               "FP64 state, 512-frequency DFT, energy every 10 steps", "cells": p.cells,
                   "tiling": list(b.tiling)},
        "paths": {k: round(v, 4) for k, v in out.items()},
    }), flush=True)


def bench_closure2d(args):
    """Learned closure vs explicit N_b = 64 bath on the 2D 2048^2 TM grid with a 1024^2 Lorentzian-bath
    patch: cell-updates/s of both, and the errors against the explicit run."""
    import numpy as np
    import torch
    from fdtdb_inputs import configs
    from fdtdb_inputs.philox import Stream
    from fdtdb_inputs.problem import LorentzBath
    from paper_2505_23963_amd import Grid, closure
    torch.cuda.init()
    stream = torch.cuda.Stream()
    s = stream.cuda_stream
    # training data: the same material on a 512^2 grid (256^2 patch), every patch cell recorded for 1024 steps:
    # 65536 trajectories x 16 windows of 64 steps = 1.05e6 windows per epoch
    rec = configs.config4_2d(n=512, patch=(128, 384), src_x=120, flux_x=400)
    cells = np.arange(256 * 256)
    t0 = time.perf_counter()
    E, P = closure.record(rec, 0, 2, cells, 1024, stream=s)
    res = closure.train(E, P, rec.courant, rec.materials[0], configs.closure_init(5), epochs=args.train_epochs,
                        stream=s)
    t_train = time.perf_counter() - t0
    # multiply-adds per window-step: forward 1408, backward 1312, weight gradients 1477
    train_flops = 2.0 * (1408 + 1312 + 1477) * len(cells) * 1024 * len(res["curve"])
    print(f"[bench] closure trained in {t_train:.1f} s: loss {res['loss_tanh']:.3e}", file=sys.stderr, flush=True)
    p = configs.config4_2d()
    steps = args.steps if args.steps != 64 else 2000

    def timed(closures=None, prob=None):
        g = Grid(prob or p, stream=s, closures=closures)
        g.step(args.warmup)
        g.synchronize()
        g.set_profiling(True, bath_only=True)
        g.kernel_records()
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.step(steps)
        g.synchronize()
        dt = time.perf_counter() - t
        recs = g.kernel_records()
        lb = max((r for r in recs if r["phase"] == 0), key=lambda r: r["ms_total"])
        return p.cells * steps / dt / 1e9, dt / steps * 1e3, lb["ms_total"] / max(lb["launches"], 1), g

    v_exp, ms_exp, k_exp, _ = timed()
    bx = p.materials[0].box
    patch_cells = int(np.prod([bx[1][a] - bx[0][a] for a in range(3)]))
    cl = {0: {"weights": res["weights"], "scales": res["scales"]}}
    v_cl, ms_cl, k_cl, _ = timed(cl)
    # accuracy over the workload's 10000 steps (and before the explicit bath's revival)
    out_err = {}
    for horizon in (() if args.skip_accuracy else (2500, 10000)):
        fe = Grid(p, stream=s)
        fe.step(horizon)
        ref_f, ref_e = fe.flux(0), fe.field(2)
        del fe
        runs = {"closure": (p, cl)}
        pl = configs.config4_2d()
        m = pl.materials[0]
        pl.materials[0] = LorentzBath(m.box, omega0=m.omega0, gamma0=m.gamma0 + m.dephasing, eps_inf=m.eps_inf,
                                      sigma=m.sigma, n_bath=0)
        runs["lorentz_gamma0_plus_dephasing"] = (pl, None)
        runs["explicit_nb2"] = (configs.config4_2d(nb=2), None)
        for name, (pp, c) in runs.items():
            g = Grid(pp, stream=s, closures=c)
            g.step(horizon)
            f, e = g.flux(0), g.field(2)
            nf = float(np.max(np.abs(ref_f)))
            out_err.setdefault(name, {})[str(horizon)] = {
                "spectral": float(np.max(np.abs(f - ref_f)) / nf) if nf > 0 else None,
                "field": float(np.linalg.norm(e - ref_e) / np.linalg.norm(ref_e))}
            del g
    print(json.dumps({
        "metric": METRIC, "value": round(v_cl, 4), "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(ms_cl, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2D TM 2048x2048, PML 32, 1024x1024 Lorentzian-bath patch (N_b=64 explicit vs "
                               "K=4 learned closure), line source, 256-frequency flux line", "cells": p.cells},
        "explicit": {"value": round(v_exp, 4), "ms_per_step": round(ms_exp, 4), "patch_kernel_ms": round(k_exp, 4)},
        "learned": {"value": round(v_cl, 4), "ms_per_step": round(ms_cl, 4), "patch_kernel_ms": round(k_cl, 4)},
        "learned_over_explicit": round(v_cl / v_exp, 3),
        "learned_kernel_roofline": {"bound": "alu", "achieved": round(patch_cells * 2816 / (k_cl * 1e-3) / 1e12, 2),
                                    "peak": 157.3, "unit": "TFLOP/s",
                                    "frac": round(patch_cells * 2816 / (k_cl * 1e-3) / 1e12 / 157.3, 4),
                                    "flops_per_cell": 2816},
        "training": {"seconds": round(res["train_seconds"], 2), "loss_linear": res["loss_linear"],
                     "loss_tanh": res["loss_tanh"], "trajectories": res["trajectories"], "steps": 1024, "window": 64,
                     "windows_per_epoch": res["trajectories"] * res["windows_per_epoch"],
                     "adam_steps": len(res["curve"]) * res["windows_per_epoch"],
                     "roofline": {"bound": "alu", "achieved": round(train_flops / res["train_seconds"] / 1e12, 2),
                                  "peak": 157.3, "unit": "TFLOP/s",
                                  "frac": round(train_flops / res["train_seconds"] / 1e12 / 157.3, 4)}},
        "errors_vs_explicit": out_err,
        "k4_linear_closure_bound": _k4_bound(),
    }), flush=True)


def _k4_bound():
    """The smallest spectral error a 4-state linear closure was found to reach on this workload's bath (a layer
    as thick as the patch, steady state), as stored by tests/golden/make_closure_bound.py."""
    path = os.path.join(ROOT, "tests", "golden", "closure_bound_k4.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    return {"best_spectral_error": d["best_spectral_error"], "layer_cells": d["layer_cells"], "starts": d["starts"]}


def _whole_periods(n: int) -> int:
    """Steps rounded up to whole 64-step DFT flush periods (at least one)."""
    return 64 * max(1, -(-int(n) // 64))


def timed_grid(p, stream, warmup: int, steps: int, closures=None, reps: int = 1):
    """Build a grid, run `warmup` steps, then time `steps` steps (bracketed by device synchronisation)
    with HIP events around the Lorentz-Bath or closure launches.  Returns the seconds of the first timed
    region, of every repeat, the launch records of the first, and the grid's byte model."""
    import torch
    from paper_2505_23963_amd import Grid
    g = Grid(p, stream=stream.cuda_stream, closures=closures)
    stats = g.stats()
    g.step(warmup)
    g.synchronize()
    g.set_profiling(True, bath_only=True)
    g.kernel_records()                        # start from empty event lists
    times, recs = [], None
    for r in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        stream.synchronize()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        if r == 0:
            recs = g.kernel_records()
    g.synchronize()                           # watchdog (outside the timed region)
    del g
    return times, recs, stats


def bench_large3d(args):
    """The 512^3 grid (Lorentz-Bath slab over 40 % of z, N_b = 16 Ohmic, explicit bath): the benchmark line.
    Extras: the median of five more timed regions, the K = 4 learned closure in place of the bath
    (trained on a 32 x 32 crop) with its errors against the explicit run on a 64 x 64 crop."""
    import numpy as np
    import torch
    from fdtdb_inputs import configs
    torch.cuda.init()
    stream = torch.cuda.Stream()
    warmup, steps = _whole_periods(args.warmup), _whole_periods(args.steps)
    p = configs.config5_3d_large(steps=0)
    print(f"[bench] 512^3 explicit bath: warm-up {warmup}, timed {steps} steps (x6)", file=sys.stderr, flush=True)
    times, recs, stats = timed_grid(p, stream, warmup, steps, reps=6)
    elapsed = times[0]
    dom = max(recs, key=lambda r: r["ms_total"])
    avg_ms = dom["ms_total"] / max(dom["launches"], 1)
    achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
    tag = f"E_{KIND[dom['kind']]}_nb{dom['n_bath']}"
    ms_step = elapsed / steps * 1e3
    step_gbps = stats["bytes_per_step"] / (ms_step * 1e-3) / 1e9
    value = p.cells * steps / elapsed / 1e9
    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps,
        "steps_requested": args.steps, "warmup": warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D 512x512x512 (134M cells), periodic x,y, CPML z (32 cells), 205-cell Lorentz-Bath "
                               "slab (40% of z, sigma 0.05, N_b=16 Ohmic bath modes, explicit), Gaussian-profile "
                               "plane source, 256-frequency FP64 z-flux plane",
                   "cells": p.cells, "bath_cells": stats["bath_cells"], "n_bath": 16, "state_dtype": "f32",
                   "arith_dtype": "f64", "dft_dtype": "f64", "flush_period_steps": 64, "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(tag),
                     "kernel": tag, "bytes_per_launch": dom["bytes"], "avg_launch_ms": round(avg_ms, 4),
                     "cells_per_launch": dom["cells"]},
        "step_roofline": {"bound": "hbm", "achieved": round(step_gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(step_gbps / HBM_PEAK_GBS, 4), "bytes_per_step": stats["bytes_per_step"]},
        "repeats_ms_per_step": [round(t / steps * 1e3, 4) for t in times],
        "median_ms_per_step": round(float(np.median(times[1:])) / steps * 1e3, 4),
    }
    if not args.no_learned:
        out["learned"] = _learned_large3d(args, stream, warmup, steps, value)
    if not args.no_bath16:
        out["bath_f16"] = _bath16_large3d(stream, warmup, steps, value)
    if not args.no_thermal:
        out["thermal"] = _thermal_large3d(stream, warmup, steps, value)
    if not args.no_cpu_baseline:
        print("[bench] oracle on crops", file=sys.stderr, flush=True)

        def crop(spec):
            nx, ny = (int(v) for v in spec.split("x")[:2])
            return configs.config5_3d_large(nx=nx, ny=ny, steps=0)
        out["cpu_baseline"] = cpu_baseline(crop, "16x16x512", "64x64x512", stream=stream.cuda_stream)
    print(json.dumps(out), flush=True)


def _bath16_large3d(stream, warmup, steps, v_exp):
    """The same grid with the bath coordinates stored as binary16 (Y * 1024), a reduced-precision mode reported
    beside the FP32 line: cell-updates/s, the bath launch against its own algorithmic bytes, and the error the
    format adds, measured on a 16 x 16 x 512 crop over 2000 steps against the FP32-state run of the same crop
    (which matches the FP64 oracle to about 1e-6)."""
    import numpy as np
    from fdtdb_inputs import configs
    from paper_2505_23963_amd import Grid

    def layout(nx=512, ny=512, fmt="f16"):
        p = configs.config5_3d_large(nx=nx, ny=ny, steps=0)
        if fmt:
            p.materials[0].bath_storage, p.materials[0].bath_scale = fmt, 1024.0
        return p
    p = layout()
    print(f"[bench] 512^3 with the bath stored as binary16: warm-up {warmup}, timed {steps} steps",
          file=sys.stderr, flush=True)
    times, recs, stats = timed_grid(p, stream, warmup, steps)
    dom = max(recs, key=lambda r: r["ms_total"])
    avg_ms = dom["ms_total"] / max(dom["launches"], 1)
    value = p.cells * steps / times[0] / 1e9
    errs = {}
    grids = {fmt: Grid(layout(16, 16, fmt), stream=stream.cuda_stream) for fmt in ("f16", None)}
    for g in grids.values():
        g.step(2000)
        g.synchronize()
    a, b = grids["f16"], grids[None]
    for name, get in (("E", lambda g: np.concatenate([g.field(c).ravel() for c in range(3)])),
                      ("H", lambda g: np.concatenate([g.field(c).ravel() for c in range(3, 6)])),
                      ("P", lambda g: np.concatenate([g.polarization(0, c) for c in range(3)])),
                      ("Y", lambda g: np.concatenate([g.bath(0, c).ravel() for c in range(3)]))):
        x, y = get(a), get(b)
        errs[name] = float(f"{np.linalg.norm(x - y) / np.linalg.norm(y):.3e}")
    return {"value": round(value, 4), "ms_per_step": round(times[0] / steps * 1e3, 4),
            "over_fp32_bath": round(value / v_exp, 3), "format": "binary16 of Y * 1024",
            "bath_kernel_ms": round(avg_ms, 4), "bath_bytes_per_launch": dom["bytes"],
            "bath_achieved_gbs": round(dom["bytes"] / (avg_ms * 1e-3) / 1e9, 1),
            "bath_frac_of_hbm_peak": round(dom["bytes"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "rel_l2_vs_fp32_state_16x16x512_2000_steps": errs}


def _thermal_large3d(stream, warmup, steps, v_exp):
    """The same grid with its bath made thermal (Langevin forces at kT = 1e-6, Philox noise) and anharmonic
    (lambda_j = 50): cell-updates/s and the bath launch against its algorithmic bytes (the same 648 B per
    cell: the noise is generated in registers).  Its parity against the oracle is that of the thermal tests
    (FP64 1e-12, FP32 1e-5 on a crop of this layout with this set-up)."""
    from fdtdb_inputs import configs
    p = configs.thermal_setup(configs.config5_3d_large(steps=0))
    m = p.materials[0]
    print(f"[bench] 512^3 thermal + anharmonic bath: warm-up {warmup}, timed {steps} steps", file=sys.stderr, flush=True)
    times, recs, _ = timed_grid(p, stream, warmup, steps)
    dom = max(recs, key=lambda r: r["ms_total"])
    avg_ms = dom["ms_total"] / max(dom["launches"], 1)
    value = p.cells * steps / times[0] / 1e9
    return {"value": round(value, 4), "ms_per_step": round(times[0] / steps * 1e3, 4),
            "over_plain_bath": round(value / v_exp, 3), "kT": m.kT, "lambda_j": float(m.anharmonic[0]),
            "bath_kernel_ms": round(avg_ms, 4), "bath_bytes_per_launch": dom["bytes"],
            "bath_achieved_gbs": round(dom["bytes"] / (avg_ms * 1e-3) / 1e9, 1),
            "bath_frac_of_hbm_peak": round(dom["bytes"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "parity": "tests/test_gpu_thermal.py"}


def _learned_large3d(args, stream, warmup, steps, v_exp):
    """The learned closure on the same grid: cell-updates/s and its errors against the explicit bath."""
    import numpy as np
    from fdtdb_inputs import configs
    from fdtdb_inputs.philox import Stream
    from paper_2505_23963_amd import Grid, closure
    s = stream.cuda_stream
    print("[bench] learned closure: record and train on a 32 x 32 crop", file=sys.stderr, flush=True)
    rec = configs.config5_3d_large(nx=32, ny=32)
    ncell = 32 * 32 * 205
    cells = np.unique(Stream(1005, 5).integers(11000, 0, ncell - 1))[:8192]
    t0 = time.perf_counter()
    E, P = closure.record(rec, 0, 0, cells, 1024, stream=s)
    res = closure.train(E, P, rec.courant, rec.materials[0], configs.closure_init(5), stream=s)
    t_train = time.perf_counter() - t0
    cl = {0: {"weights": res["weights"], "scales": res["scales"]}}
    p = configs.config5_3d_large(steps=0)
    times, recs, _ = timed_grid(p, stream, warmup, steps, closures=cl)
    lb = max((r for r in recs if r["phase"] == 0), key=lambda r: r["ms_total"])
    v_cl = p.cells * steps / times[0] / 1e9
    errs = {}
    pc = configs.config5_3d_large(nx=64, ny=64)
    for horizon in (1200, 4000):
        ge = Grid(pc, stream=s)
        ge.step(horizon)
        fe, ee = ge.flux(0), ge.field(0)
        del ge
        gc = Grid(pc, stream=s, closures=cl)
        gc.step(horizon)
        fc, ec = gc.flux(0), gc.field(0)
        del gc
        errs[str(horizon)] = {"spectral": float(np.max(np.abs(fc - fe)) / np.max(np.abs(fe))),
                              "field": float(np.linalg.norm(ec - ee) / np.linalg.norm(ee))}
    return {"value": round(v_cl, 4), "ms_per_step": round(times[0] / steps * 1e3, 4),
            "slab_kernel_ms": round(lb["ms_total"] / max(lb["launches"], 1), 4),
            "learned_over_explicit": round(v_cl / v_exp, 3), "training_seconds": round(t_train, 1),
            "loss_linear": res["loss_linear"], "errors_vs_explicit_64x64_crop": errs,
            "accepted": False if max(e["spectral"] for e in errs.values()) > 1e-3 else True}


def bench_planar3d(args):
    """The 3D planar cavity (256 x 256 x 512, Drude mirrors, 400-cell Lorentz-Bath layer, N_b = 8, per-cell
    sigma)."""
    import numpy as np
    import torch
    from fdtdb_inputs import configs
    torch.cuda.init()
    stream = torch.cuda.Stream()
    warmup, steps = _whole_periods(args.warmup), _whole_periods(args.steps)
    p = configs.config2_3d(nx=args.nx, ny=args.ny, steps=0)
    print(f"[bench] planar cavity {p.n}: warm-up {warmup}, timed {steps} steps", file=sys.stderr, flush=True)
    times, recs, stats = timed_grid(p, stream, warmup, steps)
    dom = max(recs, key=lambda r: r["ms_total"])
    avg_ms = dom["ms_total"] / max(dom["launches"], 1)
    achieved = dom["bytes"] / (avg_ms * 1e-3) / 1e9
    tag = f"E_{KIND[dom['kind']]}_nb{dom['n_bath']}"
    ms_step = times[0] / steps * 1e3
    step_gbps = stats["bytes_per_step"] / (ms_step * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(p.cells * steps / times[0] / 1e9, 4), "unit": "Gcell-updates/s", "n_gpus": 1,
        "steps": steps, "steps_requested": args.steps, "warmup": warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D planar cavity 256x256x512 (periodic x,y; CPML z; Drude mirrors; 400-cell "
                               "Lorentz-Bath layer, N_b=8, per-cell sigma; plane Gaussian source; 256-frequency FP64 "
                               "z-flux DFT)", "cells": p.cells, "n_bath": 8, "state_dtype": "f32", "arith_dtype": "f64",
                   "dft_dtype": "f64", "parallelism": "single-gpu"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(tag), "kernel": tag,
                     "bytes_per_launch": dom["bytes"], "avg_launch_ms": round(avg_ms, 4), "cells_per_launch": dom["cells"]},
        "step_roofline": {"bound": "hbm", "achieved": round(step_gbps, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(step_gbps / HBM_PEAK_GBS, 4), "bytes_per_step": stats["bytes_per_step"]},
    }
    if not args.no_cpu_baseline:
        def crop(spec):
            nx, ny = (int(v) for v in spec.split("x")[:2])
            return configs.config2_3d(nx=nx, ny=ny, steps=0)
        out["cpu_baseline"] = cpu_baseline(crop, "16x16x512", "64x64x512", stream=stream.cuda_stream)
    print(json.dumps(out), flush=True)


def bench_variants(args):
    """The method's variants timed at full size: (i) the 512^3 layout with its slab a sum of three terms
    (Lorentz, Lorentz, Drude; Sec. II.A) on the general kernel; (ii) a 2048 x 1024 2D grid (CPML along x,
    N_b = 64 Lorentzian-form patch over all of y) Bloch-periodic along y with phase 0.8, against the same grid
    plain periodic.  Gcell-updates/s (a complex cell counted once) and the dominant launch against its
    algorithmic bytes (events around every launch, in a separate profiled run)."""
    import numpy as np
    import torch
    from fdtdb_inputs import configs
    from fdtdb_inputs.problem import PML, PERIODIC, LorentzBath, MultiPole, Problem, Source, box
    from paper_2505_23963_amd import Grid
    torch.cuda.init()
    stream = torch.cuda.Stream()
    warmup, steps = _whole_periods(args.warmup), _whole_periods(args.steps)

    def run(p):
        g = Grid(p, stream=stream.cuda_stream)
        g.step(warmup)
        g.synchronize()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        stream.synchronize()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.set_profiling(True)
        g.kernel_records()
        g.step(16)
        g.synchronize()
        recs = [r for r in g.kernel_records() if r["launches"]]
        dom = max(recs, key=lambda r: r["ms_total"] / r["launches"])
        ms = dom["ms_total"] / dom["launches"]
        del g
        return {"value": round(p.cells * steps / dt / 1e9, 4), "ms_per_step": round(dt / steps * 1e3, 4),
                "dominant_kernel": KIND[dom["kind"]], "kernel_ms": round(ms, 4), "kernel_bytes": dom["bytes"],
                "kernel_frac_of_hbm_peak": round(dom["bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    out = {"metric": METRIC, "unit": "Gcell-updates/s", "n_gpus": 1, "steps": steps, "warmup": warmup,
           "higher_is_better": True, "dtype": "f32", "data": "synthetic"}
    p = configs.config5_3d_large(steps=0, nfreq=16)
    slab = p.materials[0]
    p.materials[0] = MultiPole(slab.box, eps_inf=1.0, kinds=("lorentz", "lorentz", "drude"), omega=(1.0, 1.2, 0.5),
                               gamma=(0.01, 0.02, 0.01), sigma=(0.05, 0.02, 0.0))
    print(f"[bench] 512^3 with a three-term slab: warm-up {warmup}, timed {steps} steps", file=sys.stderr, flush=True)
    out["multi_term_512cubed"] = run(p)

    def bloch2d(phase):
        nx, ny, nb = 2048, 1024, 64
        q = Problem(name="bloch2d", ndim=2, n=(nx, ny, 1), bc=(PML, PERIODIC, PERIODIC), pml_cells=(32, 0, 0),
                    dtype="f32", steps=0, bloch=None if phase is None else (0.0, phase, 0.0))
        q.materials.append(LorentzBath(box((512, 1536), (0, ny)), omega0=1.0, gamma0=0.001, eps_inf=1.0, sigma=0.05,
                                       n_bath=nb, form="lorentzian", width=0.4, bath_gamma=0.4 / (nb - 1) / 2,
                                       dephasing=0.02))
        y = np.arange(ny)
        k = (phase or 0.0) / ny
        q.sources.append(Source(comp=2, box=box((48, 49), (0, ny)), omega_c=1.0, width=0.5, profile=np.cos(k * y),
                                profile_im=None if phase is None else np.sin(k * y)))
        return q
    print("[bench] 2D Bloch grid and its plain twin", file=sys.stderr, flush=True)
    out["bloch_2d_2048x1024"] = run(bloch2d(0.8))
    out["periodic_2d_2048x1024"] = run(bloch2d(None))
    out["bloch_over_periodic"] = round(out["bloch_2d_2048x1024"]["value"] / out["periodic_2d_2048x1024"]["value"], 3)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64,
                    help="timed steps, rounded up to whole 64-step DFT flush periods")
    ap.add_argument("--warmup", type=int, default=64, help="warm-up steps, rounded up like --steps")
    ap.add_argument("--train-epochs", type=int, default=600,
                    help="closure training epochs (closure2d; fewer only to profile the inference kernels)")
    ap.add_argument("--skip-accuracy", action="store_true",
                    help="closure2d: skip the accuracy runs against the explicit bath (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="large3d: leave out the learned-closure comparison")
    ap.add_argument("--no-bath16", action="store_true", help="large3d: leave out the 16-bit bath storage line")
    ap.add_argument("--no-thermal", action="store_true", help="large3d: leave out the thermal / anharmonic bath line")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--traffic-from", default=None,
                    help="write profiles/traffic_counters.json from rocprofv3 counter runs under this folder")
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=256)
    ap.add_argument("--workload", choices=["large3d", "planar3d", "cavities", "closure2d", "fp1d", "variants"],
                    default="large3d",
                    help="large3d: the 512^3 line (default); planar3d: the 256x256x512 planar cavity; cavities: the "
                         "64-cavity batched 1D workload; closure2d: learned closure vs explicit bath on the 2D 2048^2 "
                         "grid; fp1d: the 1D Fabry-Perot workload in FP64; variants: a three-term slab on the "
                         "512^3 layout and a Bloch-periodic 2D grid against its plain twin")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: fdtdb runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(a slab decomposition over several GPUs is designed but not built)",
              file=sys.stderr, flush=True)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.traffic_from:
        traffic_from_rocprof(args.traffic_from)
        return
    {"large3d": bench_large3d, "planar3d": bench_planar3d, "cavities": bench_cavities, "closure2d": bench_closure2d,
     "fp1d": bench_fp1d, "variants": bench_variants}[args.workload](args)


if __name__ == "__main__":
    main()
