"""Benchmark: q-batched lattice site-updates/s of the hybrid LBM Bloch-Torrey
step on one MI355X, with the HBM roofline of the step kernel, the adjoint
(reverse sweep) on the adjoint workload, the FP32-vs-FP64 signal error over a
full echo time, the plain FP64 one-q-sample-per-launch rate, and the FP64
CPU oracle timed on the host as a baseline.

Default workload (the q-batched case): 256^3 lattice, dx = 0.25 um, periodic
faces, z-cylinders (Gamma(4, mean 1 um) radii, kappa 0.02 um/ms) to 40 %
plus spheres (radius U(2, 6) um, kappa 0.05 um/ms) to +15 %, D 2.0/1.0/1.0
um^2/ms, T2 90/70/70 ms, PGSE delta 10 Delta 30 ms, dt = 0.004 ms, 64
golden-spiral directions x b in {500, 1000, 2000, 3000} s/mm^2 = 256
q-samples, one field each.  Their two population copies (2 x 240 GB in FP32)
exceed device memory, so the library runs them in q-waves.

A benchmark step is one lattice time step of the whole q-batch: stream with
boundaries and membranes, reaction, signal reduction and collision for
every q-sample.  `value` counts q-sample site-updates per second (256 x 256^3
per step).  The adjoint leg runs on the adjoint workload (96^3 cylinders,
30 q-samples): a taped forward and the reverse sweep.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload cfg3a]
(--workload selects one of the other synthetic workloads).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "q-batched site-updates/s + % HBM peak, fwd & adjoint, at stated err vs FP64"
HBM_PEAK_GBS = 8000.0
BYTES_PER_FIELD_SITE_F32 = 112      # read 7 complex float + write 7 complex float
BYTES_PER_FIELD_SITE_F64 = 224
ADJ_BYTES_PER_FIELD_SITE_F32 = 168  # read adjoint + read forward state + write adjoint
KERNEL_SRC = os.path.join(ROOT, "paper_1907_00908_amd", "csrc", "btl_kernels.hip")
ADJOINT_SRC = os.path.join(ROOT, "paper_1907_00908_amd", "csrc", "btl_adjoint.hip")


def source_hash(path) -> str:
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


WORKLOAD_NAMES = {
    "cfg1": "uniform 32^3 periodic free diffusion, PGSE, G || x, b=1000 (plain case)",
    "cfg2": "two-phase axon model 128^3, mirror BC, 6 oblique directions, b=1000",
    "cfg3a": "cylinders+spheres 256^3 periodic, 64 directions x 4 b-values = 256 q (q-batched)",
    "cfg3b": "16 cylinder geometries 96^3..192^3 (ragged batch), 6 directions each",
    "cfg4": "two-phase cylinders 96^3 periodic, 30 directions (adjoint workload)",
    "cfg5": "three-phase ellipsoid cells 512^3 periodic, cosine OGSE, 32 directions",
    "cfg2d": "2D axon cross-sections 512^2 on the D2Q5 lattice, 64 in-plane dirs x 4 b-values",
}
TRAFFIC_FILES = {
    ("cfg3a", "k_step"): os.path.join(ROOT, "profiles", "k_step_f32_cylspheres256_traffic.json"),
    ("cfg4", "k_adj"): os.path.join(ROOT, "profiles", "k_adj_f32_cyl96_traffic.json"),
}


def workload(name: str, K: int, membranes: str = "half-link"):
    import workloads as w
    cfg = w.make_config(name, membranes=membranes)
    f = cfg["f"]
    if K > len(f):
        f = np.resize(f, K)
    cfg["f_full"] = cfg["f"]
    cfg["f"] = f[:K]
    return cfg


def fields_of(G, bc, classical=False) -> int:
    # fields per q-sample: 2^(k-1) for k mirrored axes with non-zero gradient
    # (all non-zero axes mirrored, hybrid scheme: conjugate pairs), else 2^k
    nz = [a for a in range(3) if G[a] != 0.0]
    mir = [a for a in nz if bc[a] == 1]
    k = len(mir)
    if k == 0:
        return 1
    return 2 ** (k - 1) if len(mir) == len(nz) and not classical else 2 ** k


def field_sites(cfg, classical=False, qs=None) -> int:
    """Sum over all fields of the batch (or of the listed q-samples) of
    their site counts."""
    qs = range(len(cfg["gG0"])) if qs is None else qs
    return sum(fields_of(cfg["gG0"][q], cfg["bc"], classical) *
               cfg["geoms"][int(cfg["q_geom"][q])].comp.size for q in qs)


def q_sites(cfg) -> int:
    return sum(cfg["geoms"][int(g)].comp.size for g in cfg["q_geom"])


TUNE_Q = 256


def tune_probe(cfg, tune_q, classical=False, prec="f32"):
    """q-samples and steps of the autotuner's probe: the first tune_q
    q-samples, of which the library probes one q-wave (those whose two
    states fit 85 % of device memory), and about 6e9 field-site updates per
    candidate over that wave, 3 to 40 steps (short probes time the forward's
    set-up as much as its steps)."""
    import torch
    Q = len(cfg["gG0"])
    Qt = max(1, min(Q, tune_q))
    nq = 5 if cfg.get("lattice", 0) == 1 else 7
    esz = 8 if prec == "f32" else 16
    mem = (torch.cuda.get_device_properties(0).total_memory if torch.cuda.is_available()
           else 288e9)
    wave = 0.85 * mem / (2 * nq * esz)          # field sites of one q-wave
    fst = min(field_sites(cfg, classical, range(Qt)), wave)
    return Qt, max(3, min(40, int(6e9 / fst)))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_share() -> int:
    """Host cores this process may use: its CPU affinity, at most 16 (the
    host share of one GPU on the benchmark machine)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def timed(torch, fn, reps):
    """Median and all times (ms) of `reps` calls of fn, each bracketed by
    HIP events on the current stream (the stream the library launches on)."""
    stream = torch.cuda.current_stream()
    times = []
    out = None
    for _ in range(reps):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        out = fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        times.append(ev0.elapsed_time(ev1))
    return float(np.median(times)), times, out


def forward_fn(sim, cfg, K, qs=None, ckpt_every=0):
    gG0 = cfg["gG0"] if qs is None else cfg["gG0"][qs]
    qg = cfg["q_geom"] if qs is None else cfg["q_geom"][qs]
    return lambda: sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:K], gG0,
                               qg, ckpt_every=ckpt_every)


def traffic_for(key, kernel_sha, launch):
    """Measured HBM bytes per step (calibrated FETCH_SIZE + WRITE_SIZE over
    the step's launches), when the committed counter profile is of this
    kernel source and of this launch shape (the forward launch, for the
    adjoint, whose tile shape follows it)."""
    path = TRAFFIC_FILES.get(key)
    if not path:
        return None
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sha") != kernel_sha:
        return None
    if launch is None or t.get("launch", t.get("forward_launch")) == launch:
        return t.get("bytes_per_step")
    # counters taken for other launches of the same kernel source
    for o in t.get("other_launches", []):
        if o.get("launch") == launch:
            return o.get("bytes_per_step")
    return None


def cpu_baseline(cfg, budget_s: float = 25.0):
    """The FP64 oracle on the host cores, a bounded number of full-size steps
    of q-sample 0 (on mirrored faces with an oblique gradient the oracle
    steps the reflected, doubled domain, and the rate counts those sites)."""
    import oracle
    threads = cpu_share()
    g = cfg["geoms"][0]
    args = (g.comp, g.comp_phase, g.n_phase, cfg["bc"], cfg["dx"], cfg["dt"], cfg["D"],
            cfg["T2"], cfg["kappa"])
    lat = cfg.get("lattice", 0)
    doubled = oracle.needs_doubling(cfg["bc"], cfg["gG0"][0])
    sites = g.comp.size * (2 ** sum(1 for b in cfg["bc"] if b == 1) if doubled else 1)

    fw = cfg.get("f_full", cfg["f"])   # the timed forward may be shorter than n

    def run(n, th):
        t0 = time.perf_counter()
        oracle.simulate(*args, np.resize(fw, n), cfg["gG0"][0], threads=th, want_M=False,
                        lattice=lat)
        return time.perf_counter() - t0
    # per-step cost from two short runs (their difference removes the setup),
    # after one run that pays the first touch of the buffers and the thread
    # start-up
    run(1, threads)
    per = max((run(3, threads) - run(1, threads)) / 2.0, 1e-3)
    n = int(max(2, min(400, budget_s / per)))
    t_set = run(1, threads)
    t_all = run(1 + n, threads)
    dt_main = max(t_all - t_set, 1e-9)
    # the same oracle on one thread, a few steps (about a quarter of the budget)
    n1 = int(max(1, min(50, 0.25 * budget_s / (dt_main / n * threads))))
    t1_set = run(1, 1)
    t1 = max(run(1 + n1, 1) - t1_set, 1e-9)
    note = "; the oracle steps the reflected, doubled domain" if doubled else ""
    return {"value": sites * n / dt_main, "unit": "site-updates/s", "cores": threads,
            "kind": "oracle", "nproc": os.cpu_count(),
            "threads_note": "the host share of one GPU (at most 16 threads, the process's "
                            "CPU affinity)",
            "sample": f"q-sample 0 of the workload, {n} full-size steps beyond a 1-step run "
                      f"({sites} lattice sites{note}), {dt_main:.1f} s",
            "single_thread": {"value": sites * n1 / t1, "cores": 1,
                              "sample": f"{n1} full-size steps beyond a 1-step run, {t1:.1f} s"}}


def err_full_te(btl, cfg, qs, prec_pair=("f32", "f64")):
    """Signal error of FP32 storage against FP64 storage over a full echo
    time (every step), for the listed q-samples of the workload."""
    c = dict(cfg)
    c["f"] = cfg["f_full"]
    c["gG0"] = cfg["gG0"][qs]
    c["q_geom"] = cfg["q_geom"][qs]
    E32 = btl.simulate_config(c, prec=prec_pair[0]).cpu().numpy()
    E64 = btl.simulate_config(c, prec=prec_pair[1]).cpu().numpy()
    big = np.abs(E64) >= 1e-2
    rel = float(np.max(np.abs(E32 - E64)[big] / np.abs(E64)[big])) if big.any() else 0.0
    small = float(np.max(np.abs(E32 - E64)[~big])) if (~big).any() else 0.0
    return {"max_rel_E": rel, "max_abs_E_below_1e-2": small, "steps": len(c["f"]),
            "q_samples": [int(q) for q in qs], "what": "FP32 storage vs FP64 storage on the "
            "GPU path over a full echo time, every step (the FP64 path matches the FP64 "
            "oracle to 1e-12)"}


def bench_adjoint(btl, torch, args):
    """Reverse sweep of the adjoint workload: a taped forward of adj_steps
    steps with a checkpoint every adj_ckpt steps, then btl_backward for a
    linear loss in E.  The end-to-end rate counts q-sample site-updates of
    the reverse sweep (it recomputes each segment forward and runs one
    adjoint step per forward step); the adjoint kernel's time per step is
    the backward time minus the recompute steps at the measured forward
    step time of the same workload."""
    name = args.adj_workload
    Kb, C = args.adj_steps, args.adj_ckpt
    cfg = workload(name, Kb)
    if args.adj_q:
        cfg["gG0"], cfg["q_geom"] = cfg["gG0"][:args.adj_q], cfg["q_geom"][:args.adj_q]
    Q = len(cfg["gG0"])
    qs = q_sites(cfg)
    fs = field_sites(cfg)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], args.prec)
    try:
        stream = torch.cuda.current_stream().cuda_stream
        Qt, probe = tune_probe(cfg, TUNE_Q, prec=args.prec)
        sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:2], cfg["gG0"][:Qt],
                    cfg["q_geom"][:Qt])
        if args.adj_launch:
            btl.btl_set_launch(sim._h, *(int(v) for v in args.adj_launch.split(",")))
        else:
            btl.btl_autotune(sim._h, Qt, probe, stream)
        fwd_launch = dict(zip(("tile", "zc", "xcd"), btl.btl_get_launch(sim._h)))
        # forward step time on the same workload (for the adjoint kernel's
        # share of the sweep); at most 200 steps
        Kf = min(Kb, 200)
        fwd = forward_fn(sim, cfg, Kf)
        fwd()
        fwd_ms, _, _ = timed(torch, fwd, 3)
        gen = torch.Generator(device="cpu").manual_seed(0)
        g = torch.randn((Q, Kb + 1, 2), generator=gen, dtype=torch.float64).to("cuda")
        tape = forward_fn(sim, cfg, Kb, ckpt_every=C)
        log(f"adjoint: taped forward of {Kb} steps")
        tape()
        if not args.adj_cold:
            sim.backward(g)                               # warm
        times = []
        grads = None
        for r in range(1 if args.adj_cold else args.reps):
            if r > 0 or not args.adj_cold:
                tape()
            log(f"adjoint: timed reverse sweep {r + 1}")
            ms, _, grads = timed(torch, lambda: sim.backward(g), 1)
            times.append(ms)
        ms = float(np.median(times))
        stats = btl.btl_get_backward_stats(sim._h)
        # the adjoint-step launches of the last sweep, timed by the library
        # with HIP events on this stream (uniform tapes only)
        try:
            adj_timed = btl.btl_get_backward_timing(sim._h)
        except btl.BtlError:
            adj_timed = None
    finally:
        sim.close()
    fwd_step = fwd_ms / Kf
    recompute_ms = stats[0] * fwd_step
    if adj_timed is not None and adj_timed[1] > 0:
        adj_ms = adj_timed[0] / adj_timed[1]
        how = ("HIP events the library records on the launch stream around each segment's run "
               "of adjoint steps (last timed sweep), per adjoint step")
    else:
        adj_ms = max(ms - recompute_ms, 1e-9) / Kb
        how = ("estimate: backward time minus the recomputed forward steps at the measured "
               "forward step time, per adjoint step")
    nq = 5 if cfg.get("lattice", 0) == 1 else 7
    bpf = (ADJ_BYTES_PER_FIELD_SITE_F32 if args.prec == "f32" else 2 * ADJ_BYTES_PER_FIELD_SITE_F32) * nq // 7
    ach = fs * bpf / (adj_ms * 1e-3) / 1e9
    dD, dT2, dk, df = grads
    finite = bool(torch.isfinite(dD).all() and torch.isfinite(df).all())
    return {"value": qs * Kb / (ms * 1e-3), "unit": "site-updates/s",
            "workload": f"{WORKLOAD_NAMES[name]} ({name})",
            "what": "end-to-end reverse sweep (forward recompute + adjoint steps), "
                    + ("one cold sweep" if args.adj_cold else f"median of {args.reps}"),
            "steps": Kb, "ckpt_every": C, "ms_total": ms,
            "ms_all": times, "q_samples": Q, "forward_steps_recomputed": stats[0],
            "groups": stats[1], "kept_states_per_group": stats[2],
            "tape": "deferred (binomial checkpointing)" if stats[2] > 0 else "uniform",
            "forward_ms_per_step": fwd_step, "forward_launch": fwd_launch,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS,
                         "traffic": traffic_for((name, "k_adj"), source_hash(ADJOINT_SRC),
                                                fwd_launch) if args.prec == "f32" else None,
                         "kernel": f"k_adj<{'float2' if args.prec == 'f32' else 'double2'}>",
                         "bytes_per_launch_algorithmic": fs * bpf,
                         "ms_per_launch": adj_ms, "timing": how},
            "gradients_finite": finite}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="cfg3a", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=40,
                    help="warmup steps: ceil(W/K) untimed forwards of the timed K steps (at "
                         "least one), so that the graphs are captured before timing")
    ap.add_argument("--reps", type=int, default=5, help="timed forwards (median reported)")
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--scheme", default="hybrid", choices=["hybrid", "classical"],
                    help="classical: the classical LBM of Appendix A (no adjoint)")
    ap.add_argument("--membranes", default="half-link", choices=["half-link", "positions", "curved"],
                    help="positions: exact membrane positions on the links and the "
                         "general membrane condition taken normal to the link; curved: "
                         "also the membrane normals, the condition at any angle "
                         "(neither has an adjoint)")
    ap.add_argument("--launch", default=None,
                    help="tile,zc,xcd: fix the step kernel's launch (btl_set_launch) "
                         "instead of autotuning")
    ap.add_argument("--tune-q", type=int, default=TUNE_Q,
                    help="q-samples the autotuner may probe (it takes one q-wave of them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adj-workload", default="cfg4", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--adj-steps", type=int, default=400)
    ap.add_argument("--adj-ckpt", type=int, default=20)
    ap.add_argument("--adj-only", action="store_true",
                    help="only the adjoint leg (profiling)")
    ap.add_argument("--adj-launch", default=None,
                    help="tile,zc,xcd: the forward launch of the adjoint leg (its tile shape "
                         "is also the adjoint's) instead of autotuning")
    ap.add_argument("--adj-q", type=int, default=0,
                    help="the adjoint leg on the first N q-samples only (0: all)")
    ap.add_argument("--adj-cold", action="store_true",
                    help="one timed reverse sweep without a warm one (long sweeps)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64 comparison runs (profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a device copy of known size (counter calibration)")
    ap.add_argument("--copy-rate", action="store_true",
                    help="only time torch's device-to-device copy of 1.41 GB, for scale")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU; splitting the q-samples "
                                   "over several GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    btl.load_library()

    if args.calib_copy:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes}), flush=True)
        return

    if args.copy_rate:
        nbytes = 12 * 2097152 * 56          # 12 fields x 128^3 sites x 7 complex FP32
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 50
        e0.record()
        for _ in range(reps):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        rate = 2 * nbytes / (us * 1e-6) / 1e9
        print(json.dumps({"copy_bytes_each_way": nbytes, "us_per_copy": us,
                          "GBs_read_plus_write": rate, "frac_of_peak": rate / HBM_PEAK_GBS}),
              flush=True)
        return

    if args.adj_only:
        log("adjoint leg only")
        print(json.dumps({"adjoint": bench_adjoint(btl, torch, args)}), flush=True)
        return

    K = max(1, args.steps)
    W = max(0, args.warmup)
    log(f"building workload {args.workload}")
    if args.membranes != "half-link" or args.scheme != "hybrid":
        args.no_adjoint = True          # the adjoint covers hybrid half-link runs
    scheme = 0 if args.scheme == "hybrid" else 1
    cfg = workload(args.workload, 2 * K, args.membranes)
    Q = len(cfg["gG0"])
    qs = q_sites(cfg)
    fs = field_sites(cfg, args.scheme == "classical")
    lattice = cfg.get("lattice", 0)
    nq = 5 if lattice == 1 else 7
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], args.prec, scheme=scheme, lattice=lattice)
    # read nq complex populations + write nq, per field site
    bpf = (BYTES_PER_FIELD_SITE_F32 if args.prec == "f32" else BYTES_PER_FIELD_SITE_F64) * nq // 7
    stream = torch.cuda.current_stream().cuda_stream
    Qt, probe = tune_probe(cfg, max(1, args.tune_q), args.scheme == "classical", args.prec)
    tq = list(range(Qt))
    sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:2], cfg["gG0"][tq],
                cfg["q_geom"][tq])
    if args.launch:
        t, z, x = (int(v) for v in args.launch.split(","))
        btl.btl_set_launch(sim._h, t, z, x)
    elif not args.no_autotune:
        # launch shape chosen by timed probes on the first q-wave of the
        # batch (setup, untimed)
        log(f"autotune (one q-wave of the first {Qt} q-samples, {probe} steps per candidate)")
        btl.btl_autotune(sim._h, Qt, probe, stream)
    launch = dict(zip(("tile", "zc", "xcd"), btl.btl_get_launch(sim._h)))
    fwd = forward_fn(sim, cfg, K)
    fwd2 = forward_fn(sim, cfg, 2 * K)
    n_warm = max(1, -(-W // K))
    log(f"warmup: {n_warm} forward(s) of {K} steps, one of {2 * K}")
    for _ in range(n_warm):
        fwd()
    fwd2()
    torch.cuda.synchronize()
    log(f"timed: {args.reps} forwards of {K} steps")
    ms, ms_all, E = timed(torch, fwd, args.reps)
    ms_step = ms / K
    value = qs * K / (ms * 1e-3)
    bytes_step = fs * bpf
    # the step launches alone: a forward of 2K steps less one of K steps
    # (same q-waves, initial states, tables and signal launches per call)
    log(f"timed: {args.reps} forwards of {2 * K} steps")
    ms2, ms2_all, _ = timed(torch, fwd2, args.reps)
    kern_ms_step = max(ms2 - ms, 1e-9) / K
    achieved = bytes_step / (kern_ms_step * 1e-3) / 1e9
    kname = f"k_step<{'float2' if args.prec == 'f32' else 'double2'}, {'D2Q5' if nq == 5 else 'D3Q7'}>"
    traffic = None
    if args.prec == "f32" and args.membranes == "half-link" and scheme == 0:
        traffic = traffic_for((args.workload, "k_step"), source_hash(KERNEL_SRC), launch)
    # the first step of an untaped hybrid forward without curved links starts
    # from the equilibrium constants: it writes its state but reads none
    fused = scheme == 0 and args.membranes != "curved"
    bytes_fwd = K * bytes_step - (bytes_step / 2 if fused else 0)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
            "bytes_per_step_algorithmic": bytes_step,
            "ms_per_step_launches": kern_ms_step,
            "bytes_per_forward_algorithmic": bytes_fwd,
            "frac_whole_forward": bytes_fwd / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "timing": "HIP events on the launch stream around forwards of K and of 2K steps "
                      f"(medians of {args.reps}); the step launches of one step (one per "
                      "q-wave) take the difference over K; frac_whole_forward divides the "
                      "forward's algorithmic bytes (K steps, the first of which reads no "
                      "state) by the whole K-step forward (tables, signal sums included)"}
    out = {"metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{WORKLOAD_NAMES[args.workload]} ({args.workload})",
                      "q_sites": qs, "q_samples": Q, "field_sites": fs,
                      "geometries": len(cfg["geoms"]),
                      "storage": args.prec, "arithmetic": "f64", "sums": "f64",
                      "steps_per_forward": K, "membranes": args.membranes,
                      "scheme": args.scheme, "launch": launch, "reps": args.reps,
                      "ms_per_forward_all": ms_all, "ms_per_forward_2K_all": ms2_all},
           "roofline": roof}
    if not args.no_extras:
        log("FP64 comparison runs")
        # stated error vs FP64 storage over a full echo time, and the plain
        # FP64 one-sample-per-launch form as the speedup denominator
        qerr = [0, Q - 1] if Q > 1 else [0]
        out["err_vs_fp64"] = err_full_te(btl, cfg, qerr)
        sim64 = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", scheme=scheme, lattice=lattice)
        try:
            one = forward_fn(sim64, cfg, K, qs=[0])
            one()
            if not args.no_autotune:
                c1 = dict(cfg, gG0=cfg["gG0"][:1], q_geom=cfg["q_geom"][:1])
                btl.btl_autotune(sim64._h, 1, tune_probe(c1, 1, prec="f64")[1], stream)
                one()
            ms1, _, _ = timed(torch, one, args.reps)
            v1 = cfg["geoms"][int(cfg["q_geom"][0])].comp.size * K / (ms1 * 1e-3)
            out["fp64_one_q_per_launch"] = {"value": v1, "unit": "site-updates/s",
                                            "speedup_of_value": value / v1,
                                            "launch": dict(zip(("tile", "zc", "xcd"),
                                                               btl.btl_get_launch(sim64._h))),
                                            "what": "FP64 storage, q-sample 0 alone, autotuned "
                                                    "launch, median of reps"}
            allq = forward_fn(sim64, cfg, K)
            Qt64, probe64 = tune_probe(cfg, 8, prec="f64")
            sim64.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:2],
                          cfg["gG0"][:Qt64], cfg["q_geom"][:Qt64])
            if not args.no_autotune:
                btl.btl_autotune(sim64._h, Qt64, probe64, stream)
            allq()
            ms64, _, _ = timed(torch, allq, 1)
            out["fp64_batched"] = {"value": qs * K / (ms64 * 1e-3),
                                   "launch": dict(zip(("tile", "zc", "xcd"),
                                                      btl.btl_get_launch(sim64._h))),
                                   "what": "FP64 storage, the whole batch, autotuned launch"}
        finally:
            sim64.close()
    sim.close()
    if not args.no_adjoint:
        log(f"reverse sweep on {args.adj_workload}")
        out["adjoint"] = bench_adjoint(btl, torch, args)
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
