"""Benchmark: q-batched lattice site-updates/s of the hybrid LBM Bloch-Torrey
step on one MI355X, with the HBM roofline of the step kernel and the FP64
CPU oracle timed on the host as a baseline.

Workload: the two-phase axon model -- 128^3 lattice, dx = 0.25 um, mirroring
outer faces, z-cylinders with Gamma(4, mean 1 um) radii packed to ~60 %,
D 2.0/1.0 um^2/ms, T2 90/70 ms, kappa 0.02 um/ms, PGSE delta 10 Delta 30 ms,
6 oblique directions at b = 1000 s/mm^2, dt = 0.004 ms.  Each oblique
direction on mirrored faces carries two fields (the primary and one
reflected image), so one step updates 12 fields of 2,097,152 sites.

A benchmark step is one lattice time step of the whole q-batch: stream with
boundaries and membranes, reaction, signal reduction and collision for
every q-sample.  `value` counts q-sample site-updates (6 x 128^3 per step).

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload cfg2]
(--workload selects one of the other synthetic workloads; the default is the
one described above.)
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_f32_axon128_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1907_00908_amd", "csrc", "btl_kernels.hip")


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


WORKLOAD_NAMES = {
    "cfg1": "uniform 32^3 periodic free diffusion, PGSE, G || x, b=1000 (plain case)",
    "cfg2": "two-phase axon model 128^3, mirror BC, 6 oblique directions, b=1000",
    "cfg3a": "cylinders+spheres 256^3 periodic, 64 directions x 4 b-values = 256 q",
    "cfg3b": "16 cylinder geometries 96^3..192^3 (ragged batch), 6 directions each",
    "cfg4": "two-phase cylinders 96^3 periodic, 30 directions",
    "cfg5": "three-phase ellipsoid cells 512^3 periodic, cosine OGSE, 32 directions",
    "cfg2d": "2D axon cross-sections 512^2 on the D2Q5 lattice, 64 in-plane dirs x 4 b-values",
}


def workload(name: str, K: int, membranes: str = "half-link"):
    import workloads as w
    cfg = w.make_config(name, membranes=membranes)
    f = cfg["f"]
    if K > len(f):
        f = np.resize(f, K)
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


def field_sites(cfg, classical=False) -> int:
    """Sum over all fields of the batch of their site counts."""
    return sum(fields_of(G, cfg["bc"], classical) * cfg["geoms"][int(g)].comp.size
               for G, g in zip(cfg["gG0"], cfg["q_geom"]))


def q_sites(cfg) -> int:
    return sum(cfg["geoms"][int(g)].comp.size for g in cfg["q_geom"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_forward(sim, cfg, K, prec_bytes, reps=1):
    import torch
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    best = None
    E = None
    for _ in range(reps):
        torch.cuda.synchronize()
        ev0.record(stream)
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:K],
                        cfg["gG0"], cfg["q_geom"])
        ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        best = ms if best is None else min(best, ms)
    return best, E


def cpu_baseline(cfg, budget_s: float = 25.0):
    """The FP64 oracle on the host cores, a bounded number of full-size steps
    of q-sample 0 (oblique gradient on mirrored faces: the oracle runs the
    reflected, doubled domain)."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    g = cfg["geoms"][0]
    args = (g.comp, g.comp_phase, g.n_phase, cfg["bc"], cfg["dx"], cfg["dt"], cfg["D"],
            cfg["T2"], cfg["kappa"])
    lat = cfg.get("lattice", 0)

    def run(n):
        t0 = time.perf_counter()
        oracle.simulate(*args, cfg["f"][:n], cfg["gG0"][0], threads=threads, want_M=False,
                        lattice=lat)
        return time.perf_counter() - t0
    # per-step cost from two short runs (their difference removes the setup),
    # after one run that pays the first touch of the buffers and the thread
    # start-up
    run(1)
    per = max((run(3) - run(1)) / 2.0, 1e-3)
    n = int(max(1, min(400, budget_s / per)))
    t0 = time.perf_counter()
    oracle.simulate(*args, cfg["f"][:n], cfg["gG0"][0], threads=threads, want_M=False,
                    lattice=lat)
    t1 = time.perf_counter()
    sites = g.comp.size
    note = ("; the oracle steps the reflected, doubled domain"
            if oracle.needs_doubling(cfg["bc"], cfg["gG0"][0]) else "")
    # the same oracle on one thread, a few steps (about a quarter of the
    # budget); a one-step run's time is subtracted to remove the setup
    def run1(n):
        t = time.perf_counter()
        oracle.simulate(*args, cfg["f"][:n], cfg["gG0"][0], threads=1, want_M=False,
                        lattice=lat)
        return time.perf_counter() - t
    per_main = (t1 - t0) / n
    n1 = int(max(2, min(50, 0.25 * budget_s / (per_main * threads))))
    t_setup = run1(1)
    t_run = run1(1 + n1)
    t2, t3 = 0.0, max(t_run - t_setup, 1e-9)
    return {"value": sites * n / (t1 - t0), "unit": "site-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"q-sample 0 of the workload, {n} full-size steps ({sites} REV sites"
                      f"{note}), {t1 - t0:.1f} s",
            "single_thread": {"value": sites * n1 / (t3 - t2), "cores": 1,
                              "sample": f"{n1} full-size steps beyond a 1-step run, "
                                        f"{t3 - t2:.1f} s"}}


def bench_adjoint(btl, torch, sim, cfg, args, fwd_ms_step, fs, qs, Q):
    """Reverse sweep of the same workload: forward with a checkpoint every
    adj_ckpt steps, then btl_backward for a linear loss in E.  The end-to-end
    rate counts q-sample site-updates of the reverse sweep (it recomputes
    each segment forward and runs one adjoint step per forward step)."""
    Kb, C = min(args.adj_steps, len(cfg["f"])), args.adj_ckpt
    c = dict(cfg)
    c["f"] = cfg["f"][:Kb]
    stream = torch.cuda.current_stream()
    E = sim.forward(c["dt"], c["D"], c["T2"], c["kappa"], c["f"], c["gG0"], c["q_geom"],
                    ckpt_every=C)
    gen = torch.Generator(device="cpu").manual_seed(0)
    g = torch.randn((Q, Kb + 1, 2), generator=gen, dtype=torch.float64).to(E.device)
    P = len(c["D"])
    sim.backward(g, P, Kb)                      # warm
    sim.forward(c["dt"], c["D"], c["T2"], c["kappa"], c["f"], c["gG0"], c["q_geom"],
                ckpt_every=C)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    dD, dT2, dk, df = sim.backward(g, P, Kb)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    nseg = (Kb + C - 1) // C
    recompute_ms = (Kb - nseg) * fwd_ms_step
    adj_ms = max(ms - recompute_ms, 1e-9) / Kb
    # read the adjoint and the forward state, write the adjoint: 3 x nq complex
    nq = 5 if cfg.get("lattice", 0) == 1 else 7
    bpf = (168 if args.prec == "f32" else 336) * nq // 7
    ach = fs * bpf / (adj_ms * 1e-3) / 1e9
    finite = bool(torch.isfinite(dD).all() and torch.isfinite(df).all())
    return {"value": qs * Kb / (ms * 1e-3), "unit": "site-updates/s",
            "what": "end-to-end reverse sweep (segment recompute + adjoint step)",
            "steps": Kb, "ckpt_every": C, "ms_total": ms,
            "adjoint_kernel": {"ms_per_step_est": adj_ms,
                               "bytes_per_launch_algorithmic": fs * bpf,
                               "achieved_GBs": ach, "frac": ach / HBM_PEAK_GBS,
                               "estimate": "backward time minus the recompute steps at the "
                                           "measured forward step time"},
            "gradients_finite": finite}


def traffic_for(launch):
    """Measured HBM bytes per step launch, when the committed counter
    profile is of this kernel source and of this launch shape."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    if t.get("launch") == launch:
        return t["bytes_per_launch"]
    row = t.get("by_launch", {}).get(f"{launch['tile']},{launch['zc']},{launch['xcd']}")
    return row["bytes_per_launch"] if row else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--prec", default="f32", choices=["f32", "f64"])
    ap.add_argument("--scheme", default="hybrid", choices=["hybrid", "classical"],
                    help="classical: the classical LBM of Appendix A (no adjoint)")
    ap.add_argument("--membranes", default="half-link", choices=["half-link", "positions"],
                    help="positions: exact membrane positions on the links and the "
                         "general membrane condition (no adjoint)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adj-steps", type=int, default=400)
    ap.add_argument("--adj-ckpt", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64 comparison runs (profiling)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a device copy of known size (counter calibration)")
    ap.add_argument("--copy-rate", action="store_true",
                    help="only time torch's device-to-device copy of 1.41 GB (the step "
                         "kernel's per-launch reads of the default workload), for scale")
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

    K, W = args.steps, args.warmup
    log(f"building workload {args.workload}")
    if args.membranes == "positions" or args.scheme != "hybrid":
        args.no_adjoint = True          # the adjoint covers hybrid half-link runs
    scheme = 0 if args.scheme == "hybrid" else 1
    cfg = workload(args.workload, max(K, W, 0 if args.no_adjoint else args.adj_steps),
                   args.membranes)
    Q = len(cfg["gG0"])
    qs = q_sites(cfg)
    fs = field_sites(cfg, args.scheme == "classical")
    sites = cfg["geoms"][0].comp.size
    lattice = cfg.get("lattice", 0)
    nq = 5 if lattice == 1 else 7
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], args.prec, scheme=scheme, lattice=lattice)
    # read nq complex populations + write nq, per field site
    bpf = (BYTES_PER_FIELD_SITE_F32 if args.prec == "f32" else BYTES_PER_FIELD_SITE_F64) * nq // 7
    log("first forward")
    time_forward(sim, cfg, max(W, 1), bpf)
    if not args.no_autotune:
        # launch shape chosen by timed probes of this workload (setup, untimed)
        probe = max(2, min(40, int(1.5e9 / fs)))   # about 1.5e9 field-site updates per candidate
        log(f"autotune ({probe} steps per candidate)")
        btl.btl_autotune(sim._h, Q, probe, torch.cuda.current_stream().cuda_stream)
    launch = dict(zip(("tile", "zc", "xcd"), btl.btl_get_launch(sim._h)))
    if W > 0:
        log("warmup")
        time_forward(sim, cfg, W, bpf)
    log("timed forward")
    ms, E = time_forward(sim, cfg, K, bpf)
    ms_step = ms / K
    value = qs * K / (ms * 1e-3)
    bytes_launch = fs * bpf
    achieved = bytes_launch / (ms_step * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (traffic_for(launch) if args.workload == "cfg2" and args.prec == "f32"
                        and args.membranes == "half-link" and scheme == 0 else None),
            "kernel": f"k_step<{'float2' if args.prec == 'f32' else 'double2'}, {'D2Q5' if nq == 5 else 'D3Q7'}>",
            "bytes_per_launch_algorithmic": bytes_launch}
    out = {"metric": METRIC, "value": value, "unit": "site-updates/s", "n_gpus": 1,
           "steps": K, "warmup": W, "ms_per_step": ms_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{WORKLOAD_NAMES[args.workload]} ({args.workload})",
                      "q_sites": qs, "q_samples": Q, "field_sites": fs,
                      "geometries": len(cfg["geoms"]),
                      "storage": args.prec, "steps_per_forward": K,
                      "membranes": args.membranes, "scheme": args.scheme,
                      "launch": launch},
           "roofline": roof}
    if not args.no_extras:
        log("FP64 comparison runs")
        # stated error vs FP64 storage over the same steps, and the plain FP64
        # one-sample-per-launch form as the speedup denominator
        sim64 = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", scheme=scheme, lattice=lattice)
        ms64, E64 = time_forward(sim64, cfg, K, BYTES_PER_FIELD_SITE_F64)
        e32 = E.cpu().numpy()
        e64 = E64.cpu().numpy()
        big = np.abs(e64) >= 1e-2
        rel = np.max(np.abs(e32 - e64)[big] / np.abs(e64)[big])
        out["err_vs_fp64"] = {"max_rel_E": float(rel), "steps": K}
        one = dict(cfg)
        one["gG0"] = cfg["gG0"][:1]
        one["q_geom"] = cfg["q_geom"][:1]
        ms1, _ = time_forward(sim64, one, K, BYTES_PER_FIELD_SITE_F64)
        v1 = cfg["geoms"][int(cfg["q_geom"][0])].comp.size * K / (ms1 * 1e-3)
        out["fp64_one_q_per_launch"] = {"value": v1, "unit": "site-updates/s",
                                        "speedup_of_value": value / v1}
        out["fp64_batched"] = {"value": qs * K / (ms64 * 1e-3)}
        sim64.close()
    state_gb = fs * (8 if args.prec == "f32" else 16) * (5 if cfg.get("lattice", 0) == 1 else 7) / 1e9
    adj_states = min(args.adj_steps, K) / args.adj_ckpt + args.adj_ckpt + 4
    if not args.no_adjoint and state_gb * adj_states > 120.0:
        out["adjoint"] = {"skipped": f"tape would need {state_gb * adj_states:.0f} GB"}
    elif not args.no_adjoint:
        log("reverse sweep")
        out["adjoint"] = bench_adjoint(btl, torch, sim, cfg, args, ms_step, fs, qs, Q)
    sim.close()
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
