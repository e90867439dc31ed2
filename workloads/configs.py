"""The benchmark workloads as seeded synthetic problems.

Each config returns a plain dict of inputs: geometries, boundary kinds per
axis, lattice spacing, time step, per-phase D and T2, the symmetric phase-pair
permeability table, the per-step waveform and one gamma*G0 vector per q-sample
(with the index of the geometry it runs on).  Parameters the paper does not
fix (time steps, directions, seeds, packing laws) are choices made here so
that runs are reproducible; they use the magnitudes of the paper's own
experiments (D ~ 1-2.5 um^2/ms, T2 ~ 10-100 ms, kappa ~ 10-50 um/s,
b = 1000 s/mm^2, PGSE timings of tens of ms).

The tissue micrographs the paper segments (Sec. 3.6) are not available;
the random cylinder, sphere and ellipsoid-cell packings stand in for them.

`n` and `K` may be overridden to get a reduced-size case with the same
structure (used by parity tests that the CPU oracle has to finish quickly).
"""
from __future__ import annotations

import math

import numpy as np

from . import geometry as geo
from . import sequences as seq

INF = math.inf

PERIODIC, MIRROR = 0, 1


def _pair_table(n_phase, pairs):
    k = np.full((n_phase, n_phase), INF)
    for (a, b), v in pairs.items():
        k[a, b] = k[b, a] = v
    return k


def _cfg1(n=32, K=None, n_q=None, seed=None):
    dx, dt = 0.5, 0.01
    delta, Delta, b = 5.0, 20.0, 1.0
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    gG = seq.gamma_g_for_b_pgse(b, delta, Delta)
    return dict(name="cfg1", geoms=[geo.uniform(n, dx)], bc=[PERIODIC] * 3,
                dx=dx, dt=dt, D=np.array([2.5]), T2=np.array([80.0]),
                kappa=_pair_table(1, {}), f=f,
                gG0=np.array([[gG, 0.0, 0.0]]), q_geom=np.zeros(1, np.int32),
                b=np.array([b]), TE=delta + Delta,
                desc="uniform 32^3 periodic free diffusion, PGSE d=5 D=20, G||x, b=1000")


def _axon_params():
    # phase 0 extracellular, phase 1 intracellular
    return (np.array([2.0, 1.0]), np.array([90.0, 70.0]),
            _pair_table(2, {(0, 1): 0.02}))


def _cfg2(n=128, K=None, n_q=None, seed=2):
    dx, dt = 0.25, 0.004
    delta, Delta, b = 10.0, 30.0, 1.0
    g = geo.cylinders_z(n, dx, seed, vf_target=0.6, periodic=False)
    D, T2, kap = _axon_params()
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    gG = seq.gamma_g_for_b_pgse(b, delta, Delta)
    dirs = seq.axon_directions()
    if n_q is not None:
        dirs = dirs[:n_q]
    return dict(name="cfg2", geoms=[g], bc=[MIRROR] * 3, dx=dx, dt=dt, D=D, T2=T2,
                kappa=kap, f=f, gG0=gG * dirs, q_geom=np.zeros(len(dirs), np.int32),
                b=np.full(len(dirs), b), TE=delta + Delta,
                desc="two-phase axon model 128^3 mirror BC, 6 directions b=1000")


def _cfg3a(n=256, K=None, n_q=None, seed=3):
    dx, dt = 0.25, 0.004
    delta, Delta = 10.0, 30.0
    g = geo.cylinders_spheres(n, dx, seed)
    D = np.array([2.0, 1.0, 1.0])
    T2 = np.array([90.0, 70.0, 70.0])
    k01, k02 = 0.02, 0.05
    kap = _pair_table(3, {(0, 1): k01, (0, 2): k02,
                          (1, 2): 1.0 / (1.0 / k01 + 1.0 / k02)})
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    dirs = seq.golden_spiral(64)
    bs = np.array([0.5, 1.0, 2.0, 3.0])
    gG0 = np.concatenate([seq.gamma_g_for_b_pgse(bb, delta, Delta) * dirs for bb in bs])
    bq = np.repeat(bs, len(dirs))
    if n_q is not None:
        sel = np.linspace(0, len(gG0) - 1, n_q).round().astype(int)
        gG0, bq = gG0[sel], bq[sel]
    return dict(name="cfg3a", geoms=[g], bc=[PERIODIC] * 3, dx=dx, dt=dt, D=D, T2=T2,
                kappa=kap, f=f, gG0=gG0, q_geom=np.zeros(len(gG0), np.int32), b=bq,
                TE=delta + Delta,
                desc="cylinders+spheres 256^3 periodic, 64 dirs x 4 b = 256 q")


def _cfg3b(n=None, K=None, n_q=None, seed=300):
    dx, dt = 0.25, 0.004
    delta, Delta, b = 10.0, 30.0, 1.0
    sizes = [96 + (96 * i) // 15 for i in range(16)]
    if n is not None:                      # reduced: scale sizes down
        sizes = [max(8, (s * n) // 192) for s in sizes]
    geoms = [geo.cylinders_z(s, dx, seed + i, vf_target=0.6, periodic=True)
             for i, s in enumerate(sizes)]
    D, T2, kap = _axon_params()
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    gG = seq.gamma_g_for_b_pgse(b, delta, Delta)
    dirs = seq.axon_directions()
    if n_q is not None:
        dirs = dirs[:n_q]
    gG0 = np.concatenate([gG * dirs for _ in geoms])
    qg = np.repeat(np.arange(len(geoms), dtype=np.int32), len(dirs))
    return dict(name="cfg3b", geoms=geoms, bc=[PERIODIC] * 3, dx=dx, dt=dt, D=D,
                T2=T2, kappa=kap, f=f, gG0=gG0, q_geom=qg, b=np.full(len(gG0), b),
                TE=delta + Delta,
                desc="16 cylinder geometries 96^3..192^3 ragged batch, 6 dirs each")


def _cfg4(n=96, K=None, n_q=None, seed=4):
    dx, dt = 0.25, 0.01
    delta, Delta, b = 10.0, 30.0, 1.0
    g = geo.cylinders_z(n, dx, seed, vf_target=0.6, periodic=True)
    D, T2, kap = _axon_params()
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    gG = seq.gamma_g_for_b_pgse(b, delta, Delta)
    dirs = seq.golden_spiral(30 if n_q is None else n_q)
    return dict(name="cfg4", geoms=[g], bc=[PERIODIC] * 3, dx=dx, dt=dt, D=D, T2=T2,
                kappa=kap, f=f, gG0=gG * dirs, q_geom=np.zeros(len(dirs), np.int32),
                b=np.full(len(dirs), b), TE=delta + Delta,
                desc="adjoint workload 96^3 cylinders periodic, 30 q, K=4000")


def _cfg5(n=512, K=None, n_q=None, seed=5):
    dx, dt = 0.2, 0.002
    # reduced boxes shrink the cells with the box (at least 3-8 voxels)
    sc = max(n / 512.0, 0.2)
    g = geo.ellipsoid_cells(n, dx, seed, semi=(3.0 * sc, 8.0 * sc))
    D = np.array([2.5, 1.5, 1.0])
    T2 = np.array([90.0, 70.0, 60.0])
    kap = _pair_table(3, {(0, 1): 0.03, (1, 2): 0.1})
    kap[1, 1] = 0.03 / 2.0           # two cell membranes in series
    f = seq.ogse_cosine_waveform(20.0, 1, 25.0, dt)
    if K is not None:
        f = f[:K]
    full = seq.ogse_cosine_waveform(20.0, 1, 25.0, dt)
    gG = math.sqrt(1.0 / seq.b_of_waveform(full, dt))
    dirs = seq.golden_spiral(32 if n_q is None else n_q)
    return dict(name="cfg5", geoms=[g], bc=[PERIODIC] * 3, dx=dx, dt=dt, D=D, T2=T2,
                kappa=kap, f=f, gG0=gG * dirs, q_geom=np.zeros(len(dirs), np.int32),
                b=np.full(len(dirs), 1.0), TE=45.0,
                desc="three-phase ellipsoid cells 512^3, cosine OGSE 50 Hz, 32 dirs")


def _cfg2d(n=512, K=None, n_q=None, seed=6):
    # two-dimensional axon cross-sections on the D2Q5 lattice (Sec. 2.2):
    # a periodic 128^2 disk packing (the cfg2 law) tiled to n x n, in-plane
    # gradient directions at four b-values
    dx, dt = 0.25, 0.004
    delta, Delta = 10.0, 30.0
    base = geo.cylinders_z((min(n, 128), min(n, 128), 1), dx, seed, vf_target=0.6,
                           periodic=True)
    r = max(1, n // 128)
    g = geo.tile_xy(base, r, r) if r > 1 else base
    D, T2, kap = _axon_params()
    f = seq.pgse_waveform(delta, Delta, dt)
    if K is not None:
        f = f[:K]
    th = np.pi * (np.arange(64) + 0.5) / 64
    dirs = np.stack([np.cos(th), np.sin(th), np.zeros_like(th)], axis=1)
    bs = np.array([0.5, 1.0, 2.0, 3.0])
    gG0 = np.concatenate([seq.gamma_g_for_b_pgse(bb, delta, Delta) * dirs for bb in bs])
    bq = np.repeat(bs, len(dirs))
    if n_q is not None:
        sel = np.linspace(0, len(gG0) - 1, n_q).round().astype(int)
        gG0, bq = gG0[sel], bq[sel]
    return dict(name="cfg2d", geoms=[g], bc=[PERIODIC] * 3, dx=dx, dt=dt, D=D, T2=T2,
                kappa=kap, f=f, gG0=gG0, q_geom=np.zeros(len(gG0), np.int32), b=bq,
                TE=delta + Delta, lattice=1,
                desc="2D axon cross-sections 512^2 (D2Q5), 64 in-plane dirs x 4 b = 256 q")


CONFIGS = {"cfg1": _cfg1, "cfg2": _cfg2, "cfg3a": _cfg3a, "cfg3b": _cfg3b,
           "cfg4": _cfg4, "cfg5": _cfg5, "cfg2d": _cfg2d}


def make_config(name: str, n=None, K=None, n_q=None, seed=None,
                membranes: str = "half-link") -> dict:
    """Build a config; n/K/n_q/seed override the full-size defaults.

    membranes="positions" attaches to every geometry the exact positions
    where its analytic surfaces cut the lattice links (`geometry.link_delta`),
    for the general membrane condition with the membrane taken normal to the
    link; "curved" also attaches the surface normals at those points
    (`geometry.link_normal`) for the condition at any angle; the default
    leaves them out (every membrane at mid-link)."""
    fn = CONFIGS[name]
    kw = {}
    if n is not None:
        kw["n"] = n
    if seed is not None:
        kw["seed"] = seed
    cfg = fn(K=K, n_q=n_q, **kw)
    if membranes in ("positions", "curved"):
        for g in cfg["geoms"]:
            g.link_delta = geo.link_delta(g)
            if membranes == "curved":
                g.link_normal = geo.link_normal(g)
        cfg["name"] += "+" + membranes
    elif membranes != "half-link":
        raise ValueError("membranes must be 'half-link', 'positions' or 'curved'")
    return cfg
