"""Parity of the general membrane condition at any angle (membrane positions
and normals on the links; Sec. 2.4.2 and Appendix B) on the HIP path with
the FP64 oracle, through the C ABI.

The library builds per-link term lists on the host (they depend on kappa,
dt and the lattice) and the step kernel applies them; the oracle evaluates
the side relations and the 2 x 2 permeability system per link and step.
Same tolerances as the other parity tests: FP64 storage to rounding order
(|dE| <= 1e-12 |E| + 1e-14), FP32 storage |dE| <= 1e-5 |E| where
|E| >= 1e-2 and 1e-7 absolute below that.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from .test_gpu_parity import _check, _gpu

pytestmark = pytest.mark.gpu
INF = math.inf


def _both(cfg, prec, want_M=False, **options):
    btl = _gpu()
    print(f"GPU curved {cfg['name']} prec={prec} shapes={[g.shape_xyz for g in cfg['geoms']]} "
          f"K={len(cfg['f'])} Q={len(cfg['gG0'])} {options}", flush=True)
    out = btl.simulate_config(cfg, prec=prec, want_M=want_M, **options)
    Eo, Mo = oracle.simulate_config(cfg, threads=8, want_M=want_M)
    if want_M:
        Eg, Mg = out
        return Eg.cpu().numpy(), [m.cpu().numpy() for m in Mg], Eo, Mo
    return out.cpu().numpy(), None, Eo, None


def _strong(cfg, rad=4.0):
    # gradients scaled so that the phase across the largest lattice reaches
    # `rad` over the run: the magnetization varies strongly near the
    # membranes (with the configs' own gradients and these short runs it
    # stays nearly uniform, where every membrane rule agrees)
    L = max(max(g.shape_xyz) for g in cfg["geoms"]) * cfg["dx"]
    T = len(cfg["f"]) * cfg["dt"]
    gn = np.linalg.norm(cfg["gG0"], axis=1).max()
    cfg["gG0"] = cfg["gG0"] * (rad / (gn * T * L))
    return cfg


def _tilted(n=40, K=300, n_q=3):
    # D2Q5 box crossed by straight membranes whose normal makes 26.6 degrees
    # with x: two permeable membranes between walls, in-plane gradients
    X = 10.0 * math.sqrt(5.0)
    dx = X / n
    g = w.angled_slabs_2d(n, dx, [2.03, 4.71, 7.33])
    g.link_normal = w.link_normal(g)
    D = np.array([1.5, 1.0, 2.0])
    dt = 0.3 * dx * dx / (3.0 * 1.0)
    kap = np.array([[INF, 0.0, 0.0], [0.0, INF, 0.05], [0.0, 0.05, INF]])
    ang = np.linspace(0.0, math.pi, n_q, endpoint=False) + 0.3
    gG0 = 0.25 * np.stack([np.cos(ang), np.sin(ang), np.zeros(n_q)], axis=1)
    return dict(name="tilted_slabs", geoms=[g], bc=[0, 0, 0], dx=dx, dt=dt, D=D,
                T2=np.array([60.0, 50.0, 80.0]), kappa=kap, f=w.pgse_waveform(2.0, 6.0, dt)[:K],
                gG0=gG0, q_geom=np.zeros(n_q, np.int32), lattice=1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_curved_d2q5_tilted_slabs(prec):
    cfg = _tilted()
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "tilted slabs")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"tilted slabs M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_curved_periodic_cylinders(prec):
    cfg = _strong(w.make_config("cfg4", n=(20, 18, 6), K=300, n_q=4, membranes="curved"))
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg4 curved")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"cfg4 curved M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_curved_mirror_oblique_image_fields(prec):
    # mirrored faces with oblique gradients: the image fields use the
    # geometry's term lists in their own frame
    cfg = _strong(w.make_config("cfg2", n=20, K=300, membranes="curved"))
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg2 curved")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"cfg2 curved M_final q={q}")


def test_curved_spheres_and_cells():
    cfg = _strong(w.make_config("cfg3a", n=24, K=200, n_q=3, membranes="curved"))
    Eg, _, Eo, _ = _both(cfg, "f64")
    _check(Eg, Eo, "f64", "cfg3a curved")
    cfg = _strong(w.make_config("cfg5", n=28, K=200, n_q=3, membranes="curved"))
    Eg, _, Eo, _ = _both(cfg, "f32")
    _check(Eg, Eo, "f32", "cfg5 curved")


def test_curved_ragged_batch_and_kappa_limits():
    # one batch mixing geometries with normals, with positions only and with
    # neither; then the same with an impermeable (kappa = 0) and a missing
    # (kappa = inf) membrane, which rebuilds the term lists
    cfg = w.make_config("cfg3b", n=16, K=120, n_q=1)
    for i in (1, 5):
        g = cfg["geoms"][i]
        g.link_delta = w.link_delta(g)
        g.link_normal = w.link_normal(g)
    cfg["geoms"][3].link_delta = w.link_delta(cfg["geoms"][3])
    cfg["q_geom"] = np.array([1, 3, 5, 0, 1, 5, 2, 3, 1, 4, 5, 0], np.int32)
    cfg["gG0"] = cfg["gG0"][:12] * np.linspace(0.5, 1.5, 12)[:, None]
    cfg["name"] = "cfg3b mixed"
    _strong(cfg)
    Eg, _, Eo, _ = _both(cfg, "f64")
    _check(Eg, Eo, "f64", "cfg3b mixed")
    P = len(cfg["D"])
    for k in (0.0, INF):
        kap = np.array(cfg["kappa"], dtype=np.float64).copy()
        kap[0, 1:] = kap[1:, 0] = k
        c = dict(cfg, kappa=kap, name=f"cfg3b mixed kappa01={k}")
        Eg, _, Eo, _ = _both(c, "f64")
        _check(Eg, Eo, "f64", f"cfg3b mixed kappa {k}")
    assert P >= 2


def test_curved_tables_follow_the_constants():
    # one simulator, forwards with changing dt and kappa (graphs on): every
    # forward matches the oracle, and the first result comes back exactly
    btl = _gpu()
    cfg = _strong(w.make_config("cfg4", n=(18, 16, 5), K=80, n_q=2, membranes="curved"))
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    try:
        runs = []
        for dt_scale, ks in [(1.0, 1.0), (0.5, 1.0), (1.0, 3.0), (1.0, 1.0)]:
            kap = np.array(cfg["kappa"], dtype=np.float64) * ks
            dt = cfg["dt"] * dt_scale
            E = sim.forward(dt, cfg["D"], cfg["T2"], kap, cfg["f"], cfg["gG0"],
                            cfg["q_geom"]).cpu().numpy()
            c = dict(cfg, dt=dt, kappa=kap)
            Eo, _ = oracle.simulate_config(c, threads=8)
            _check(E, Eo, "f64", f"dt x{dt_scale} kappa x{ks}")
            runs.append(E)
        assert np.array_equal(runs[0], runs[-1])
    finally:
        sim.close()


@pytest.mark.parametrize("shape,zc,order", [(0, 0, 1), (1, 3, 3), (2, 0, 2), (3, 7, 1), (5, 1, 3)])
def test_curved_every_launch_shape(shape, zc, order):
    btl = _gpu()
    cfg = _strong(w.make_config("cfg2", n=20, K=120, membranes="curved"))
    Eo, _ = oracle.simulate_config(cfg, threads=8)
    print(f"GPU curved shape {shape} zc {zc} order {order}", flush=True)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f32", launch=(shape, zc, order))
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        cfg["q_geom"]).cpu().numpy()
    finally:
        sim.close()
    _check(E, Eo, "f32", f"curved shape {shape} zc {zc}")


def test_curved_errors_and_noalloc():
    btl = _gpu()
    import torch
    cfg = w.make_config("cfg4", n=(16, 14, 5), K=40, n_q=1, membranes="curved")
    g = cfg["geoms"][0]
    # normals need positions
    ld = g.link_delta
    g.link_delta = None
    with pytest.raises(btl.BtlError) as ei:
        btl.Simulator([g], cfg["bc"], "f64")
    assert ei.value.status == btl.BTL_E_INVAL
    g.link_delta = ld
    # a zero normal on a membrane link
    bad = g.link_normal.copy()
    z, y, x = [v[0] for v in np.nonzero(g.comp != np.roll(g.comp, -1, axis=2))]
    bad[0, :, z, y, x] = 0.0      # the x link of a membrane
    ln = g.link_normal
    g.link_normal = bad
    with pytest.raises(btl.BtlError) as ei:
        btl.Simulator([g], cfg["bc"], "f64")
    assert ei.value.status == btl.BTL_E_INVAL
    g.link_normal = ln
    sim = btl.Simulator([g], cfg["bc"], "f64")
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"], cfg["q_geom"])
        # the adjoint does not cover the general membrane condition
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(*args, ckpt_every=10)
        assert ei.value.status == btl.BTL_E_UNSUPPORTED
        E1 = sim.forward(*args).cpu().numpy()
        E2 = sim.forward(*args, noalloc=True).cpu().numpy()
        assert np.array_equal(E1, E2)
        # new constants: the allocation-free call rebuilds the tables in place
        a2 = (cfg["dt"] * 0.5,) + args[1:]
        E3 = sim.forward(*a2, noalloc=True).cpu().numpy()
        E4 = sim.forward(*a2).cpu().numpy()
        assert np.array_equal(E3, E4)
        torch.cuda.synchronize()
    finally:
        sim.close()
