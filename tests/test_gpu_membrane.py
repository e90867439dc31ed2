"""Parity of the general membrane condition (membrane positions on the links,
theta = 0 form of Eqs. B2a_text/B2b_text with Eqs. B4a-B4c) on the HIP path
with the FP64 oracle, through the C ABI.

Same tolerances as the other parity tests: FP64 storage to rounding order
(|dE| <= 1e-12 |E| + 1e-14), FP32 storage |dE| <= 1e-5 |E| where |E| >= 1e-2
and 1e-7 absolute below that.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from .test_gpu_parity import _check, _gpu

pytestmark = pytest.mark.gpu
INF = math.inf


def _both(cfg, prec, want_M=False):
    btl = _gpu()
    print(f"GPU membranes {cfg['name']} prec={prec} shapes={[g.shape_xyz for g in cfg['geoms']]} "
          f"K={len(cfg['f'])} Q={len(cfg['gG0'])}", flush=True)
    out = btl.simulate_config(cfg, prec=prec, want_M=want_M)
    Eo, Mo = oracle.simulate_config(cfg, threads=8, want_M=want_M)
    if want_M:
        Eg, Mg = out
        return Eg.cpu().numpy(), [m.cpu().numpy() for m in Mg], Eo, Mo
    return out.cpu().numpy(), None, Eo, None


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_positions_periodic_cylinders(prec):
    cfg = w.make_config("cfg4", n=(20, 18, 6), K=400, n_q=4, membranes="positions")
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg4 positions")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_positions_mirror_oblique_image_fields(prec):
    # mirrored faces with oblique gradients: the image fields share the
    # geometry's membrane positions in their own frame
    cfg = w.make_config("cfg2", n=20, K=400, membranes="positions")
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg2 positions")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_positions_spheres_and_cells(prec):
    cfg = w.make_config("cfg3a", n=24, K=250, n_q=3, membranes="positions")
    Eg, _, Eo, _ = _both(cfg, prec)
    _check(Eg, Eo, prec, "cfg3a positions")
    cfg = w.make_config("cfg5", n=28, K=250, n_q=3, membranes="positions")
    Eg, _, Eo, _ = _both(cfg, prec)
    _check(Eg, Eo, prec, "cfg5 positions")


def test_positions_ragged_batch_with_and_without():
    # one batch mixing a geometry with positions and one without
    btl = _gpu()
    cfg = w.make_config("cfg3b", n=40, K=300, n_q=2)
    cfg["geoms"][1].link_delta = w.link_delta(cfg["geoms"][1])
    cfg["geoms"][5].link_delta = w.link_delta(cfg["geoms"][5])
    Eg = btl.simulate_config(cfg, prec="f64").cpu().numpy()
    Eo, _ = oracle.simulate_config(cfg, threads=8)
    _check(Eg, Eo, "f64", "cfg3b mixed")


def test_positions_with_classical_scheme_and_kappa_limits():
    btl = _gpu()
    cfg = w.make_config("cfg4", n=(16, 14, 5), K=300, n_q=2, membranes="positions")
    for scheme in (0, 1):
        for kap in (0.0, 0.02, 3.0):
            c = dict(cfg, scheme=scheme, kappa=np.array([[INF, kap], [kap, INF]]))
            Eg = btl.simulate_config(c, prec="f64").cpu().numpy()
            Eo, _ = oracle.simulate_config(c, threads=8)
            _check(Eg, Eo, "f64", f"scheme={scheme} kappa={kap}")


def test_mid_link_positions_equal_half_link():
    btl = _gpu()
    cfg = w.make_config("cfg4", n=(16, 14, 5), K=300, n_q=2)
    E0 = btl.simulate_config(cfg, prec="f64").cpu().numpy()
    g = cfg["geoms"][0]
    g.link_delta = np.full((3,) + g.comp.shape, 0.5, np.float32)
    E1 = btl.simulate_config(cfg, prec="f64").cpu().numpy()
    assert np.max(np.abs(E1 - E0)) < 1e-14


def test_positions_errors():
    btl = _gpu()
    cfg = w.make_config("cfg4", n=(16, 14, 5), K=40, n_q=1, membranes="positions")
    g = cfg["geoms"][0]
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        ckpt_every=10)
        assert ei.value.status == btl.BTL_E_UNSUPPORTED
    finally:
        sim.close()
    bad = g.link_delta.copy()
    a, z, y, x = [v[0] for v in np.nonzero(bad != 0.5)]
    bad[a, z, y, x] = 1.0
    g.link_delta = bad
    with pytest.raises(btl.BtlError) as ei:
        btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    assert ei.value.status == btl.BTL_E_INVAL


@pytest.mark.parametrize("shape,zc", [(5, 3), (1, 4), (3, 0)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_positions_every_launch_shape(shape, zc, prec):
    # the general condition walks each column chunk one site at a time: runs
    # of 256 sites with 3-site chunks (a ragged last chunk), 32x8 tiles with
    # 4-site chunks and 128x2 tiles over whole columns, against the oracle
    btl = _gpu()
    import torch
    cfg = w.make_config("cfg2", n=20, K=150, membranes="positions")
    print(f"GPU membranes shape={shape} zc={zc} prec={prec}", flush=True)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec)
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"])
        btl.btl_set_launch(sim._h, shape, zc, -1)
        assert btl.btl_get_launch(sim._h)[:2] == (shape, zc)
        E = sim.forward(*args, cfg["f"], cfg["gG0"]).cpu().numpy()
    finally:
        sim.close()
    Eo, _ = oracle.simulate_config(cfg, threads=8)
    _check(E, Eo, prec, f"positions shape {shape} zc {zc}")
