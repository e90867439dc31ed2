"""Parity of the D2Q5 lattice (Sec. 2.2, Eq. omega_i; single-layer
geometries) on the HIP path with the FP64 oracle, through the C ABI.
Tolerances as in the other parity tests."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from .test_gpu_parity import _check, _gpu

pytestmark = pytest.mark.gpu
INF = math.inf
D2Q5 = 1


def _both(cfg, prec, want_M=False):
    btl = _gpu()
    print(f"GPU D2Q5 {cfg['name']} prec={prec} shapes={[g.shape_xyz for g in cfg['geoms']]} "
          f"bc={cfg['bc']} K={len(cfg['f'])} Q={len(cfg['gG0'])}", flush=True)
    out = btl.simulate_config(cfg, prec=prec, want_M=want_M)
    Eo, Mo = oracle.simulate_config(cfg, threads=8, want_M=want_M)
    if want_M:
        Eg, Mg = out
        return Eg.cpu().numpy(), [m.cpu().numpy() for m in Mg], Eo, Mo
    return out.cpu().numpy(), None, Eo, None


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_d2q5_periodic_disks(prec):
    cfg = w.make_config("cfg2d", n=40, K=400, n_q=5)
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg2d 40^2")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bc", [[1, 1, 1], [1, 0, 0], [0, 1, 0]])
def test_d2q5_mirror_faces_oblique(prec, bc):
    g = w.cylinders_z((30, 26, 1), 0.25, seed=91, vf_target=0.55, periodic=False)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    gG = np.array([[6.0, 4.0, 0.0], [0.0, 7.0, 0.0], [-3.0, 5.0, 0.0]])
    cfg = dict(name=f"d2q5-bc{bc}", geoms=[g], bc=bc, dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([90.0, 70.0]),
               kappa=np.array([[INF, 0.02], [0.02, INF]]), f=f, gG0=gG,
               q_geom=np.zeros(len(gG), np.int32), lattice=D2Q5)
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, f"D2Q5 bc={bc}")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


def test_d2q5_with_positions_classical_and_substeps():
    btl = _gpu()
    base = w.make_config("cfg2d", n=48, K=300, n_q=3, membranes="positions")
    for extra in (dict(), dict(scheme=1), dict(substeps=3)):
        cfg = dict(base, **extra)
        if "substeps" in extra:
            cfg["f"] = np.repeat(base["f"], 3) * np.tile([0.5, 1.0, 1.5], len(base["f"]))
        Eg = btl.simulate_config(cfg, prec="f64").cpu().numpy()
        Eo, _ = oracle.simulate_config(cfg, threads=8)
        _check(Eg, Eo, "f64", f"cfg2d positions {extra}")


def test_d2q5_ragged_batch_and_errors():
    btl = _gpu()
    geoms = [w.cylinders_z((n, n + 3, 1), 0.25, seed=100 + n, vf_target=0.5) for n in (17, 29)]
    f = w.pgse_waveform(0.2, 0.6, 0.004)
    gG = np.array([[5.0, 2.0, 0.0], [1.0, -6.0, 0.0], [4.0, 4.0, 0.0]])
    cfg = dict(name="d2q5-ragged", geoms=geoms, bc=[0, 0, 0], dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([90.0, 70.0]),
               kappa=np.array([[INF, 0.05], [0.05, INF]]), f=f, gG0=gG,
               q_geom=np.array([0, 1, 1], np.int32), lattice=D2Q5)
    Eg = btl.simulate_config(cfg, prec="f64").cpu().numpy()
    Eo, _ = oracle.simulate_config(cfg, threads=8)
    _check(Eg, Eo, "f64", "D2Q5 ragged")
    sim = btl.Simulator(geoms, [0, 0, 0], "f64", lattice=D2Q5)
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], f[:20])
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(*args, np.array([[1.0, 0.0, 0.5]]))
        assert ei.value.status == btl.BTL_E_INVAL
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(*args, gG[:1], ckpt_every=5)
        assert ei.value.status == btl.BTL_E_UNSUPPORTED
        with pytest.raises(btl.BtlError) as ei:
            btl.btl_set_lattice(sim._h, 3)
        assert ei.value.status == btl.BTL_E_INVAL
    finally:
        sim.close()
    g3 = w.uniform((6, 5, 4), 0.5)
    sim = btl.Simulator([g3], [0, 0, 0], "f64", lattice=D2Q5)
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(0.01, [2.0], [INF], [[INF]], np.zeros(5), np.array([[1.0, 0.0, 0.0]]))
        assert ei.value.status == btl.BTL_E_INVAL
    finally:
        sim.close()
