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
            btl.btl_set_lattice(sim._h, 3)
        assert ei.value.status == btl.BTL_E_INVAL
        # a geometry index out of range is refused before the D2Q5 checks
        # read the geometry it names
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(*args, np.array([[1.0, 0.0, 0.0]]), q_geom=[7])
        assert ei.value.status == btl.BTL_E_INVAL
        assert "q_geom" in str(ei.value)
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


def _loss_fd(cfg, a, b, which, idx, h):
    vals = []
    for sgn in (1, -1):
        c = dict(cfg)
        arr = np.array(cfg[which], float).copy()
        arr[idx] += sgn * h
        if which == "kappa":
            arr[idx[::-1]] = arr[idx]
        c[which] = arr
        E, _ = oracle.simulate_config(c, threads=8)
        vals.append(float(np.sum(a * E.real + b * E.imag)))
    return (vals[0] - vals[1]) / (2 * h)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-3)])
@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1]])
def test_d2q5_adjoint_vs_oracle_fd(prec, tol, bc):
    # the adjoint on the D2Q5 lattice (eps_D = 1/3 in tau and in the
    # membrane number), gradients of D, T2, kappa, f and gamma G0 (x, y)
    import torch
    btl = _gpu()
    g = w.cylinders_z((18, 15, 1), 0.25, seed=93, vf_target=0.5, periodic=bc[0] == 0)
    f = w.pgse_waveform(0.12, 0.36, 0.004)
    gG = np.array([[7.0, 4.0, 0.0], [0.0, 6.0, 0.0]])
    cfg = dict(name="d2q5-adj", geoms=[g], bc=bc, dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([60.0, 40.0]),
               kappa=np.array([[INF, 0.05], [0.05, INF]]), f=f, gG0=gG,
               q_geom=np.zeros(len(gG), np.int32), lattice=D2Q5)
    Q, K = len(gG), len(f)
    r = np.random.default_rng(11)
    a, b = r.normal(size=(Q, K + 1)), r.normal(size=(Q, K + 1))
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, lattice=D2Q5, grad_gG0=True)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], f, gG, cfg["q_geom"],
                        ckpt_every=25)
        gt = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        dD, dT2, dk, df, dG = [t.cpu().numpy() for t in sim.backward(gt, 2, K, grad_gG0=True)]
    finally:
        sim.close()
    checks = [("D", 0, dD[0], 1e-5), ("D", 1, dD[1], 1e-5), ("T2", 0, dT2[0], 1e-3),
              ("kappa", (0, 1), dk[0, 1] + dk[1, 0], 1e-6), ("f", 10, df[10], 1e-4),
              ("f", 70, df[70], 1e-4), ("gG0", (0, 0), dG[0, 0], 2e-4),
              ("gG0", (0, 1), dG[0, 1], 2e-4), ("gG0", (1, 1), dG[1, 1], 2e-4),
              ("gG0", (1, 0), dG[1, 0], 2e-4)]
    rows, scale = [], {}
    for which, idx, gval, h in checks:
        fd = _loss_fd(cfg, a, b, which, idx, h)
        rows.append((which, idx, gval, fd))
        scale[which] = max(scale.get(which, 0.0), abs(fd))
    for which, idx, gval, fd in rows:
        err = abs(gval - fd) / max(scale[which], 1e-30)
        print(f"D2Q5 {prec} bc={bc} {which}{idx}: adjoint {gval:.9e} fd {fd:.9e} rel {err:.2e}",
              flush=True)
        assert err <= tol, (which, idx, gval, fd)
    assert dG[0, 2] == 0.0 and dG[1, 2] == 0.0
