"""Reaction sub-steps dt' = dt/m (Sec. 2.3) on the HIP path, through the C
ABI: forward parity with the oracle, which applies the m sub-step factors
one by one (the library sums their angles), and the adjoint per waveform
sample against central differences of the oracle.  Tolerances as in the
other parity and adjoint tests."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from .test_gpu_adjoint import _fd, _loss_weights
from .test_gpu_parity import _check, _gpu

pytestmark = pytest.mark.gpu
INF = math.inf


def _cfg(bc, m, K=150, gG=None, seed=81):
    g = w.cylinders_z((14, 12, 6), 0.25, seed=seed, vf_target=0.5, periodic=bc[0] == 0)
    dt = 0.004
    f = w.ogse_cosine_waveform(0.16, 2, 0.34, dt / m)[:K * m]
    if gG is None:
        gG = np.array([[9.0, 5.0, 3.0], [0.0, 0.0, 8.0]])
    return dict(name=f"substeps{m}", geoms=[g], bc=bc, dx=0.25, dt=dt,
                D=np.array([2.0, 1.0]), T2=np.array([40.0, 25.0]),
                kappa=np.array([[INF, 0.05], [0.05, INF]]), f=f, gG0=gG,
                q_geom=np.zeros(len(gG), np.int32), substeps=m)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1], [1, 0, 0]])
def test_substeps_forward_parity(prec, bc):
    btl = _gpu()
    cfg = _cfg(bc, 4)
    print(f"GPU substeps bc={bc} prec={prec}", flush=True)
    Eg, Mg = btl.simulate_config(cfg, prec=prec, want_M=True)
    Eo, Mo = oracle.simulate_config(cfg, threads=8, want_M=True)
    assert Eg.shape == (2, len(cfg["f"]) // 4 + 1)
    _check(Eg.cpu().numpy(), Eo, prec, f"substeps bc={bc}")
    for q in range(len(Mo)):
        _check(Mg[q].cpu().numpy(), Mo[q], prec, f"M_final q={q}")


def test_substeps_change_the_result():
    # a waveform varying within steps: m = 4 differs from the step-sampled
    # m = 1 run, and both match the oracle
    btl = _gpu()
    c4 = _cfg([0, 0, 0], 4)
    c1 = dict(c4, f=c4["f"][::4], substeps=1)
    E4 = btl.simulate_config(c4, prec="f64").cpu().numpy()
    E1 = btl.simulate_config(c1, prec="f64").cpu().numpy()
    assert np.max(np.abs(E4 - E1)) > 1e-6
    _check(E1, oracle.simulate_config(c1, threads=8)[0], "f64", "m=1")


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-3)])
def test_substeps_adjoint_vs_oracle_fd(prec, tol):
    import torch
    btl = _gpu()
    cfg = _cfg([0, 0, 0], 3, K=90)
    m = 3
    Q, K = len(cfg["gG0"]), len(cfg["f"]) // m
    a, b = _loss_weights(Q, K)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, substeps=m)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        cfg["q_geom"], ckpt_every=20)
        g = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        dD, dT2, dk, df = [t.cpu().numpy() for t in sim.backward(g, 2, K)]
    finally:
        sim.close()
    assert df.shape == (K * m,)
    checks = [("D", 0, dD[0]), ("T2", 1, dT2[1])]
    checks += [("f", i, df[i]) for i in (0, 1, 2, 40, 41, 130)]
    scale = {}
    rows = []
    for which, idx, gval in checks:
        fd = _fd(cfg, a, b, which, idx)
        rows.append((which, idx, gval, fd))
        scale[which] = max(scale.get(which, 0.0), abs(fd))
    for which, idx, gval, fd in rows:
        err = abs(gval - fd) / max(scale[which], 1e-30)
        print(f"{prec} {which}[{idx}]: adjoint {gval:.9e} fd {fd:.9e} rel {err:.2e}", flush=True)
        assert err <= tol, (which, idx, gval, fd)


def test_substeps_gG0_gradient_vs_oracle_fd():
    # the gamma G0 gradient with m = 3 sub-steps: the reaction angle of a
    # step is the sum of its sub-step angles, the face phases use F advanced
    # by the same sums
    import torch
    btl = _gpu()
    m = 3
    cfg = _cfg([1, 1, 0], m, K=60, gG=np.array([[7.0, 4.0, 2.0], [0.0, 6.0, -3.0]]))
    Q, K = len(cfg["gG0"]), len(cfg["f"]) // m
    a, b = _loss_weights(Q, K)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", substeps=m, grad_gG0=True)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        cfg["q_geom"], ckpt_every=20)
        g = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        dG = sim.backward(g, 2, K, grad_gG0=True)[4].cpu().numpy()
    finally:
        sim.close()
    h = 2e-4
    fd = np.zeros((Q, 3))
    for q in range(Q):
        for ax in range(3):
            vals = []
            for sgn in (1, -1):
                G = np.array(cfg["gG0"], float).copy()
                G[q, ax] += sgn * h
                E_o, _ = oracle.simulate_config(dict(cfg, gG0=G), threads=8)
                vals.append(float(np.sum(a * E_o.real + b * E_o.imag)))
            fd[q, ax] = (vals[0] - vals[1]) / (2 * h)
    scale = np.max(np.abs(fd))
    print("dgG0", dG, "fd", fd, flush=True)
    assert np.max(np.abs(dG - fd)) <= 1e-6 * scale


def test_substeps_errors():
    btl = _gpu()
    cfg = _cfg([0, 0, 0], 2, K=20)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", scheme=btl.BTL_CLASSICAL, substeps=2)
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"])
        assert ei.value.status == btl.BTL_E_UNSUPPORTED
        with pytest.raises(btl.BtlError) as ei:
            btl.btl_set_substeps(sim._h, 0)
        assert ei.value.status == btl.BTL_E_INVAL
        with pytest.raises(ValueError):
            sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:-1], cfg["gG0"])
    finally:
        sim.close()
