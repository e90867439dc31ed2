"""Parity of the classical LBM (Appendix A, Eq. A12) on the HIP path with the
FP64 oracle's classical scheme, through the C ABI.

Same tolerances as the hybrid parity tests: FP64 storage to rounding order
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
CLASSICAL = 1


def _both(cfg, prec, want_M=False):
    btl = _gpu()
    cfg = dict(cfg, scheme=CLASSICAL)
    print(f"GPU classical {cfg['name']} prec={prec} K={len(cfg['f'])} Q={len(cfg['gG0'])}",
          flush=True)
    out = btl.simulate_config(cfg, prec=prec, want_M=want_M)
    Eo, Mo = oracle.simulate_config(cfg, threads=8, want_M=want_M)
    if want_M:
        Eg, Mg = out
        return Eg.cpu().numpy(), [m.cpu().numpy() for m in Mg], Eo, Mo
    return out.cpu().numpy(), None, Eo, None


def _cyl_cfg(bc, gG, K_scale=1.0, seed=51):
    g = w.cylinders_z((14, 12, 8), 0.25, seed=seed, vf_target=0.5,
                      periodic=all(b == 0 for b in bc))
    f = w.pgse_waveform(0.3 * K_scale, 0.9 * K_scale, 0.004)
    return dict(name=f"classical-cyl-bc{bc}", geoms=[g], bc=list(bc), dx=0.25, dt=0.004,
                D=np.array([2.0, 1.0]), T2=np.array([80.0, 60.0]),
                kappa=np.array([[INF, 0.03], [0.03, INF]]), f=f,
                gG0=np.asarray(gG, np.float64), q_geom=np.zeros(len(gG), np.int32))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_classical_periodic_oblique(prec):
    cfg = _cyl_cfg([0, 0, 0], [[5.0, 0, 0], [3.0, -2.0, 4.0], [0, 0, 0]])
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "classical periodic")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"classical M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_classical_mirror_oblique(prec):
    # every axis mirrored: the classical path keeps all 2^k image fields
    cfg = _cyl_cfg([1, 1, 1], [[0, 0, 6.0], [4.0, 3.0, 0], [2.0, -3.0, 4.0]])
    Eg, Mg, Eo, Mo = _both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "classical mirror")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"classical M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_classical_mixed_bc_and_ragged(prec):
    cfg = _cyl_cfg([1, 0, 0], [[4.0, 3.0, 0.0], [0.0, 4.0, 1.0]])
    Eg, _, Eo, _ = _both(cfg, prec)
    _check(Eg, Eo, prec, "classical mixed bc")
    cfg = w.make_config("cfg4", n=(13, 11, 7), K=300, n_q=3)
    Eg, _, Eo, _ = _both(cfg, prec)
    _check(Eg, Eo, prec, "classical cfg4 13x11x7")


def test_classical_T2_closed_form():
    # uniform medium, no gradient: E_k = (1 - dt/T2)^k (the forward Euler
    # of the decay), not exp(-k dt/T2) as in the hybrid scheme
    btl = _gpu()
    g = w.uniform((8, 6, 5), 0.5)
    K, dt, T2 = 300, 0.01, 0.7
    sim = btl.Simulator([g], [0, 0, 0], "f64", scheme=btl.BTL_CLASSICAL)
    try:
        E = sim.forward(dt, np.array([1.5]), np.array([T2]), np.array([[INF]]),
                        np.full(K, 0.3), np.zeros((1, 3)))[0].cpu().numpy()
    finally:
        sim.close()
    exact = (1.0 - dt / T2) ** np.arange(K + 1)
    assert np.max(np.abs(E - exact) / exact) < 1e-13


def test_classical_K0_K1_and_graph_replay():
    btl = _gpu()
    cfg = _cyl_cfg([0, 0, 0], [[3.0, -2.0, 4.0]])
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", scheme=btl.BTL_CLASSICAL)
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"])
        # K = 0: E_0 = 1 and M = 1 everywhere
        E0, M0 = sim.forward(*args, np.zeros(0), cfg["gG0"], want_M=True)
        assert np.allclose(E0.cpu().numpy(), 1.0, rtol=0, atol=0)
        assert np.allclose(M0[0].cpu().numpy(), 1.0, rtol=0, atol=0)
        # K = 1 against the oracle
        E1 = sim.forward(*args, cfg["f"][:1], cfg["gG0"]).cpu().numpy()
        Eo, _ = oracle.simulate_config(dict(cfg, f=cfg["f"][:1], scheme=CLASSICAL))
        _check(E1, Eo, "f64", "classical K=1")
        # graph replays (K >= 16) against eager launches
        f = cfg["f"][:200]
        reps = [sim.forward(*args, f, cfg["gG0"]).cpu().numpy() for _ in range(3)]
        btl.btl_set_graphs(sim._h, 0)
        try:
            eager = sim.forward(*args, f, cfg["gG0"]).cpu().numpy()
        finally:
            btl.btl_set_graphs(sim._h, 1)
        for r in reps:
            assert np.array_equal(r, eager)
        # the classical initial state depends on the gradient: another
        # gradient of the same shape must not replay the cached graph's init
        gG2 = np.asarray(cfg["gG0"]) * 1.7
        Eg2 = sim.forward(*args, f, gG2).cpu().numpy()
        btl.btl_set_graphs(sim._h, 0)
        try:
            eager2 = sim.forward(*args, f, gG2).cpu().numpy()
        finally:
            btl.btl_set_graphs(sim._h, 1)
        assert np.array_equal(Eg2, eager2)
        assert not np.array_equal(Eg2, eager)
        # switching back to the hybrid scheme reproduces a fresh hybrid run
        btl.btl_set_scheme(sim._h, btl.BTL_HYBRID)
        Eh = sim.forward(*args, f, cfg["gG0"]).cpu().numpy()
    finally:
        sim.close()
    Eo_h, _ = oracle.simulate_config(dict(cfg, f=f))
    _check(Eh, Eo_h, "f64", "hybrid after classical")


def test_classical_adjoint_unsupported_and_bad_scheme():
    btl = _gpu()
    cfg = _cyl_cfg([0, 0, 0], [[3.0, 0, 0]])
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", scheme=btl.BTL_CLASSICAL)
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"][:40],
                        cfg["gG0"], ckpt_every=10)
        assert ei.value.status == btl.BTL_E_UNSUPPORTED
        with pytest.raises(btl.BtlError) as ei:
            btl.btl_set_scheme(sim._h, 7)
        assert ei.value.status == btl.BTL_E_INVAL
    finally:
        sim.close()
