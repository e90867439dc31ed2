"""btl_forward_noalloc: the forward for callers that cannot allocate (code
under stream capture, serving loops), with every internal device buffer in
the library's fixed device scratch.  Checked through the C ABI against
btl_forward on the same simulator (the same kernels and launch shape: the
results must be bitwise equal), on two calls in a row, the second smaller,
and against the oracle.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from .test_gpu_parity import _check

pytestmark = pytest.mark.gpu
INF = math.inf


def _gpu():
    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    btl.load_library()
    return btl, torch


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_forward_twice_second_smaller(prec):
    # mirrored faces with oblique gradients (two image fields per q-sample),
    # membranes; first call 6 q-samples x 150 steps, then 2 x 60
    btl, torch = _gpu()
    cfg = w.make_config("cfg2", n=20, K=150)
    args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"])
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec)
    try:
        for qs, K in ((list(range(6)), 150), ([1, 4], 60)):
            print(f"GPU noalloc {prec} q={qs} K={K}", flush=True)
            f, G = cfg["f"][:K], cfg["gG0"][qs]
            E_na, M_na = sim.forward(*args, f, G, want_M=True, noalloc=True)
            E_ref, M_ref = sim.forward(*args, f, G, want_M=True)
            assert np.array_equal(E_na.cpu().numpy(), E_ref.cpu().numpy())
            for a, b in zip(M_na, M_ref):
                assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        Eo, _ = oracle.simulate_config(dict(cfg, f=cfg["f"][:60], gG0=cfg["gG0"][[1, 4]],
                                            q_geom=cfg["q_geom"][[1, 4]]), threads=8)
        _check(E_na.cpu().numpy(), Eo, prec, "noalloc vs oracle")
    finally:
        sim.close()


def test_noalloc_leaves_tape_and_refuses_oversize():
    btl, torch = _gpu()
    cfg = w.make_config("cfg4", n=(14, 12, 10), K=80, n_q=3)
    args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"])
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f32")
    try:
        g = torch.ones((3, 81, 2), dtype=torch.float64, device="cuda")
        sim.forward(*args, ckpt_every=20)
        ref = [t.cpu().numpy() for t in sim.backward(g)]
        sim.forward(*args, ckpt_every=20)
        sim.forward(*args, noalloc=True)           # no tape of its own, keeps the last one
        got = [t.cpu().numpy() for t in sim.backward(g)]
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
    finally:
        sim.close()
    # a problem beyond the scratch is refused before any device work
    big = w.uniform((128, 128, 128), 0.5)
    sim = btl.Simulator([big], [0, 0, 0], "f32")
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(0.01, np.array([1.0]), np.array([50.0]), np.array([[INF]]),
                        np.ones(4), np.array([[0.01, 0, 0]]), noalloc=True)
        assert ei.value.status == btl.BTL_E_INVAL
        assert "scratch" in str(ei.value)
        E = sim.forward(0.01, np.array([1.0]), np.array([50.0]), np.array([[INF]]),
                        np.ones(4), np.array([[0.0, 0, 0]]))
        assert abs(E.cpu().numpy()[0, -1] - math.exp(-0.04 / 50.0)) < 1e-6
    finally:
        sim.close()
