"""The first step of an untaped forward starts from the equilibrium constants
instead of a written initial state; a taped forward writes that state (its
first checkpoint) and loads it.  Both must give the same signal and final
magnetization bit for bit: the constants are the stored values.  Cases:
mirrored faces with oblique image fields, half-link membranes, the D2Q5
lattice, both storage precisions, every tile shape.  (Forwards with
membrane positions keep no tape; their first step is checked against the
oracle by the membrane parity tests.)
"""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    btl.load_library()
    return btl, torch


def _both(cfg, prec, launch=None):
    btl, torch = _gpu()
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, lattice=cfg.get("lattice", 0))
    try:
        if launch is not None:
            btl.btl_set_launch(sim._h, *launch)
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"], cfg["q_geom"])
        E0, M0 = sim.forward(*args, want_M=True)
        E1, M1 = sim.forward(*args, want_M=True, ckpt_every=4)
        torch.cuda.synchronize()
        # M_final comes back as one tensor per q-sample
        M0 = np.concatenate([m.cpu().numpy() for m in M0])
        M1 = np.concatenate([m.cpu().numpy() for m in M1])
        return E0.cpu().numpy(), M0, E1.cpu().numpy(), M1
    finally:
        sim.close()


CASES = {
    "mirror-oblique": lambda: w.make_config("cfg2", n=20, K=12),
    "cylinders": lambda: w.make_config("cfg4", n=(16, 14, 5), K=12, n_q=2),
    "d2q5": lambda: w.make_config("cfg2d", n=40, K=12, n_q=3),
}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_first_step_from_constants_equals_written_state(case, prec):
    cfg = CASES[case]()
    print(f"GPU first step {case} prec={prec}", flush=True)
    E0, M0, E1, M1 = _both(cfg, prec)
    assert np.array_equal(E0, E1)
    assert np.array_equal(M0, M1)
    assert np.all(E0[:, 0] == 1.0)


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 5])
def test_first_step_every_tile_shape(shape):
    cfg = w.make_config("cfg4", n=(16, 14, 5), K=6, n_q=2)
    print(f"GPU first step, tile shape {shape}", flush=True)
    E0, M0, E1, M1 = _both(cfg, "f32", launch=(shape, 3, 1))
    assert np.array_equal(E0, E1)
    assert np.array_equal(M0, M1)
