"""The seeded input generators: determinism and the sequence formulas."""
import math

import numpy as np

import workloads as w


def test_pgse_waveform_shape_and_b():
    dt = 0.01
    f = w.pgse_waveform(5.0, 20.0, dt)
    assert len(f) == 2500 and f[0] == 1.0 and f[499] == 1.0 and f[500] == 0.0
    assert f[1999] == 0.0 and f[2000] == -1.0 and f[-1] == -1.0
    assert abs(f.sum()) < 1e-12                    # refocused at the echo
    gG = w.gamma_g_for_b_pgse(1.0, 5.0, 20.0)
    # Sec. 2.1: b = (gamma G0)^2 delta^2 (Delta - delta/3); the sampled
    # waveform gives the same b up to the O(dt) sampling of the ramps
    assert abs(gG * gG * 25.0 * (20.0 - 5.0 / 3.0) - 1.0) < 1e-12
    assert abs(w.b_of_waveform(f, dt, gG) - 1.0) < 1e-9


def test_ogse_refocuses_and_has_requested_b():
    dt = 0.002
    f = w.ogse_cosine_waveform(20.0, 1, 25.0, dt)
    assert len(f) == int(round(45.0 / dt))
    assert abs(np.sum(f) * dt) < 1e-9
    gG = math.sqrt(1.0 / w.b_of_waveform(f, dt))
    assert abs(w.b_of_waveform(f, dt, gG) - 1.0) < 1e-12


def test_directions_are_unit_vectors():
    d = w.golden_spiral(64)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0)
    assert np.all(d[:, 2] >= 0)
    a = w.axon_directions()
    assert np.allclose(np.linalg.norm(a, axis=1), 1.0) and len(a) == 6


def test_geometries_are_deterministic_and_valid():
    for fn in (lambda: w.cylinders_z((24, 20, 4), 0.25, seed=9),
               lambda: w.cylinders_spheres((24, 24, 24), 0.25, seed=9, r_sph=(0.8, 1.2)),
               lambda: w.ellipsoid_cells((24, 24, 24), 0.2, seed=9, semi=(0.6, 1.2))):
        a, b = fn(), fn()
        assert np.array_equal(a.comp, b.comp)
        assert a.comp.max() < len(a.comp_phase)
        assert a.comp_phase.max() < a.n_phase


def test_cylinders_do_not_touch():
    # every lattice link between two cylinders would be an intra-intra
    # membrane; the packing keeps a gap of at least dx
    g = w.cylinders_z((40, 40, 2), 0.25, seed=5, vf_target=0.6)
    c = g.comp[0]
    for ax in (0, 1):
        nb = np.roll(c, 1, axis=ax)
        both = (c > 0) & (nb > 0)
        assert not np.any(both & (c != nb))


def test_configs_have_consistent_shapes():
    for name in ("cfg1", "cfg2", "cfg4"):
        cfg = w.make_config(name, n=12, K=20, n_q=3)
        P = len(cfg["D"])
        assert cfg["kappa"].shape == (P, P) and np.allclose(cfg["kappa"], cfg["kappa"].T)
        assert cfg["gG0"].shape[1] == 3 and len(cfg["q_geom"]) == len(cfg["gG0"])
        assert len(cfg["f"]) == 20
