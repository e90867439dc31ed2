"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden), closed forms, exact invariants, a plane-wave
recurrence and a dense brute-force step matrix written independently in
tests/pins.py, and limiting cases of the membrane condition.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as w
from tests import pins

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF = math.inf


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_tau_matches_fig11_caption():
    g = _load("fig11_tau.json")
    assert oracle.tau(g["D"], g["dt"], g["dx"]) == pytest.approx(g["tau"], abs=1e-15)


def _run(comp, cp, nph, bc, dx, dt, D, T2, kap, f, gG0, **kw):
    return oracle.simulate(comp, cp, nph, bc, dx, dt, np.asarray(D, float),
                           np.asarray(T2, float), np.asarray(kap, float), f, gG0, **kw)


def test_plane_wave_periodic_oblique():
    # homogeneous periodic box, non-cubic, oblique gradient, PGSE waveform
    g = w.uniform((5, 4, 3), 0.5)
    f = w.pgse_waveform(0.05, 0.2, 0.01)
    gG0 = np.array([0.9, -0.5, 0.7])
    E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], 0.5, 0.01, [2.5], [30.0],
                [[INF]], f, gG0)
    ref = pins.plane_wave_E((5, 4, 3), 0.5, 0.01, 2.5, 30.0, f, gG0)
    assert np.max(np.abs(E - ref)) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_plane_wave_mirror_axis_aligned(axis):
    # mirroring on every face with an axis-aligned gradient keeps the plane
    # wave exact: normal faces use the conjugate rule, parallel faces the
    # plain direction mirror
    g = w.uniform((6, 5, 4), 0.5)
    f = w.pgse_waveform(0.04, 0.12, 0.01)
    gG0 = np.zeros(3)
    gG0[axis] = 1.3
    E, _ = _run(g.comp, g.comp_phase, 1, [1, 1, 1], 0.5, 0.01, [1.7], [INF],
                [[INF]], f, gG0, mirror="paper")
    ref = pins.plane_wave_E((6, 5, 4), 0.5, 0.01, 1.7, INF, f, gG0)
    assert np.max(np.abs(E - ref)) < 1e-13


def test_uniform_ic_closed_form_cfg1():
    # exact solution exp(-bD) exp(-TE/T2); the hybrid scheme is second order
    # in dx, with leading relative error below 1e-3 at dx = 0.5 um
    gold = _load("uniform_ic_exact.json")
    cfg = w.make_config("cfg1", n=4)
    E, _ = oracle.simulate_config(cfg)
    e = E[0, -1]
    assert abs(e.imag) < 1e-14
    assert abs(e.real - gold["E_TE"]) / gold["E_TE"] < 1.5e-3
    # apparent diffusivity recovered from the signal is the D put in
    D_app = -math.log(e.real / math.exp(-gold["TE"] / gold["T2"])) / gold["b"]
    assert D_app == pytest.approx(gold["D"], rel=5e-4)


def test_second_order_in_dx_at_fixed_tau():
    # halve dx with dt ~ dx^2 (tau fixed): the error falls by ~4
    D, T2 = 2.5, 80.0
    delta, Delta = 5.0, 20.0
    exact = math.exp(-1.0 * D) * math.exp(-(delta + Delta) / T2)
    errs = []
    for dx in (0.5, 0.25, 0.125):
        dt = 0.01 * (dx / 0.5) ** 2
        f = w.pgse_waveform(delta, Delta, dt)
        gG = w.gamma_g_for_b_pgse(1.0, delta, Delta)
        g = w.uniform((2, 2, 2), dx)
        E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [D], [T2], [[INF]],
                    f, [gG, 0, 0], want_M=False)
        errs.append(abs(E[-1].real - exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.2 for r in rates), rates


@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1], [1, 0, 1]])
def test_pure_T2_decay_any_geometry(bc):
    # G = 0, one T2 everywhere: E_k = exp(-k dt / T2) for any D, kappa, BC
    g = w.cylinders_z((12, 10, 3), 0.25, seed=11, vf_target=0.5)
    f = np.zeros(60)
    E, _ = _run(g.comp, g.comp_phase, 2, bc, 0.25, 0.004, [2.0, 1.0], [40.0, 40.0],
                [[INF, 0.02], [0.02, INF]], f, [0, 0, 0])
    k = np.arange(61)
    assert np.max(np.abs(E - np.exp(-k * 0.004 / 40.0))) < 1e-14


def test_T2_mixture_impermeable():
    # G = 0, kappa = 0: compartments decay independently with their own T2
    g = w.cylinders_z((12, 10, 2), 0.25, seed=12, vf_target=0.5)
    v = g.phase_fractions()
    f = np.zeros(50)
    dt = 0.004
    E, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, dt, [2.0, 1.0], [40.0, 15.0],
                [[INF, 0.0], [0.0, INF]], f, [0, 0, 0])
    k = np.arange(51)
    ref = v[0] * np.exp(-k * dt / 40.0) + v[1] * np.exp(-k * dt / 15.0)
    assert np.max(np.abs(E - ref)) < 1e-14


@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1]])
def test_conservation_after_echo(bc):
    # T2 = inf: once the PGSE pair has refocused (F = 0) and the gradient is
    # off, total magnetization is conserved by collision, streaming,
    # membranes and both outer boundary conditions
    g = w.cylinders_z((10, 9, 4), 0.25, seed=13, vf_target=0.5)
    f = np.concatenate([w.pgse_waveform(0.04, 0.1, 0.004), np.zeros(40)])
    gG0 = [0.0, 3.0, 0.0] if bc[0] == 1 else [2.0, 3.0, -1.0]
    E, _ = _run(g.comp, g.comp_phase, 2, bc, 0.25, 0.004, [2.0, 1.0], [INF, INF],
                [[INF, 0.05], [0.05, INF]], f, gG0)
    K0 = len(f) - 40
    tail = E[K0:]
    assert abs(E[K0] - 1.0) > 1e-6          # the gradient did something
    assert np.max(np.abs(tail - tail[0])) < 1e-14


def _tiny_geom():
    comp = np.zeros((2, 3, 4), np.uint32)
    comp[:, 1:, 1:3] = 1
    comp[1, 0, 3] = 2
    return comp, np.array([0, 1, 1], np.uint8)


@pytest.mark.parametrize("case", ["periodic_oblique", "mirror_x", "mirror_mixed"])
def test_dense_bruteforce(case):
    comp, cp = _tiny_geom()
    kap = np.array([[INF, 0.03], [0.03, 0.01]])
    D, T2 = [2.0, 0.7], [30.0, 12.0]
    dx, dt = 0.5, 0.01
    f = np.array([1.0, 1.0, 0.3, 0.0, -0.5, -1.0, -1.0, 0.2])
    if case == "periodic_oblique":
        bc, gG0 = [0, 0, 0], np.array([1.1, -0.6, 0.8])
    elif case == "mirror_x":
        bc, gG0 = [1, 1, 1], np.array([1.4, 0.0, 0.0])
    else:
        bc, gG0 = [1, 0, 1], np.array([0.0, 0.9, 0.0])
    mats = pins.dense_step_matrices(comp, cp, bc, dx, dt, D, T2, kap, f, gG0)
    ref = pins.dense_run(mats, comp.size)
    E, _ = _run(comp, cp, 2, bc, dx, dt, D, T2, kap, f, gG0, mirror="paper")
    assert np.max(np.abs(E - ref)) < 1e-14


def test_dense_matrix_conserves_mass_and_is_stable():
    comp, cp = _tiny_geom()
    kap = np.array([[INF, 0.03], [0.03, 0.0]])
    mats = pins.dense_step_matrices(comp, cp, [0, 1, 0], 0.5, 0.01, [2.0, 0.7],
                                    [INF, INF], kap, np.zeros(1), np.zeros(3))
    A = mats[0]
    S7 = 7 * comp.size
    colsum = A[:S7, :].sum(axis=0)
    assert np.allclose(colsum[:S7], 1.0, atol=1e-14)
    assert np.allclose(colsum[S7:], 0.0, atol=1e-14)
    assert np.max(np.abs(np.linalg.eigvals(A))) <= 1.0 + 1e-12


def test_impermeable_plates_diffraction():
    # two impermeable plates of width a = 20 dx (membranes on the middle link
    # and on the periodic wrap), one-step pulses, long separation: the signal
    # tends to |(1/n) sum_j exp(-i q x_j)|^2, the lattice form of the
    # narrow-pulse plate result 2(1 - cos qa)/(qa)^2
    n, dx, dt = 20, 0.25, 0.002
    D = 2.3
    g = w.slabs((2 * n, 1, 1), dx, [n])
    Delta_steps = 50000
    f = np.zeros(Delta_steps + 1)
    f[0], f[-1] = 1.0, -1.0
    a = n * dx
    for qa in (0.5 * math.pi, math.pi, 2 * math.pi, 3 * math.pi):
        q = qa / a
        gG = q / dt
        E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [D], [INF],
                    [[0.0]], f, [gG, 0, 0], want_M=False)
        lat = abs(np.mean(np.exp(-1j * q * dx * np.arange(n)))) ** 2
        cont = 2.0 * (1.0 - math.cos(qa)) / qa ** 2
        assert abs(E[-1] - lat) < 1e-12
        # lattice vs continuum differ by the factor (th/2)^2 / sin^2(th/2),
        # th = q dx, i.e. by about th^2/12 relative
        th = q * dx
        assert abs(E[-1].real - cont) <= th * th / 8.0 * cont + 1e-14


def test_plates_3d_equals_1d():
    g1 = w.slabs((16, 1, 1), 0.25, [7])
    g3 = w.slabs((16, 5, 3), 0.25, [7])
    f = w.pgse_waveform(0.02, 0.1, 0.004)
    args = ([0, 0, 0], 0.25, 0.004, [2.3], [50.0], [[0.05]], f, [4.0, 0, 0])
    E1, _ = _run(g1.comp, g1.comp_phase, 1, *args)
    E3, _ = _run(g3.comp, g3.comp_phase, 1, *args)
    assert np.max(np.abs(E1 - E3)) < 1e-14


def _axon_small(seed=21, shape=(10, 9, 4)):
    g = w.cylinders_z(shape, 0.25, seed=seed, vf_target=0.5)
    return g, [2.0, 1.0], [90.0, 70.0], np.array([[INF, 0.02], [0.02, INF]])


def test_gradient_reversal_conjugates_signal():
    g, D, T2, kap = _axon_small()
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = np.array([3.0, -2.0, 1.0])
    E1, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, D, T2, kap, f, G)
    E2, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, D, T2, kap, f, -G)
    assert np.max(np.abs(E2 - np.conj(E1))) < 1e-14


def test_axis_swap_invariance():
    # exchanging the x and y axes of geometry and gradient leaves E unchanged
    g, D, T2, kap = _axon_small(shape=(9, 9, 3))
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = np.array([3.0, -2.0, 1.0])
    E1, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, D, T2, kap, f, G)
    comp_sw = np.ascontiguousarray(np.swapaxes(g.comp, 1, 2))
    E2, _ = _run(comp_sw, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, D, T2, kap, f,
                 G[[1, 0, 2]])
    assert np.max(np.abs(E2 - E1)) < 1e-13


def test_periodic_translation_at_echo():
    # rolling the periodic medium by s rolls the solution by s up to the
    # quasi-periodic wrap phases; at the echo (F = 0) these vanish, so the
    # final magnetization is the rolled one and E(TE) is unchanged
    g, D, T2, kap = _axon_small()
    dt, dx = 0.004, 0.25
    f = w.pgse_waveform(0.04, 0.12, dt)
    G = np.array([3.0, -2.0, 1.5])
    s = (1, 2, 3)                                  # (z, y, x) shifts
    E1, M1 = _run(g.comp, g.comp_phase, 2, [0, 0, 0], dx, dt, D, T2, kap, f, G)
    rolled = np.roll(g.comp, shift=s, axis=(0, 1, 2))
    E2, M2 = _run(rolled, g.comp_phase, 2, [0, 0, 0], dx, dt, D, T2, kap, f, G)
    assert abs(E2[-1] - E1[-1]) < 1e-14
    assert np.max(np.abs(M2 - np.roll(M1, shift=s, axis=(0, 1, 2)))) < 1e-13


def test_kappa_inf_equals_no_membrane():
    g, _, _, _ = _axon_small()
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = [2.0, 1.0, 0.5]
    kap = np.full((2, 2), INF)
    E1, M1 = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [1.5, 1.5],
                  [50.0, 50.0], kap, f, G)
    u = np.zeros_like(g.comp)
    E2, M2 = _run(u, np.zeros(1, np.uint8), 1, [0, 0, 0], 0.25, 0.004, [1.5], [50.0],
                  [[INF]], f, G)
    assert np.array_equal(E1, E2) and np.array_equal(M1, M2)


def test_large_kappa_approaches_free_streaming():
    g, _, _, _ = _axon_small()
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = [2.0, 1.0, 0.5]
    E1, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [1.5, 1.5],
                 [50.0, 50.0], np.array([[INF, 1e9], [1e9, INF]]), f, G)
    u = np.zeros_like(g.comp)
    E2, _ = _run(u, np.zeros(1, np.uint8), 1, [0, 0, 0], 0.25, 0.004, [1.5], [50.0],
                 [[INF]], f, G)
    assert np.max(np.abs(E1 - E2)) < 1e-7


def test_impermeable_isolates_compartments():
    # kappa = 0: the extracellular field does not see intracellular D, T2
    g, D, T2, _ = _axon_small()
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = [2.0, 1.0, 0.5]
    kap = np.array([[INF, 0.0], [0.0, INF]])
    _, M1 = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [2.0, 1.0],
                 [90.0, 70.0], kap, f, G)
    _, M2 = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [2.0, 0.3],
                 [90.0, 20.0], kap, f, G)
    ex = g.phase_volume() == 0
    assert np.array_equal(M1[ex], M2[ex])
    assert not np.allclose(M1[~ex], M2[~ex])


@pytest.mark.parametrize("axis", [0, 1])
def test_mirror_rule_equals_reflected_doubling(axis):
    # the paper's mirror rule (axis-aligned gradient) coincides with the
    # medium reflected and doubled across every mirrored face
    g, D, T2, kap = _axon_small(shape=(8, 7, 3))
    f = w.pgse_waveform(0.04, 0.12, 0.004)
    G = np.zeros(3)
    G[axis] = 4.0
    E1, M1 = _run(g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, D, T2, kap, f, G,
                  mirror="paper")
    E2, M2 = _run(g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, D, T2, kap, f, G,
                  mirror="double")
    assert np.max(np.abs(E1 - E2)) < 1e-13
    assert np.max(np.abs(M1 - M2)) < 1e-13


def test_oblique_mirror_is_rejected_by_paper_rule():
    g, D, T2, kap = _axon_small(shape=(6, 6, 2))
    with pytest.raises(NotImplementedError):
        _run(g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, D, T2, kap,
             np.ones(3), [1.0, 1.0, 0.0], mirror="paper")


def test_z_invariance_oblique_gradient():
    # z-aligned permeable cylinders, periodic on all faces, oblique gradient:
    # |M| has no z dependence, and at the echo M itself has none (Sec. 3.2)
    g = w.cylinders_z((11, 11, 5), 1.0, seed=31, vf_target=0.5, mean_r=2.5)
    dt = 0.025
    f = w.pgse_waveform(0.2, 0.6, dt)
    G = np.ones(3) / math.sqrt(3.0) * 0.8
    E, M = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 1.0, dt, [2.0, 1.5], [10.0, 30.0],
                np.array([[INF, 0.01], [0.01, INF]]), f, G)
    assert np.max(np.abs(M - M[0:1])) < 1e-14
    _, Mh = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 1.0, dt, [2.0, 1.5], [10.0, 30.0],
                 np.array([[INF, 0.01], [0.01, INF]]), f[:12], G)
    assert np.max(np.abs(np.abs(Mh) - np.abs(Mh[0:1]))) < 1e-14


# ---- classical LBM (Appendix A, Eq. A12): reaction inside the collision ----

@pytest.mark.parametrize("bc", [[0, 0, 0], [0, 1, 0]])
def test_classical_dense_bruteforce(bc):
    comp, cp = _tiny_geom()
    kap = np.array([[INF, 0.03], [0.03, 0.01]])
    D, T2 = [2.0, 0.7], [30.0, 12.0]
    f = np.array([1.0, 1.0, 0.3, 0.0, -0.5, -1.0, -1.0, 0.2])
    gG0 = np.array([1.1, 0.0 if bc[1] else -0.6, 0.8])
    mats = pins.dense_step_matrices(comp, cp, bc, 0.5, 0.01, D, T2, kap, f, gG0, scheme=1)
    ref = pins.dense_run(mats, comp.size)
    E, _ = _run(comp, cp, 2, bc, 0.5, 0.01, D, T2, kap, f, gG0, mirror="double", scheme=1)
    assert np.max(np.abs(E - ref)) < 1e-14


def test_classical_T2_decay_closed_form():
    # G = 0: the classical collision multiplies M by (1 - dt/T2) per step
    g = w.cylinders_z((10, 9, 3), 0.25, seed=14, vf_target=0.5)
    E, _ = _run(g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [2.0, 1.0], [40.0, 40.0],
                [[INF, 0.02], [0.02, INF]], np.zeros(50), [0, 0, 0], scheme=1)
    k = np.arange(51)
    assert np.max(np.abs(E - (1.0 - 0.004 / 40.0) ** k)) < 1e-14


def test_hybrid_error_independent_of_domain_size_classical_not():
    # Sec. 3.1 (uniform initial condition): the hybrid scheme's error does
    # not depend on the REV size L, the classical scheme's grows with L
    D, T2, dx, dt = 2.5, 80.0, 0.5, 0.01
    f = w.pgse_waveform(5.0, 20.0, dt)
    gG = w.gamma_g_for_b_pgse(1.0, 5.0, 20.0)
    exact = math.exp(-D) * math.exp(-25.0 / T2)
    err = {}
    for L in (20, 100):
        g = w.uniform((int(L / dx), 1, 1), dx)
        for sch in (0, 1):
            E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [D], [T2], [[INF]], f,
                        [gG, 0, 0], want_M=False, scheme=sch)
            err[(L, sch)] = abs(E[-1] - exact) / exact
    assert abs(err[(20, 0)] - err[(100, 0)]) < 1e-12 and err[(20, 0)] < 1e-3
    assert err[(20, 1)] > 10 * err[(20, 0)]
    assert err[(100, 1)] > 10 * err[(20, 1)]


# ---- general membrane condition with sub-link positions (theta = 0) -------

EPSD = 0.25


@pytest.mark.parametrize("kappa", [0.0, 0.004, 0.05, 0.7, 20.0])
def test_memb_coeffs_reduce_to_half_link(kappa):
    # Eq. B5: at Delta_m = 1/2 only A_1 = P/(1+P) and B_1 = 1/(1+P) survive
    dx, dt = 0.3, 0.002
    c = oracle.memb_coeffs(0.5, kappa * dt, EPSD * dx)
    if kappa == 0.0:
        ref = [1.0, 0, 0, 0, 0, 0]
    else:
        P = EPSD * dx / (2 * kappa * dt)
        ref = [P / (1 + P), 0, 0, 1 / (1 + P), 0, 0]
    assert np.max(np.abs(c - ref)) < 1e-15


def test_memb_coeffs_impermeable_is_interpolated_bounce_back():
    # kappa = 0: zero normal flux, the Neumann condition of Eq. c_n alone
    for d in (0.05, 0.3, 0.5, 0.77, 0.99):
        c = oracle.memb_coeffs(d, 0.0, EPSD * 0.5)
        r = (2 * d - 1) / (2 * d + 1)
        assert np.max(np.abs(c - [1.0, -r, r, 0, 0, 0])) < 1e-15


def test_memb_coeffs_keep_uniform_states():
    # a uniform equilibrium (all populations w M) must stream unchanged
    # across any membrane: the six coefficients sum to one for every
    # Delta_m and kappa (Dirichlet consistency sum c_dj = 1 - 2 c_d4 and
    # sum c_nj = 1 carry through Eqs. B4a-B4c)
    rng = np.random.default_rng(5)
    for _ in range(200):
        d = rng.uniform(1e-4, 1 - 1e-4)
        kdt = 10 ** rng.uniform(-6, 1)
        c = oracle.memb_coeffs(d, kdt, EPSD * rng.uniform(0.05, 2.0))
        assert abs(c.sum() - 1.0) < 1e-13


def _cyl_with_delta(bc_periodic=True):
    g = w.cylinders_z((12, 11, 4), 0.25, seed=61, vf_target=0.5, periodic=bc_periodic)
    return g, w.link_delta(g)


def test_general_membrane_at_mid_link_equals_half_link():
    g, _ = _cyl_with_delta()
    ld = np.full((3,) + g.comp.shape, 0.5, np.float32)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    args = (g.comp, g.comp_phase, 2, [0, 0, 0], 0.25, 0.004, [2.0, 1.0], [90.0, 70.0],
            [[INF, 0.03], [0.03, INF]], f, [3.0, -2.0, 1.0])
    E0, M0 = _run(*args)
    E1, M1 = _run(*args, link_delta=ld)
    assert np.max(np.abs(E1 - E0)) < 1e-14
    assert np.max(np.abs(M1 - M0)) < 1e-14


@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1]])
def test_general_membrane_uniform_decay(bc):
    # G = 0 and one T2: the uniform state only decays, E_k = exp(-k dt/T2),
    # whatever the membrane positions
    g, ld = _cyl_with_delta(bc[0] == 0)
    f = np.zeros(80)
    E, _ = _run(g.comp, g.comp_phase, 2, bc, 0.25, 0.004, [2.0, 1.0], [40.0, 40.0],
                [[INF, 0.02], [0.02, INF]], f, [0, 0, 0], link_delta=ld)
    k = np.arange(81)
    assert np.max(np.abs(E - np.exp(-k * 0.004 / 40.0))) < 1e-13


def test_general_membrane_mirror_rule_equals_doubling():
    # axis-aligned gradient on mirrored faces: the paper's buffer rule and the
    # reflected, doubled medium (with the reflected membrane positions) agree
    g, ld = _cyl_with_delta(False)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    args = (g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, [2.0, 1.0], [90.0, 70.0],
            [[INF, 0.03], [0.03, INF]], f, [0.0, 4.0, 0.0])
    Ep, _ = _run(*args, mirror="paper", link_delta=ld)
    Ed, _ = _run(*args, mirror="double", link_delta=ld)
    assert np.max(np.abs(Ep - Ed)) < 1e-13


_SLAB_X, _SLAB_ALPHA = 2.0, 0.3
_SLAB_D, _SLAB_T2, _SLAB_G = [1.5, 1.0, 2.0], [60.0, 50.0, 80.0], 0.25
_slab_refs = {}


def _slab_case(m, general, kappa=0.05, lattice=0):
    # 1D: outer compartment C, permeable pair A | B on [X, 3X] walled off from
    # C by impermeable membranes; interfaces at X, 2X, 3X and spacing
    # dx = X/(m + alpha), so every refinement sees the same sub-link
    # positions frac(c alpha) = 0.3, 0.6, 0.9
    X = _SLAB_X
    dx = X / (m + _SLAB_ALPHA)
    n = int(math.floor(3 * (m + _SLAB_ALPHA))) + 5
    x = np.arange(n) * dx
    comp = np.where(x < X, 0, np.where(x < 2 * X, 1, np.where(x < 3 * X, 2, 0)))
    dt = 0.3 * (EPSD if lattice == 0 else 1.0 / 3.0) * dx * dx / _SLAB_D[1]
    K = int(math.ceil(8.0 / dt))
    f = pins.step_average_pgse(2.0, 6.0, dt, K)
    kap = [[INF, 0.0, 0.0], [0.0, INF, kappa], [0.0, kappa, INF]]
    ld = np.full((3, 1, 1, n), 0.5, np.float32)
    for c in (1, 2, 3):
        j = int(math.floor(c * X / dx))
        ld[0, 0, 0, j] = (c * X - j * dx) / dx
    _, M = _run(comp.reshape(1, 1, n), [0, 1, 2], 3, [0, 0, 0], dx, dt, _SLAB_D, _SLAB_T2,
                kap, f, [_SLAB_G, 0, 0], link_delta=ld if general else None, lattice=lattice)
    inside = (x > X) & (x < 3 * X)
    key = (m, kappa, lattice)
    if key not in _slab_refs:
        r = [pins.slab_fv_reference([X, 2 * X, 3 * X], _SLAB_D[1:], _SLAB_T2[1:], [kappa],
                                    _SLAB_G, f, dt, x[inside], cells) for cells in (40, 80)]
        _slab_refs[key] = (4 * r[1] - r[0]) / 3          # Richardson, O(h^4)
    ref = _slab_refs[key]
    return dx, np.linalg.norm(M.reshape(-1)[inside] - ref) / np.linalg.norm(ref)


def test_general_membrane_second_order_off_lattice():
    # Sec. 2.4.2 / App. B: with the membrane position on the link the
    # condition is second order in dx against an independent finite-volume
    # solution of the same Bloch-Torrey problem (permeable membrane between
    # media of different D and T2, impermeable walls); the half-link rule,
    # which moves every membrane to mid-link, is only first order there
    res = {g: [_slab_case(m, g) for m in (4, 9, 19)] for g in (True, False)}
    for g, r in res.items():
        o = [math.log(r[i][1] / r[i + 1][1]) / math.log(r[i][0] / r[i + 1][0])
             for i in range(2)]
        print("general" if g else "half-link", [f"{e:.3e}" for _, e in r], o)
        if g:
            assert all(1.8 < v < 2.2 for v in o), o
        else:
            assert all(0.8 < v < 1.3 for v in o), o
    assert res[False][-1][1] > 5 * res[True][-1][1]


# ---- reaction sub-steps dt' = dt/m (Sec. 2.3) ------------------------------

def test_substeps_plane_wave_varying_within_steps():
    # cosine waveform sampled 5 times per step: the plane wave advances its
    # wave vector sample by sample
    g = w.uniform((6, 5, 4), 0.5)
    m, dt = 5, 0.01
    f = w.ogse_cosine_waveform(0.4, 2, 0.9, dt / m)
    f = f[:len(f) // m * m]
    gG0 = np.array([0.8, -0.6, 0.5])
    E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], 0.5, dt, [2.2], [45.0], [[INF]], f,
                gG0, substeps=m)
    ref = pins.plane_wave_E((6, 5, 4), 0.5, dt, 2.2, 45.0, f, gG0, substeps=m)
    assert len(E) == len(f) // m + 1
    assert np.max(np.abs(E - ref)) < 1e-13


@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1], [1, 0, 1]])
def test_substeps_of_a_step_constant_waveform_change_nothing(bc):
    g = w.cylinders_z((12, 10, 4), 0.25, seed=71, vf_target=0.5, periodic=bc[0] == 0)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    args = (g.comp, g.comp_phase, 2, bc, 0.25, 0.004, [2.0, 1.0], [90.0, 70.0],
            [[INF, 0.03], [0.03, INF]])
    G = [0.0, 0.0, 4.0] if bc == [1, 1, 1] else [3.0, -2.0, 1.0]
    E1, M1 = _run(*args, f, G)
    E3, M3 = _run(*args, np.repeat(f, 3), G, substeps=3)
    assert np.max(np.abs(E3 - E1)) < 1e-13
    assert np.max(np.abs(M3 - M1)) < 1e-13


# ---- D2Q5 lattice on a single layer (Sec. 2.2) ------------------------------

D2Q5 = 1


def test_d2q5_plane_wave():
    g = w.uniform((7, 5, 1), 0.5)
    f = w.pgse_waveform(0.05, 0.2, 0.01)
    gG0 = np.array([0.9, -0.7, 0.0])
    E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], 0.5, 0.01, [2.5], [30.0], [[INF]], f,
                gG0, lattice=D2Q5)
    ref = pins.plane_wave_E((7, 5, 1), 0.5, 0.01, 2.5, 30.0, f, gG0, lattice=D2Q5)
    assert np.max(np.abs(E - ref)) < 1e-13
    # mirrored faces with an axis-aligned gradient keep the plane wave exact
    E, _ = _run(g.comp, g.comp_phase, 1, [1, 1, 1], 0.5, 0.01, [2.5], [30.0], [[INF]], f,
                [0.0, 1.2, 0.0], lattice=D2Q5, mirror="paper")
    ref = pins.plane_wave_E((7, 5, 1), 0.5, 0.01, 2.5, 30.0, f, [0.0, 1.2, 0.0],
                            lattice=D2Q5)
    assert np.max(np.abs(E - ref)) < 1e-13


@pytest.mark.parametrize("bc,scheme", [([0, 0, 0], 0), ([1, 1, 0], 0), ([1, 0, 0], 0),
                                       ([0, 0, 0], 1), ([1, 0, 0], 1)])
def test_d2q5_dense_bruteforce(bc, scheme):
    comp = np.zeros((1, 4, 5), np.uint32)
    comp[0, 1:3, 1:4] = 1
    comp[0, 3, 4] = 2
    cp = np.array([0, 1, 1], np.uint8)
    kap = np.array([[INF, 0.03], [0.03, 0.01]])
    D, T2 = [2.0, 0.7], [30.0, 12.0]
    dx, dt = 0.5, 0.01
    f = np.array([1.0, 1.0, 0.3, 0.0, -0.5, -1.0, -1.0, 0.2])
    # gradients normal to a mirrored face use the conjugate rule (hybrid);
    # the classical scheme takes gradients parallel to mirrored faces
    if bc == [1, 1, 0]:
        gG0 = np.array([0.0, 0.9, 0.0])
    elif bc == [1, 0, 0]:
        gG0 = np.array([1.1, 0.0, 0.0]) if scheme == 0 else np.array([0.0, 0.9, 0.0])
    else:
        gG0 = np.array([1.1, -0.6, 0.0])
    mats = pins.dense_step_matrices(comp, cp, bc, dx, dt, D, T2, kap, f, gG0, scheme=scheme,
                                    lattice=D2Q5)
    ref = pins.dense_run(mats, comp.size, lattice=D2Q5)
    E, _ = _run(comp, cp, 2, bc, dx, dt, D, T2, kap, f, gG0, mirror="paper" if scheme == 0
                else "double", scheme=scheme, lattice=D2Q5)
    assert np.max(np.abs(E - ref)) < 1e-14


def test_d2q5_uniform_ic_closed_form_and_diffusivity():
    # Sec. 3.1 uniform initial condition: exp(-bD) exp(-TE/T2) to second
    # order; the diffusivity recovered from the signal is the one put in only
    # with the D2Q5 lattice constant eps_D = 1/3 in tau
    gold = _load("uniform_ic_exact.json")
    D, T2, delta, Delta = gold["D"], gold["T2"], gold["delta"], gold["Delta"]
    gG = w.gamma_g_for_b_pgse(gold["b"], delta, Delta)
    errs = []
    for dx in (0.5, 0.25):
        dt = 0.01 * (dx / 0.5) ** 2
        f = w.pgse_waveform(delta, Delta, dt)
        g = w.uniform((4, 3, 1), dx)
        E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [D], [T2], [[INF]], f,
                    [gG, 0, 0], want_M=False, lattice=D2Q5)
        errs.append(abs(E[-1].real - gold["E_TE"]) / gold["E_TE"])
        D_app = -math.log(E[-1].real / math.exp(-gold["TE"] / T2)) / gold["b"]
        assert D_app == pytest.approx(D, rel=2e-3)
    assert errs[0] < 3e-3 and 3.5 < errs[0] / errs[1] < 4.5


def test_d2q5_impermeable_plates_diffraction():
    n, dx, dt = 20, 0.25, 0.002
    g = w.slabs((2 * n, 1, 1), dx, [n])
    f = np.zeros(40001)
    f[0], f[-1] = 1.0, -1.0
    a = n * dx
    for qa in (0.5 * math.pi, 2 * math.pi):
        q = qa / a
        E, _ = _run(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [2.3], [INF], [[0.0]], f,
                    [q / dt, 0, 0], want_M=False, lattice=D2Q5)
        lat = abs(np.mean(np.exp(-1j * q * dx * np.arange(n)))) ** 2
        assert abs(E[-1] - lat) < 1e-12


def test_d2q5_rejects_3d_input():
    g = w.uniform((4, 3, 2), 0.5)
    with pytest.raises(ValueError):
        _run(g.comp, g.comp_phase, 1, [0, 0, 0], 0.5, 0.01, [2.0], [INF], [[INF]],
             np.zeros(3), [1.0, 0, 0], lattice=D2Q5)
    g = w.uniform((4, 3, 1), 0.5)
    with pytest.raises(ValueError):
        _run(g.comp, g.comp_phase, 1, [0, 0, 0], 0.5, 0.01, [2.0], [INF], [[INF]],
             np.zeros(3), [1.0, 0, 0.5], lattice=D2Q5)


def test_d2q5_general_membrane_second_order_off_lattice():
    # the slab problem above on the D2Q5 lattice (eps_D = 1/3 in tau, P and
    # the membrane coefficients)
    r = [_slab_case(m, True, lattice=D2Q5) for m in (4, 9, 19)]
    o = [math.log(r[i][1] / r[i + 1][1]) / math.log(r[i][0] / r[i + 1][0]) for i in range(2)]
    print([f"{e:.3e}" for _, e in r], o)
    assert all(1.8 < v < 2.2 for v in o), o


def _tilted_case(n, bounds, kap_if, general, curved=False):
    # D2Q5 box crossed by straight membranes whose normal is (2, 1)/sqrt(5)
    # (26.6 degrees from x, 63.4 from y); impermeable walls isolate the
    # compartments between bounds[0] and bounds[-1]; gradient along the
    # normal: the exact solution depends on s = x.nhat only and is the 1D
    # finite-volume reference of the slab problem
    X = 10.0 * math.sqrt(5.0)
    dx = X / n
    g = w.angled_slabs_2d(n, dx, bounds)
    nc = len(bounds)
    Dv, T2v = [1.5, 1.0, 2.0][:nc], [60.0, 50.0, 80.0][:nc]
    dt = 0.3 * dx * dx / (3.0 * min(Dv[1:]))
    K = int(math.ceil(8.0 / dt))
    f = pins.step_average_pgse(2.0, 6.0, dt, K)
    kap = np.full((nc, nc), INF)
    for c in range(1, nc):
        kap[0, c] = kap[c, 0] = 0.0
    for c in range(1, nc - 1):
        kap[c, c + 1] = kap[c + 1, c] = kap_if[c - 1]
    nh = np.array([2.0, 1.0]) / math.sqrt(5.0)
    _, M = _run(g.comp, g.comp_phase, nc, [0, 0, 0], dx, dt, Dv, T2v, kap, f,
                [0.25 * nh[0], 0.25 * nh[1], 0.0], lattice=D2Q5, threads=8,
                link_delta=g.link_delta if general else None,
                link_normal=w.link_normal(g) if curved else None)
    jj = np.arange(n) * dx
    XX, YY = np.meshgrid(jj, jj)
    s = np.mod(XX * nh[0] + YY * nh[1], X / math.sqrt(5.0))
    inside = (s > bounds[0]) & (s < bounds[-1])
    r = [pins.slab_fv_reference(bounds, Dv[1:], T2v[1:], kap_if, 0.25, f, dt, s[inside], c)
         for c in (40, 80)]
    ref = (4 * r[1] - r[0]) / 3
    return dx, np.linalg.norm(M[0][inside] - ref) / np.linalg.norm(ref)


def test_tilted_walls_and_membranes_theta_zero():
    # Sec. 2.4.2: the theta = 0 form imposes the flux along the link.  For
    # impermeable walls at 26.6 / 63.4 degrees with a field that varies only
    # along the normal that is exact (no tangential flux), and the condition
    # converges; for a permeable tilted membrane it imposes kappa dM along
    # the link instead of the normal, an O(1) error that does not shrink with
    # dx -- a few percent here, as Sec. 3.5 reports for theta = 0
    # (the sub-link positions change from one spacing to the next, so the
    # order is taken over the whole refinement 40 -> 160)
    walls = [_tilted_case(n, [2.03, 7.33], [], True) for n in (40, 80, 160)]
    o = math.log(walls[0][1] / walls[-1][1]) / math.log(walls[0][0] / walls[-1][0])
    print("walls", [f"{e:.3e}" for _, e in walls], o)
    assert o > 1.8 and walls[-1][1] < 1e-3
    perm = [_tilted_case(n, [2.03, 4.71, 7.33], [0.05], True) for n in (40, 80, 160)]
    print("permeable", [f"{e:.3e}" for _, e in perm])
    assert all(0.01 < e < 0.06 for _, e in perm)
    assert abs(perm[-1][1] / perm[0][1] - 1.0) < 0.2


_tilt_curved = {}


def test_curved_membrane_converges_on_tilted_slabs():
    # Sec. 2.4.2 / Appendix B with theta != 0: the permeable membrane at 26.6
    # and 63.4 degrees to the links, where the theta = 0 form stays ~3 % off
    # (test above), converges towards the 1D finite-volume solution along the
    # normal: 9.9e-3, 2.9e-3, 1.2e-3 at 40, 80, 160 nodes, 26x below theta = 0
    # at 160 (6.1e-4 at 320, measured once, 50x).  The impermeable walls,
    # where imposing zero flux along the link is exact for a field that
    # varies along the normal only, stay near 1e-3 at 160.
    perm = [_tilted_case(n, [2.03, 4.71, 7.33], [0.05], True, True) for n in (40, 80, 160)]
    walls = [_tilted_case(n, [2.03, 7.33], [], True, True) for n in (40, 80, 160)]
    print("curved permeable", [f"{e:.3e}" for _, e in perm])
    print("curved walls", [f"{e:.3e}" for _, e in walls])
    assert perm[0][1] > perm[1][1] > perm[2][1]
    assert perm[2][1] < 1.5e-3 and perm[0][1] / perm[2][1] > 6.0
    assert walls[0][1] > walls[1][1] > walls[2][1] and walls[2][1] < 1.5e-3
    theta0 = _tilted_case(160, [2.03, 4.71, 7.33], [0.05], True, False)[1]
    assert perm[2][1] < 0.1 * theta0


def _cyl_curved(bc_periodic):
    g = w.cylinders_z((12, 11, 4), 0.25, seed=61, vf_target=0.5, periodic=bc_periodic)
    return g, w.link_delta(g), w.link_normal(g)


def test_curved_membrane_with_normals_along_links_is_theta_zero():
    # normals along every link (theta = 0): the curved rule is the theta = 0
    # rule (the Delta_m = 0 relations drop out); mirrored faces, where neither
    # rule reaches through the faces
    g, ld, _ = _cyl_curved(False)
    ln = np.zeros((3, 3) + g.comp.shape, np.float32)
    for a in range(3):
        ln[a, a] = -1.0 if a == 1 else 1.0      # the orientation is free
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    args = (g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, [2.0, 1.0], [90.0, 70.0],
            [[INF, 0.03], [0.03, INF]], f, [0.0, 4.0, 0.0])
    E0, M0 = _run(*args, link_delta=ld)
    E1, M1 = _run(*args, link_delta=ld, link_normal=ln)
    assert np.max(np.abs(E1 - E0)) < 1e-13
    assert np.max(np.abs(M1 - M0)) < 1e-13
    # with the surface normals the result differs (the tangential flux)
    _, _, lnc = _cyl_curved(False)
    E2, _ = _run(*args, link_delta=ld, link_normal=lnc)
    assert np.max(np.abs(E2 - E0)) > 1e-8


@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1]])
def test_curved_membrane_uniform_decay(bc):
    # G = 0, one T2: the uniform state is a fixed point of the curved rule
    # (its weights reproduce a uniform population set), E_k = exp(-k dt/T2)
    g, ld, ln = _cyl_curved(bc[0] == 0)
    E, _ = _run(g.comp, g.comp_phase, 2, bc, 0.25, 0.004, [2.0, 1.0], [40.0, 40.0],
                [[INF, 0.02], [0.02, INF]], np.zeros(80), [0, 0, 0], link_delta=ld,
                link_normal=ln)
    k = np.arange(81)
    assert np.max(np.abs(E - np.exp(-k * 0.004 / 40.0))) < 1e-13


def test_curved_membrane_mirror_rule_equals_doubling():
    # axis-aligned gradient on mirrored faces: the paper's buffer rule and the
    # reflected, doubled medium (membrane positions and normals reflected)
    g, ld, ln = _cyl_curved(False)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    args = (g.comp, g.comp_phase, 2, [1, 1, 1], 0.25, 0.004, [2.0, 1.0], [90.0, 70.0],
            [[INF, 0.03], [0.03, INF]], f, [0.0, 4.0, 0.0])
    Ep, _ = _run(*args, mirror="paper", link_delta=ld, link_normal=ln)
    Ed, _ = _run(*args, mirror="double", link_delta=ld, link_normal=ln)
    assert np.max(np.abs(Ep - Ed)) < 1e-13
    E0, _ = _run(*args, link_delta=ld)
    assert np.max(np.abs(Ep - E0)) > 1e-8
