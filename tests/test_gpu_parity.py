"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances: FP64 storage agrees with the oracle to rounding order,
|dE| <= 1e-12 |E| + 1e-14.  FP32 storage (FP64 arithmetic, FP64 signal sums)
meets the stated bound |dE| <= 1e-5 |E| where |E| >= 1e-2, and 1e-7 absolute
below that (relative error is ill-posed near diffraction minima).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu
INF = math.inf

TOL = {"f64": (1e-12, 1e-14), "f32": (1e-5, 1e-7)}


def _gpu():
    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    btl.load_library()
    return btl


def _check(Eg, Er, prec, what=""):
    Eg = np.asarray(Eg)
    Er = np.asarray(Er)
    assert Eg.shape == Er.shape
    err = np.abs(Eg - Er)
    if prec == "f32":
        big = np.abs(Er) >= 1e-2
        bound = np.where(big, 1e-5 * np.abs(Er), 1e-7)
    else:
        bound = TOL["f64"][0] * np.abs(Er) + TOL["f64"][1]
    worst = np.max(err / bound)
    print(f"{what} prec={prec} max|dE|={err.max():.3e} worst/bound={worst:.3f}", flush=True)
    assert worst <= 1.0


def _run_both(cfg, prec, want_M=False, threads=8):
    btl = _gpu()
    print(f"GPU {cfg['name']} prec={prec} shapes={[g.shape_xyz for g in cfg['geoms']]} "
          f"K={len(cfg['f'])} Q={len(cfg['gG0'])}", flush=True)
    out = btl.simulate_config(cfg, prec=prec, want_M=want_M)
    Eo, Mo = oracle.simulate_config(cfg, threads=threads, want_M=want_M)
    if want_M:
        Eg, Mg = out
        return Eg.cpu().numpy(), [m.cpu().numpy() for m in Mg], Eo, Mo
    return out.cpu().numpy(), None, Eo, None


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cfg1_small_uniform(prec):
    cfg = w.make_config("cfg1", n=16, K=600)
    Eg, _, Eo, _ = _run_both(cfg, prec)
    _check(Eg, Eo, prec, "cfg1 16^3")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cfg1_full(prec):
    cfg = w.make_config("cfg1")
    Eg, _, Eo, _ = _run_both(cfg, prec)
    _check(Eg, Eo, prec, "cfg1 32^3 K=2500")
    exact = math.exp(-2.5) * math.exp(-25.0 / 80.0)
    assert abs(Eg[0, -1] - exact) / exact < 1.5e-3


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cfg2_reduced_mirror_oblique(prec):
    # mirror BC on all faces, six oblique directions: two image fields each
    cfg = w.make_config("cfg2", n=20, K=500)
    Eg, Mg, Eo, Mo = _run_both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg2 20^3 mirror oblique")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mirror_axis_aligned_and_3axis_oblique(prec):
    g = w.cylinders_z((14, 12, 9), 0.25, seed=41, vf_target=0.55, periodic=False)
    f = w.pgse_waveform(0.4, 1.2, 0.004)
    gG = np.array([[6.0, 0, 0], [0, 0, 5.0], [3.0, -2.0, 4.0], [0, 0, 0]])
    cfg = dict(name="mirror-mix", geoms=[g], bc=[1, 1, 1], dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([90.0, 70.0]),
               kappa=np.array([[INF, 0.02], [0.02, INF]]), f=f, gG0=gG,
               q_geom=np.zeros(len(gG), np.int32))
    Eg, Mg, Eo, Mo = _run_both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "mirror axis/3-axis oblique")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mixed_bc_oblique(prec):
    # mirrored x with periodic y, z and an oblique gradient: no conjugate
    # pairing, image fields for every sign pattern
    g = w.cylinders_z((12, 10, 6), 0.25, seed=42, vf_target=0.5)
    f = w.pgse_waveform(0.3, 0.9, 0.004)
    gG = np.array([[4.0, 3.0, 0.0], [-2.0, 0.0, 5.0], [0.0, 4.0, 1.0]])
    cfg = dict(name="mixed-bc", geoms=[g], bc=[1, 0, 0], dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([90.0, 70.0]),
               kappa=np.array([[INF, 0.05], [0.05, INF]]), f=f, gG0=gG,
               q_geom=np.zeros(len(gG), np.int32))
    Eg, _, Eo, _ = _run_both(cfg, prec)
    _check(Eg, Eo, prec, "mixed bc")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_periodic_cylinders_ragged_tail(prec):
    # site count not a multiple of the workgroup size; membranes on wrap links
    cfg = w.make_config("cfg4", n=(13, 11, 7), K=400, n_q=5)
    Eg, Mg, Eo, Mo = _run_both(cfg, prec, want_M=True)
    _check(Eg, Eo, prec, "cfg4 13x11x7")
    for q in range(len(Mo)):
        _check(Mg[q], Mo[q], prec, f"M_final q={q}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ragged_multi_geometry_batch(prec):
    cfg = w.make_config("cfg3b", n=24, K=300, n_q=2)
    cfg["geoms"] = cfg["geoms"][:5]
    sel = cfg["q_geom"] < 5
    cfg["gG0"], cfg["q_geom"] = cfg["gG0"][sel], cfg["q_geom"][sel]
    Eg, _, Eo, _ = _run_both(cfg, prec)
    _check(Eg, Eo, prec, "cfg3b ragged")
    # the q-samples of each geometry interleaved block by block (groups of
    # unequal sizes and grids), in both XCD orders
    btl = _gpu()
    for order in (2, 3):
        print(f"GPU ragged batch, workgroup order {order}", flush=True)
        sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, launch=(5, 4, order))
        try:
            E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                            cfg["q_geom"]).cpu().numpy()
        finally:
            sim.close()
        _check(E, Eo, prec, f"cfg3b ragged, order {order}")


def test_three_phase_cells_ogse():
    cfg = w.make_config("cfg5", n=40, K=400, n_q=3)
    Eg, _, Eo, _ = _run_both(cfg, "f32")
    _check(Eg, Eo, "f32", "cfg5 40^3 OGSE")


def test_membrane_limits_and_zero_steps():
    btl = _gpu()
    g = w.cylinders_z((10, 9, 5), 0.25, seed=43, vf_target=0.5)
    f = w.pgse_waveform(0.2, 0.6, 0.004)
    gG = np.array([[5.0, 2.0, 1.0]])
    for kap in (0.0, INF):
        cfg = dict(name=f"kappa={kap}", geoms=[g], bc=[0, 0, 0], dx=0.25, dt=0.004,
                   D=np.array([2.0, 1.0]), T2=np.array([90.0, INF]),
                   kappa=np.array([[INF, kap], [kap, INF]]), f=f, gG0=gG,
                   q_geom=np.zeros(1, np.int32))
        Eg, _, Eo, _ = _run_both(cfg, "f64")
        _check(Eg, Eo, "f64", f"kappa={kap}")
    cfg["f"] = f[:0]
    Eg = btl.simulate_config(cfg, prec="f32").cpu().numpy()
    assert Eg.shape == (1, 1) and Eg[0, 0] == 1.0


def test_deterministic_repeat():
    btl = _gpu()
    cfg = w.make_config("cfg4", n=16, K=200, n_q=3)
    E1 = btl.simulate_config(cfg, prec="f32").cpu().numpy()
    E2 = btl.simulate_config(cfg, prec="f32").cpu().numpy()
    assert np.array_equal(E1, E2)


def test_autotune_keeps_results():
    btl = _gpu()
    import torch
    cfg = w.make_config("cfg4", n=(20, 18, 24), K=120, n_q=3)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"])
        E1 = sim.forward(*args).cpu().numpy()
        assert btl.btl_get_launch(sim._h) == (-1, 0, -1)   # defaults before tuning
        btl.btl_autotune(sim._h, 3, 5, torch.cuda.current_stream().cuda_stream)
        tile, zc, xcd = btl.btl_get_launch(sim._h)
        assert tile in (0, 1, 2, 3, 5) and 0 <= zc < 24 and xcd in (0, 1, 2, 3)
        E2 = sim.forward(*args).cpu().numpy()
    finally:
        sim.close()
    Eo, _ = oracle.simulate_config(cfg)
    _check(E1, Eo, "f64", "before autotune")
    _check(E2, Eo, "f64", "after autotune")


_SHAPE_CACHE = {}


def _shape_case():
    cfg = w.make_config("cfg2", n=21, K=150)
    cfg["geoms"][0] = w.cylinders_z((21, 19, 9), 0.25, seed=23, vf_target=0.5, periodic=False)
    return cfg


def _shape_oracle(cfg):
    # the oracle's answer does not depend on the launch: computed once
    if "oracle" not in _SHAPE_CACHE:
        _SHAPE_CACHE["oracle"] = oracle.simulate_config(cfg, want_M=True, threads=8)
    return _SHAPE_CACHE["oracle"]


def _shape_ref_grads(btl, cfg, prec, args, g, K):
    # gradients of the default launch of a fresh simulator, once per precision
    key = ("grads", prec)
    if key not in _SHAPE_CACHE:
        sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec)
        try:
            sim.forward(*args, ckpt_every=50)
            _SHAPE_CACHE[key] = [t.cpu().numpy() for t in sim.backward(g, 2, K)]
        finally:
            sim.close()
    return _SHAPE_CACHE[key]


@pytest.mark.parametrize("shape,zc,xcd", [(5, 0, 0), (5, 3, 1), (2, 4, 0), (1, 0, 1),
                                          (0, 2, 1), (0, 0, 0), (3, 3, 1), (3, 0, 0),
                                          (5, 3, 3), (3, 0, 2), (0, 2, 2), (1, 4, 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_tile_shape_matches_oracle(shape, zc, xcd, prec):
    # each launch shape (5: runs of 256 consecutive sites of the x-y plane,
    # 3: 128x2, 2: 16x16, 1: 32x8, 0: 64x4), whole or chunked z columns, in
    # plain and XCD-contiguous workgroup order (xcd_tile renumbers the
    # workgroups), field after field or the image fields of a q-sample
    # interleaved block by block (order bit 1), on a ragged lattice with
    # mirrored faces, oblique gradients (image fields) and membranes: E and
    # M_final against the oracle, and the adjoint (in the same XCD order)
    # against the default launch
    btl = _gpu()
    import torch
    cfg = _shape_case()
    print(f"GPU launch shape={shape} zc={zc} xcd={xcd} prec={prec}", flush=True)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, launch=(shape, zc, xcd),
                        adjoint_launch=(-1, xcd & 1))
    try:
        args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"])
        E, M = sim.forward(*args, want_M=True)
        M = [m.cpu().numpy() for m in M]
        E2 = sim.forward(*args, ckpt_every=50)
        Q, K = len(cfg["gG0"]), len(cfg["f"])
        r = np.random.default_rng(3)
        g = torch.tensor(r.normal(size=(Q, K + 1, 2)), dtype=torch.float64, device=E.device)
        grads = [t.cpu().numpy() for t in sim.backward(g, 2, K)]
        E = E.cpu().numpy()
        assert np.array_equal(E, E2.cpu().numpy())
    finally:
        sim.close()
    Eo, Mo = _shape_oracle(cfg)
    _check(E, Eo, prec, f"shape {shape} zc {zc} xcd {xcd}")
    for q in range(len(Mo)):
        _check(M[q], Mo[q], prec, f"M_final q={q}")
    # gradients against the default launch shape of a fresh simulator
    ref = _shape_ref_grads(btl, cfg, prec, args, g, K)
    tol = 1e-11 if prec == "f64" else 1e-5
    for x, y in zip(grads, ref):
        assert np.max(np.abs(x - y)) <= tol * max(np.max(np.abs(y)), 1e-30)


def test_q_waves_match_single_batch():
    # a device-memory budget below the batch's population size splits the
    # q-samples into consecutive waves; every field is computed exactly as
    # in the single batch
    btl = _gpu()
    cfg = w.make_config("cfg4", n=(24, 20, 16), K=60, n_q=7)
    E1 = btl.simulate_config(cfg, prec="f32").cpu().numpy()
    per_q = 2 * 7 * 24 * 20 * 16 * 8
    Eg, Mg = btl.simulate_config(cfg, prec="f32", want_M=True, mem_budget=int(2.5 * per_q))
    assert np.array_equal(E1, Eg.cpu().numpy())
    _, M1 = btl.simulate_config(cfg, prec="f32", want_M=True)
    for a, b in zip(M1, Mg):
        assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_graph_replays_match_eager():
    # forwards of >= 16 steps run from a cached hipGraph; each replay, with
    # eager work and synchronizations in between, must equal the eager run
    btl = _gpu()
    import torch
    cfg = w.make_config("cfg2", n=(20, 18, 12), K=90, n_q=3)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f32")
    args = (cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"])
    try:
        btl.btl_set_graphs(sim._h, 0)
        E0 = sim.forward(*args, cfg["f"], cfg["gG0"]).cpu().numpy()
        btl.btl_set_graphs(sim._h, 1)
        for rep in range(3):
            E = sim.forward(*args, cfg["f"], cfg["gG0"]).cpu().numpy()
            assert np.array_equal(E, E0), rep
            # eager work of another shape in between (10 steps: no graph)
            sim.forward(*args, cfg["f"][:10], cfg["gG0"][:1])
            torch.cuda.synchronize()
        # changed parameters with the same shape replay the same graph
        D2 = np.array(cfg["D"]) * 1.1
        E2 = sim.forward(cfg["dt"], D2, cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"]).cpu().numpy()
        btl.btl_set_graphs(sim._h, 0)
        E2e = sim.forward(cfg["dt"], D2, cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"]).cpu().numpy()
        assert np.array_equal(E2, E2e)
        assert not np.array_equal(E2, E0)
    finally:
        sim.close()


def test_graph_key_tracks_field_layout():
    # a cached forward graph takes each field's range, plane stride and
    # q-sample as launch arguments: the same two geometries batched in the
    # other order have the same sizes and must still not replay it
    btl = _gpu()
    geoms = [w.cylinders_z((11, 9, 6), 0.25, seed=71, vf_target=0.5),
             w.cylinders_z((9, 12, 7), 0.25, seed=72, vf_target=0.5)]
    f = w.pgse_waveform(0.12, 0.3, 0.004)
    gG = np.array([[8.0, 2.0, 0.0], [-5.0, 0.0, 3.0]])
    args = (0.004, np.array([2.0, 1.0]), np.array([40.0, 25.0]),
            np.array([[INF, 0.05], [0.05, INF]]))
    sim = btl.Simulator(geoms, [0, 0, 0], "f32")
    try:
        seen = []
        for qg in ([0, 1], [1, 0]):
            Eg = sim.forward(*args, f, gG, qg).cpu().numpy()
            btl.btl_set_graphs(sim._h, 0)
            Ee = sim.forward(*args, f, gG, qg).cpu().numpy()
            btl.btl_set_graphs(sim._h, 1)
            assert np.array_equal(Eg, Ee), qg
            seen.append(Eg)
        assert not np.array_equal(seen[0], seen[1])
    finally:
        sim.close()


def test_invalid_arguments_raise():
    btl = _gpu()
    cfg = w.make_config("cfg1", n=4, K=3)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f32")
    try:
        with pytest.raises(btl.BtlError) as ei:
            sim.forward(cfg["dt"], np.array([-1.0]), cfg["T2"], cfg["kappa"], cfg["f"],
                        cfg["gG0"])
        assert ei.value.status == btl.BTL_E_INVAL
        with pytest.raises(btl.BtlError):
            sim.forward(-0.1, cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"])
        with pytest.raises(btl.BtlError):
            sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        q_geom=[3])
    finally:
        sim.close()


# ---- full-size cases, in the launch configuration of the benchmark ---------

def test_cfg2_full_size_sampled_steps():
    # the benchmark workload (128^3, mirror, oblique directions) for the first
    # 40 steps, two of the six q-samples checked against the oracle
    btl = _gpu()
    cfg = w.make_config("cfg2", K=40)
    print("GPU cfg2 128^3 K=40 f32", flush=True)
    Eg = btl.simulate_config(cfg, prec="f32").cpu().numpy()
    Eo, _ = oracle.simulate_config(cfg, q=[0, 5], threads=16)
    _check(Eg[[0, 5]], Eo, "f32", "cfg2 full size, 40 steps")


def test_cfg2_full_length_T2_decay_fp32():
    # full 128^3 geometry and 10^4 steps at zero gradient with one T2: the
    # exact answer is exp(-k dt / T2) at every step; FP32 storage must not
    # drift (per-step constants enter in conservation-preserving forms)
    btl = _gpu()
    cfg = w.make_config("cfg2")
    cfg["gG0"] = np.zeros((1, 3))
    cfg["q_geom"] = np.zeros(1, np.int32)
    cfg["T2"] = np.array([80.0, 80.0])
    print("GPU cfg2 128^3 K=10000 G=0 f32", flush=True)
    Eg = btl.simulate_config(cfg, prec="f32").cpu().numpy()[0]
    k = np.arange(len(Eg))
    ref = np.exp(-k * cfg["dt"] / 80.0)
    rel = np.max(np.abs(Eg - ref) / ref)
    print(f"max rel err over 10^4 steps {rel:.3e}", flush=True)
    assert rel < 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cfg2_64_full_length_vs_stored_oracle(prec):
    # the axon workload's law at 64^3 (mirror faces, oblique directions with
    # image fields), all 10^4 steps, against the oracle's signal stored by
    # tests/golden/make_cfg2_full.py (every 10th step and the last)
    import os
    btl = _gpu()
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "cfg2_64_full_E.npz"))
    cfg = w.make_config("cfg2", n=int(gold["n"]))
    qs = [int(q) for q in gold["qs"]]
    cfg["gG0"], cfg["q_geom"] = cfg["gG0"][qs], cfg["q_geom"][qs]
    assert np.array_equal(cfg["gG0"], gold["gG0"])
    print(f"GPU cfg2 64^3 K={len(cfg['f'])} q={qs} {prec}", flush=True)
    Eg = btl.simulate_config(cfg, prec=prec).cpu().numpy()[:, gold["steps"]]
    _check(Eg, gold["E"], prec, "cfg2 64^3 full length")
