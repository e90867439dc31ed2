"""Adjoint (reverse-mode gradient) of the HIP path, through the C ABI.

References: central finite differences of the FP64 CPU oracle (loss linear
in E with random weights, so the only error of the difference quotient is
its O(h^2) truncation), and the closed form dE_K/dT2 = (K dt / T2^2) E_K of
pure T2 decay.  Bounds: FP64 storage within 1e-6 relative of the FD value,
FP32 storage within 1e-3 relative (of the largest gradient component of
the same kind).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu
INF = math.inf


def _gpu():
    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    btl.load_library()
    return btl, torch


def _loss_weights(Q, K, seed=7):
    r = np.random.default_rng(seed)
    return r.normal(size=(Q, K + 1)), r.normal(size=(Q, K + 1))


def _oracle_loss(cfg, D, T2, kap, f, a, b):
    c = dict(cfg)
    c.update(D=np.asarray(D, float), T2=np.asarray(T2, float), kappa=np.asarray(kap, float),
             f=np.asarray(f, float))
    E, _ = oracle.simulate_config(c, threads=8)
    return float(np.sum(a * E.real + b * E.imag))


def _fd(cfg, a, b, which, idx, h_rel=1e-5):
    D, T2, kap, f = (np.array(cfg["D"], float), np.array(cfg["T2"], float),
                     np.array(cfg["kappa"], float), np.array(cfg["f"], float))
    arrs = {"D": D, "T2": T2, "kappa": kap, "f": f}
    x = arrs[which]
    base = x[idx]
    h = h_rel * max(abs(base), 1e-3 if which != "f" else 1.0)
    vals = []
    for sgn in (1, -1):
        y = x.copy()
        y[idx] = base + sgn * h
        if which == "kappa":
            y[idx[::-1]] = base + sgn * h
        args = dict(D=D, T2=T2, kap=kap, f=f)
        args[{"D": "D", "T2": "T2", "kappa": "kap", "f": "f"}[which]] = y
        vals.append(_oracle_loss(cfg, args["D"], args["T2"], args["kap"], args["f"], a, b))
    return (vals[0] - vals[1]) / (2 * h)


def _gpu_grads(cfg, prec, a, b, ckpt, **options):
    btl, torch = _gpu()
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, **options)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        cfg["q_geom"], ckpt_every=ckpt)
        g = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        P = len(cfg["D"])
        dD, dT2, dk, df = sim.backward(g, P, len(cfg["f"]))
        torch.cuda.synchronize()
        return dD.cpu().numpy(), dT2.cpu().numpy(), dk.cpu().numpy(), df.cpu().numpy()
    finally:
        sim.close()


def _cfg_small(bc, seed=51, K=160, n=(12, 10, 8), gG=None):
    g = w.cylinders_z(n, 0.25, seed=seed, vf_target=0.5, periodic=(bc[0] == 0))
    f = w.pgse_waveform(0.12, 0.4, 0.004)[:K]
    if gG is None:
        gG = np.array([[9.0, 5.0, 3.0], [-4.0, 8.0, 0.0]])
    return dict(name="adj", geoms=[g], bc=bc, dx=0.25, dt=0.004, D=np.array([2.0, 1.0]),
                T2=np.array([40.0, 25.0]), kappa=np.array([[INF, 0.05], [0.05, INF]]),
                f=f, gG0=gG, q_geom=np.zeros(len(gG), np.int32))


def _compare(cfg, prec, ckpt, tol, fidx=(0, 20, 55, 120)):
    Q, K = len(cfg["gG0"]), len(cfg["f"])
    a, b = _loss_weights(Q, K)
    dD, dT2, dk, df = _gpu_grads(cfg, prec, a, b, ckpt)
    checks = [("D", (0,), dD[0]), ("D", (1,), dD[1]), ("T2", (0,), dT2[0]),
              ("T2", (1,), dT2[1]), ("kappa", (0, 1), dk[0, 1] + dk[1, 0])]
    checks += [("f", (i,), df[i]) for i in fidx if i < K]
    scale = {}
    fds = []
    for which, idx, gval in checks:
        fd = _fd(cfg, a, b, which, idx if which != "D" and which != "T2" and which != "f"
                 else idx[0])
        fds.append((which, idx, gval, fd))
        scale[which] = max(scale.get(which, 0.0), abs(fd))
    for which, idx, gval, fd in fds:
        err = abs(gval - fd) / max(scale[which], 1e-30)
        print(f"{prec} {which}{idx}: adjoint {gval:.9e} fd {fd:.9e} rel {err:.2e}", flush=True)
        assert err <= tol, (which, idx, gval, fd)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-3)])
def test_adjoint_periodic_vs_oracle_fd(prec, tol):
    cfg = _cfg_small([0, 0, 0])
    _compare(cfg, prec, ckpt=40, tol=tol)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-3)])
def test_adjoint_mirror_oblique_vs_oracle_fd(prec, tol):
    # mirrored faces with oblique gradients: image fields and their
    # conjugate couplings in the transposed stream
    cfg = _cfg_small([1, 1, 1], seed=52, gG=np.array([[7.0, -5.0, 0.0], [3.0, 2.0, 6.0]]))
    _compare(cfg, prec, ckpt=33, tol=tol)


def test_adjoint_T2_closed_form():
    # G = 0, one phase, uniform medium: E_K = exp(-K dt / T2), so
    # dE_K/dT2 = (K dt / T2^2) E_K and dL/dD = dL/dkappa = 0
    btl, torch = _gpu()
    g = w.uniform((8, 8, 8), 0.5)
    K, dt, T2 = 300, 0.01, 30.0
    cfg = dict(geoms=[g], bc=[0, 0, 0], dt=dt, D=np.array([1.5]), T2=np.array([T2]),
               kappa=np.array([[INF]]), f=np.zeros(K), gG0=np.zeros((1, 3)),
               q_geom=np.zeros(1, np.int32))
    a = np.zeros((1, K + 1))
    a[0, K] = 1.0
    dD, dT2, dk, df = _gpu_grads(cfg, "f64", a, np.zeros_like(a), ckpt=64)
    EK = math.exp(-K * dt / T2)
    assert abs(dT2[0] - K * dt / T2 ** 2 * EK) < 1e-12
    assert abs(dD[0]) < 1e-13


def test_checkpoint_interval_does_not_change_gradients():
    cfg = _cfg_small([0, 0, 0], seed=53, K=90)
    Q, K = len(cfg["gG0"]), len(cfg["f"])
    a, b = _loss_weights(Q, K, seed=3)
    r1 = _gpu_grads(cfg, "f64", a, b, ckpt=90)
    r2 = _gpu_grads(cfg, "f64", a, b, ckpt=7)
    for x, y in zip(r1, r2):
        assert np.allclose(x, y, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_launch_geometry_does_not_change_gradients(prec):
    # the adjoint steps may walk whole z columns or short chunks, in plain
    # or XCD-contiguous workgroup order (chosen when the tape is recorded;
    # btl_set_adjoint_launch fixes them): the gradients agree to rounding
    # order, and with the mirror faces the chunks cross the image-field
    # partners' face rows
    cfg = _cfg_small([1, 1, 1], seed=57, K=70, n=(14, 12, 11))
    Q, K = len(cfg["gG0"]), len(cfg["f"])
    a, b = _loss_weights(Q, K, seed=5)
    ref = _gpu_grads(cfg, prec, a, b, ckpt=20, adjoint_launch=(0, 0))
    tol = 1e-12 if prec == "f64" else 1e-6
    for zc, xcd in ((1, 0), (3, 1), (4, 0), (0, 1), (2, 1)):
        got = _gpu_grads(cfg, prec, a, b, ckpt=20, adjoint_launch=(zc, xcd))
        for x, y in zip(ref, got):
            scale = max(np.max(np.abs(x)), 1e-30)
            assert np.max(np.abs(x - y)) <= tol * scale, (zc, xcd, x, y)


def _fd_gG0(cfg, a, b, q, ax, h=2e-4):
    vals = []
    for sgn in (1, -1):
        c = dict(cfg)
        g = np.array(cfg["gG0"], float).copy()
        g[q, ax] += sgn * h
        c["gG0"] = g
        E, _ = oracle.simulate_config(c, threads=8)
        vals.append(float(np.sum(a * E.real + b * E.imag)))
    return (vals[0] - vals[1]) / (2 * h)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-3)])
@pytest.mark.parametrize("bc", [[0, 0, 0], [1, 1, 1], [1, 0, 1]])
def test_adjoint_gG0_vs_oracle_fd(prec, tol, bc):
    # dL/d(gamma G0) through the reaction phase and the face factors, for a
    # fully oblique q-sample and one without a z component (on mirrored
    # faces that one needs the full field set: btl_set_grad_gG0)
    btl, torch = _gpu()
    cfg = _cfg_small(bc, seed=61, K=80, n=(10, 9, 7))
    Q, K = len(cfg["gG0"]), len(cfg["f"])
    a, b = _loss_weights(Q, K, seed=9)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], prec, grad_gG0=True)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                        cfg["q_geom"], ckpt_every=30)
        g = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        dG = sim.backward(g, 2, K, grad_gG0=True)[4].cpu().numpy()
    finally:
        sim.close()
    fd = np.array([[_fd_gG0(cfg, a, b, q, ax) for ax in range(3)] for q in range(Q)])
    scale = np.max(np.abs(fd))
    for q in range(Q):
        for ax in range(3):
            err = abs(dG[q, ax] - fd[q, ax]) / scale
            print(f"{prec} bc={bc} dgG0[{q},{ax}]: adjoint {dG[q, ax]:.9e} fd {fd[q, ax]:.9e} "
                  f"rel {err:.2e}", flush=True)
    assert np.max(np.abs(dG - fd)) <= tol * scale


def test_adjoint_ragged_batch_vs_oracle_fd():
    # two geometries of different sizes in one batch: q-samples map to their
    # own geometry's fields in the per-field sums (D, kappa, gamma G0)
    btl, torch = _gpu()
    geoms = [w.cylinders_z((11, 9, 6), 0.25, seed=71, vf_target=0.5, periodic=False),
             w.cylinders_z((9, 12, 7), 0.25, seed=72, vf_target=0.5, periodic=False)]
    f = w.pgse_waveform(0.12, 0.3, 0.004)
    gG = np.array([[8.0, 3.0, 2.0], [-5.0, 7.0, 0.0], [4.0, 0.0, 6.0]])
    cfg = dict(name="adj-ragged", geoms=geoms, bc=[1, 1, 1], dx=0.25, dt=0.004,
               D=np.array([2.0, 1.0]), T2=np.array([40.0, 25.0]),
               kappa=np.array([[INF, 0.05], [0.05, INF]]), f=f, gG0=gG,
               q_geom=np.array([0, 1, 1], np.int32))
    Q, K = len(gG), len(f)
    a, b = _loss_weights(Q, K, seed=13)
    sim = btl.Simulator(geoms, cfg["bc"], "f64", grad_gG0=True)
    try:
        E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], f, gG, cfg["q_geom"],
                        ckpt_every=20)
        g = torch.tensor(np.stack([a, b], axis=-1), dtype=torch.float64, device=E.device)
        dD, dT2, dk, df, dG = [t.cpu().numpy() for t in sim.backward(g, 2, K, grad_gG0=True)]
    finally:
        sim.close()
    checks = [(dD[1], _fd(cfg, a, b, "D", 1)), (dk[0, 1] + dk[1, 0], _fd(cfg, a, b, "kappa", (0, 1))),
              (dG[1, 1], _fd_gG0(cfg, a, b, 1, 1)), (dG[2, 2], _fd_gG0(cfg, a, b, 2, 2)),
              (dG[0, 0], _fd_gG0(cfg, a, b, 0, 0))]
    for got, fd in checks:
        print(f"ragged: adjoint {got:.9e} fd {fd:.9e}", flush=True)
        assert abs(got - fd) <= 1e-6 * max(abs(fd), 1e-3)


def test_gG0_gradient_field_set():
    # the full field set leaves the signal unchanged; without it a mirrored
    # axis with no gradient component has nothing to differentiate
    btl, torch = _gpu()
    cfg = _cfg_small([1, 1, 1], seed=62, K=60, n=(10, 9, 7))
    Q, K = len(cfg["gG0"]), len(cfg["f"])
    Es = []
    for full in (False, True):
        sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64", grad_gG0=full)
        try:
            E = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"],
                            cfg["q_geom"], ckpt_every=20)
            Es.append(E.cpu().numpy())
            g = torch.zeros((Q, K + 1, 2), dtype=torch.float64, device=E.device)
            if not full:
                sim.backward(g, 2, K)        # the other gradients still work
                with pytest.raises(btl.BtlError) as ei:
                    sim.backward(g, 2, K, grad_gG0=True)
                assert ei.value.status == btl.BTL_E_UNSUPPORTED
                with pytest.raises(btl.BtlError) as ei:
                    btl.btl_set_grad_gG0(sim._h, 2)
                assert ei.value.status == btl.BTL_E_INVAL
        finally:
            sim.close()
    assert np.max(np.abs(Es[0] - Es[1])) < 1e-13


def test_autograd_gG0_tensor():
    btl, torch = _gpu()
    cfg = _cfg_small([1, 1, 1], seed=63, K=50, n=(10, 9, 7))
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    try:
        D = torch.tensor(cfg["D"], requires_grad=True)
        G = torch.tensor(cfg["gG0"], requires_grad=True)
        E = btl.bloch_torrey_signal(D, torch.tensor(cfg["T2"]), torch.tensor(cfg["kappa"]),
                                    torch.tensor(cfg["f"]), sim, cfg["dt"], G, ckpt_every=25)
        (E[:, -1, 0] ** 2 + E[:, -1, 1] ** 2).sum().backward()
    finally:
        sim.close()
    assert G.grad.shape == (2, 3) and torch.isfinite(G.grad).all()
    assert D.grad is not None


def test_autograd_function():
    btl, torch = _gpu()
    cfg = _cfg_small([0, 0, 0], seed=54, K=80)
    sim = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    try:
        D = torch.tensor(cfg["D"], requires_grad=True)
        T2 = torch.tensor(cfg["T2"], requires_grad=True)
        kap = torch.tensor(cfg["kappa"], requires_grad=True)
        samples = torch.tensor(np.asarray(cfg["f"])[::8], requires_grad=True)
        f = samples.repeat_interleave(8)[:len(cfg["f"])]
        E = btl.bloch_torrey_signal(D, T2, kap, f, sim, cfg["dt"], cfg["gG0"], ckpt_every=25)
        loss = (E[:, -1, 0] ** 2 + E[:, -1, 1] ** 2).sum()
        loss.backward()
        # a second taped forward on the same simulator replaces the tape: the
        # first graph's backward is refused, the second's runs
        E1 = btl.bloch_torrey_signal(D, T2, kap, f, sim, cfg["dt"], cfg["gG0"], ckpt_every=25)
        E2 = btl.bloch_torrey_signal(D, T2, kap, f, sim, cfg["dt"], cfg["gG0"], ckpt_every=25)
        with pytest.raises(RuntimeError, match="adjoint tape is gone"):
            E1[:, -1, 0].sum().backward()
        g0 = D.grad.clone()
        E2[:, -1, 0].sum().backward()
        assert not torch.equal(D.grad, g0)
    finally:
        sim.close()
    assert D.grad.shape == (2,) and torch.isfinite(D.grad).all()
    assert samples.grad.shape == samples.shape and torch.isfinite(samples.grad).all()
    assert kap.grad[0, 1] == kap.grad[1, 0]


def test_cfg4_full_size_gradients_vs_fp64_fd():
    # The adjoint workload at full size (96^3 cylinders, 4000 steps,
    # checkpoint every 100): loss = sum_q |E_q(TE) - E_target,q|^2 with the
    # target made from perturbed parameters (D x1.1/0.9, T2 x1.1/0.9,
    # kappa x1.5); the waveform is parametrized by 200 samples of 20 steps.
    # FP32-storage adjoint vs central differences of the FP64-storage GPU
    # forward (itself checked against the oracle to rounding order on the
    # reduced cases; a full-size oracle forward would take the host about an
    # hour per difference quotient); all 30 q-samples.
    btl, torch = _gpu()
    cfg = w.make_config("cfg4")
    assert len(cfg["gG0"]) == 30
    K = len(cfg["f"])
    dt = cfg["dt"]
    D0, T20, k0 = np.array(cfg["D"]), np.array(cfg["T2"]), np.array(cfg["kappa"])
    samples0 = np.asarray(cfg["f"])[::20].copy()
    sim64 = btl.Simulator(cfg["geoms"], cfg["bc"], "f64")
    sim32 = btl.Simulator(cfg["geoms"], cfg["bc"], "f32")
    try:
        def fwd64(D, T2, kap, samples):
            f = np.repeat(samples, 20)[:K]
            return sim64.forward(dt, D, T2, kap, f, cfg["gG0"])[:, -1].cpu().numpy()

        kt = k0.copy()
        kt[0, 1] = kt[1, 0] = k0[0, 1] * 1.5
        Et = fwd64(D0 * np.array([1.1, 0.9]), T20 * np.array([1.1, 0.9]), kt, samples0)

        def loss64(D, T2, kap, samples):
            return float(np.sum(np.abs(fwd64(D, T2, kap, samples) - Et) ** 2))

        D = torch.tensor(D0, requires_grad=True)
        T2 = torch.tensor(T20, requires_grad=True)
        kap = torch.tensor(k0[0, 1], requires_grad=True)
        smp = torch.tensor(samples0, requires_grad=True)
        kmat = torch.stack([torch.stack([torch.tensor(math.inf, dtype=torch.float64), kap]),
                            torch.stack([kap, torch.tensor(math.inf, dtype=torch.float64)])])
        f = smp.repeat_interleave(20)[:K]
        print("GPU cfg4 96^3 K=4000 Q=30 f32 adjoint", flush=True)
        E = btl.bloch_torrey_signal(D, T2, kmat, f, sim32, dt, cfg["gG0"], ckpt_every=100)
        Etc = torch.tensor(np.stack([Et.real, Et.imag], -1))
        loss = ((E[:, -1, :].cpu() - Etc) ** 2).sum()
        loss.backward()
        g = {"D0": D.grad[0].item(), "D1": D.grad[1].item(), "T20": T2.grad[0].item(),
             "T21": T2.grad[1].item(), "kappa": kap.grad.item(),
             "s10": smp.grad[10].item(), "s80": smp.grad[80].item(),
             "s160": smp.grad[160].item()}

        def fd(name):
            Dv, Tv, kv, sv = D0.copy(), T20.copy(), k0.copy(), samples0.copy()
            if name[0] == "D":
                x, i = Dv, int(name[1])
            elif name[:2] == "T2":
                x, i = Tv, int(name[2])
            elif name == "kappa":
                x, i = None, None
            else:
                x, i = sv, int(name[1:])
            vals = []
            for sgn in (1, -1):
                if x is None:
                    h = 1e-4 * k0[0, 1]
                    kk = k0.copy()
                    kk[0, 1] = kk[1, 0] = k0[0, 1] + sgn * h
                    vals.append(loss64(Dv, Tv, kk, sv))
                else:
                    h = 1e-4 * max(abs(x[i]), 1e-2)
                    y = x.copy()
                    y[i] += sgn * h
                    args = {"D": (y, Tv, k0, sv), "T": (Dv, y, k0, sv), "s": (Dv, Tv, k0, y)}[name[0]]
                    vals.append(loss64(*args))
            return (vals[0] - vals[1]) / (2 * h)

        scale = {}
        res = {}
        for name in g:
            res[name] = fd(name)
            kind = name[0] if name != "kappa" else "k"
            scale[kind] = max(scale.get(kind, 0.0), abs(res[name]))
        for name in g:
            kind = name[0] if name != "kappa" else "k"
            err = abs(g[name] - res[name]) / scale[kind]
            print(f"{name}: adjoint {g[name]:.6e} fd64 {res[name]:.6e} rel {err:.2e}", flush=True)
            assert err < 1e-3, name
    finally:
        sim64.close()
        sim32.close()
