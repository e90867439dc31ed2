"""Adjoint of the HIP path against the tangent-linear map of the FP64 oracle
(FP64 storage).

For a loss linear in the signal, L = sum_k a_k Re E_k + b_k Im E_k, the
adjoint returns J^T w with J = dE/d(theta) and w = (a, b); the tangent-linear
map gives J v for a direction v.  The identity <J v, w> = <v, J^T w> is
checked component by component (v = unit vectors), with J v taken from the
FP64 oracle by a fourth-order central difference:

    J v ~ [-E(t + 2h) + 8 E(t + h) - 8 E(t - h) + E(t - 2h)] / (12 h),

with h = 1e-3 of the parameter's scale: truncation near 1e-12 relative.
Its rounding error is bounded by 1.5 eps_L / h, eps_L = 10 eps sum_k
(|a_k| + |b_k|) the rounding of the loss itself.  The bound on each
component is 1e-9 of the largest tangent-linear value of the same kind
plus that rounding bound -- three orders below what the second-order
differences of the FD tests resolve.  The unperturbed forward is also
checked against the dense real step matrices of `tests/pins.py` (the scheme
of Sec. 2.3 with the boundary rules of Sec. 2.4 assembled entry by entry,
sharing no code with the oracle or the library).  Short runs (4 steps) make
it a check of the adjoint of each stage of a step (there the signal has barely left
equilibrium and the rounding term dominates for kappa); longer ones (24
steps, a bipolar waveform) of the accumulated wrap phase and the waveform
sensitivities.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as w

from . import pins

pytestmark = pytest.mark.gpu
INF = math.inf


def _gpu():
    import torch
    import paper_1907_00908_amd as btl
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    btl.load_library()
    return btl, torch


def _geometry():
    # 5 x 4 x 3 sites: a 2 x 2 square "axon" along z (phase 1) in phase 0,
    # so the lattice has membrane links on x and y, and a z face crossing
    comp = np.zeros((3, 4, 5), np.uint32)
    comp[:, 1:3, 1:3] = 1
    return w.Geometry(comp=comp, comp_phase=np.array([0, 1], np.uint8), n_phase=2, dx=0.25)


def _oracle_E(g, bc, dt, D, T2, kap, f, gG0):
    E, _ = oracle.simulate(g.comp, g.comp_phase, g.n_phase, bc, g.dx, dt, D, T2, kap, f, gG0)
    return E


def _dense_E(g, bc, dt, D, T2, kap, f, gG0):
    mats = pins.dense_step_matrices(g.comp, g.comp_phase, bc, g.dx, dt, D, T2, kap, f, gG0,
                                    factors=True)
    return pins.dense_run(mats, g.comp.size)


def _d4(fun, x0, h):
    return (-fun(x0 + 2 * h) + 8 * fun(x0 + h) - 8 * fun(x0 - h) + fun(x0 - 2 * h)) / (12 * h)


CASES = {
    # periodic faces, fully oblique gradient (wrap phase on every axis)
    "periodic-oblique": ([0, 0, 0], np.array([30.0, -18.0, 12.0])),
    # mirrored faces, gradient along x: the conjugating rule on x, the plain
    # reflection on y and z (Sec. 2.4.4)
    "mirror-x": ([1, 1, 1], np.array([30.0, 0.0, 0.0])),
}


@pytest.mark.parametrize("K", [4, 24])
@pytest.mark.parametrize("case", sorted(CASES))
def test_adjoint_equals_tangent_linear_of_dense_scheme(case, K):
    btl, torch = _gpu()
    bc, G = CASES[case]
    g = _geometry()
    dt = 0.01
    D = np.array([2.0, 1.2])
    T2 = np.array([40.0, 25.0])
    kap = np.array([[INF, 0.05], [0.05, INF]])
    f = np.concatenate([np.ones(K // 3), np.zeros(K - 2 * (K // 3)), -np.ones(K // 3)])
    f = f + 0.1 * np.sin(np.arange(K))       # no two samples alike
    r = np.random.default_rng(17 + K)
    a, b = r.normal(size=K + 1), r.normal(size=K + 1)

    print(f"GPU tangent-linear {case} K={K}", flush=True)
    sim = btl.Simulator([g], bc, "f64", grad_gG0=(bc == [0, 0, 0]))
    try:
        E = sim.forward(dt, D, T2, kap, f, G[None, :], ckpt_every=max(1, K // 3))
        wgt = torch.tensor(np.stack([a, b], axis=-1)[None], dtype=torch.float64,
                           device=E.device)
        out = [t.cpu().numpy() for t in sim.backward(wgt, grad_gG0=(bc == [0, 0, 0]))]
        Eg = E.cpu().numpy()[0]        # complex, K + 1 values
    finally:
        sim.close()
    dD, dT2, dk, df = out[:4]

    # the same forward in all three formulations
    E0 = _dense_E(g, bc, dt, D, T2, kap, f, G)
    assert np.max(np.abs(_oracle_E(g, bc, dt, D, T2, kap, f, G) - E0)) < 1e-13
    assert np.max(np.abs(Eg - E0)) < 1e-12

    def L(E):
        return float(np.sum(a * E.real + b * E.imag))

    rows = []   # (kind, name, adjoint, tangent-linear, h)

    def tl_row(kind, name, adj, fun, x0, h):
        rows.append((kind, name, adj, _d4(fun, x0, h), h))

    for p in range(2):
        def fD(x, p=p):
            Dv = D.copy()
            Dv[p] = x
            return L(_oracle_E(g, bc, dt, Dv, T2, kap, f, G))

        def fT(x, p=p):
            Tv = T2.copy()
            Tv[p] = x
            return L(_oracle_E(g, bc, dt, D, Tv, kap, f, G))
        tl_row("D", f"D{p}", dD[p], fD, D[p], 1e-3 * D[p])
        tl_row("T2", f"T2{p}", dT2[p], fT, T2[p], 1e-3 * T2[p])

    def fk(x):
        kv = kap.copy()
        kv[0, 1] = kv[1, 0] = x
        return L(_oracle_E(g, bc, dt, D, T2, kv, f, G))
    # the pair's kappa enters both entries of the symmetric matrix
    tl_row("kappa", "kappa01", dk[0, 1] + dk[1, 0], fk, kap[0, 1], 1e-3 * kap[0, 1])
    for i in range(K):
        def ff(x, i=i):
            fv = f.copy()
            fv[i] = x
            return L(_oracle_E(g, bc, dt, D, T2, kap, fv, G))
        tl_row("f", f"f{i}", df[i], ff, f[i], 1e-3)
    if bc == [0, 0, 0]:
        dG = out[4]
        for ax in range(3):
            def fg(x, ax=ax):
                Gv = G.copy()
                Gv[ax] = x
                return L(_oracle_E(g, bc, dt, D, T2, kap, f, Gv))
            tl_row("gG0", f"gG0[{ax}]", dG[0, ax], fg, G[ax], 1e-3 * 30.0)

    eps_L = 10 * np.finfo(float).eps * float(np.sum(np.abs(a) + np.abs(b)))
    scale = {}
    for kind, _, _, tl, _ in rows:
        scale[kind] = max(scale.get(kind, 0.0), abs(tl))
    bad = []
    for kind, name, adj, tl, h in rows:
        bound = 1e-9 * scale[kind] + 1.5 * eps_L / h
        print(f"  {name}: adjoint {adj:.12e} tangent-linear {tl:.12e} |diff| {abs(adj - tl):.1e} "
              f"bound {bound:.1e}", flush=True)
        if not abs(adj - tl) <= bound:
            bad.append(name)
    assert not bad, bad
