"""The truncation-error harness on the GPU (uniform problem of Sec. 3.1,
Fig. 5): both schemes second order in dx at fixed tau, the hybrid error
independent of the domain size L, the classical error growing with L and
first order in dt.  Two points are checked against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu


def _conv():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1907_00908_amd import convergence
    return convergence


def _group(rows):
    g = {}
    for r in rows:
        g.setdefault((r["scheme"], r["L"]), []).append(r)
    return g


def test_spatial_convergence_and_domain_size():
    c = _conv()
    rows = c.spatial_sweep(dxs=(2.0, 1.0, 0.5, 0.25))
    g = _group(rows)
    for (s, L), rs in g.items():
        o = c.orders([r["err_l2"] for r in rs], [r["dx"] for r in rs])
        errs = " ".join("%.3e" % r["err_l2"] for r in rs)
        print(f"scheme={s} L={L} errs={errs} orders={o}", flush=True)
        assert all(1.8 < x < 2.2 for x in o), (s, L, o)
    hyb20, hyb100 = g[(0, 20.0)], g[(0, 100.0)]
    cl20, cl100 = g[(1, 20.0)], g[(1, 100.0)]
    for a, b, c20, c100 in zip(hyb20, hyb100, cl20, cl100):
        # hybrid: the same error for any L up to FP64 rounding of M (1e-15
        # of |M| per step); classical: 10x worse at 5x L
        assert abs(a["err_l2"] - b["err_l2"]) <= 1e-5 * a["err_l2"]
        assert c100["err_l2"] > 10 * c20["err_l2"] > 10 * 10 * a["err_l2"]


def test_temporal_convergence():
    c = _conv()
    rows = c.temporal_sweep()
    g = _group(rows)
    for L in (20.0, 100.0):
        cl = g[(1, L)]
        o = c.orders([r["err_l2"] for r in cl], [r["dt"] for r in cl])
        print(f"classical L={L} orders in dt {o}", flush=True)
        assert all(0.9 < x < 1.1 for x in o), o
        for h, k in zip(g[(0, L)], cl):
            assert h["err_l2"] < 0.1 * k["err_l2"]


@pytest.mark.parametrize("scheme", [0, 1])
def test_harness_matches_oracle(scheme):
    c = _conv()
    L, dx = 20.0, 1.0
    dt = c.dt_for_tau(0.6, dx, 2.0)
    r = c.uniform_error(L, dx, dt, scheme)
    g = w.uniform((int(L / dx), 2, 2), dx)
    f = c.pgse(5.0, 15.0, dt)
    _, M = oracle.simulate(g.comp, g.comp_phase, 1, [0, 0, 0], dx, dt, [2.0], [math.inf],
                           [[math.inf]], f, [c.gamma_g(23.16), 0, 0], want_M=True,
                           scheme=scheme)
    M = M.reshape(-1)
    e_or = np.linalg.norm(M - r["exact"]) / (r["exact"] * math.sqrt(M.size))
    print(f"scheme={scheme} gpu={r['err_l2']:.6e} oracle={e_or:.6e}", flush=True)
    assert abs(r["err_l2"] - e_or) < 1e-12
