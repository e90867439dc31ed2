"""Independent formulations used to pin the oracle (test code only).

Neither function here calls the oracle; each restates the scheme of the
paper in a different form:

* `plane_wave_E`: in a homogeneous periodic medium the scheme keeps the
  populations in the form g_i(x) = a_i exp(-i k.x) exactly, so K steps reduce
  to a 7-vector recurrence (collision on a, pull multiplies a_i by
  exp(+i k.e_i dx), reaction advances k by gamma G0 f_k dt).
* `dense_step_matrices`: the whole step as an explicit real matrix of size
  14N x 14N (real and imaginary parts) for a tiny lattice, built entry by
  entry from the collision, the boundary/membrane streaming rules and the
  reaction.
"""
from __future__ import annotations

import math

import numpy as np

EPS_D = 0.25
W = np.array([0.25] + [0.125] * 6)
E_DIR = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0],
                  [0, 0, 1], [0, 0, -1]])
OPP = [0, 2, 1, 4, 3, 6, 5]
# D2Q5 (Sec. 2.2, Eq. omega_i): eps_D = 1/3, rest weight 1/3, four moving 1/6
LATTICES = {0: (EPS_D, W, 7), 1: (1.0 / 3.0, np.array([1.0 / 3.0] + [1.0 / 6.0] * 4), 5)}


def _w(D, dt, dx, eps=EPS_D):
    return 1.0 / (0.5 + dt * D / (eps * dx * dx))


def dirichlet_mean(N, theta):
    """(1/N) sum_{n<N} exp(-i theta n)."""
    n = np.arange(N)
    return np.mean(np.exp(-1j * theta * n))


def plane_wave_E(n, dx, dt, D, T2, f, gG0, substeps=1, lattice=0):
    """Signal of the uniform-IC homogeneous periodic problem, all steps.
    With m sub-steps f holds m samples per step, each advancing the wave
    vector over dt/m.  lattice 1: D2Q5 on a single layer."""
    eps, Wl, nq = LATTICES[lattice]
    w = _w(D, dt, dx, eps)
    decay = 1.0 if math.isinf(T2) else math.exp(-dt / T2)
    a = Wl.astype(np.complex128)
    kvec = np.zeros(3)
    gG0 = np.asarray(gG0, np.float64)
    out = []
    K = len(f) // substeps
    for k in range(K + 1):
        geo = 1.0 + 0j
        for ax in range(3):
            geo *= dirichlet_mean(n[ax], kvec[ax] * dx)
        out.append(a.sum() * geo)
        if k == K:
            break
        ah = a - w * (a - Wl * a.sum())
        a = ah * np.exp(1j * (E_DIR[:nq] @ kvec) * dx) * decay
        for j in range(substeps):
            kvec = kvec + gG0 * f[k * substeps + j] * (dt / substeps)
    return np.array(out)


def _cblock(c, conj=False):
    cr, ci = c.real, c.imag
    if conj:
        return np.array([[cr, ci], [ci, -cr]])
    return np.array([[cr, -ci], [ci, cr]])


def dense_step_matrices(comp, comp_phase, bc, dx, dt, D, T2, kappa, f, gG0, scheme=0,
                        lattice=0, factors=False):
    """Real step matrices A_k (one per step) for a tiny lattice.

    scheme 1: classical LBM, the reaction term dt w_i R M inside the
    collision and no reaction split.

    factors=True returns each step as its factors (applied right to left:
    collision, streaming, reaction) instead of their product.

    State vector: index part*7N + i*N + s, part 0 = Re, 1 = Im, s the site
    index with x fastest.  Mirror faces use the paper's rule for gradients
    normal or parallel to the face only.
    """
    eps, Wl, nq = LATTICES[lattice]
    comp = np.asarray(comp)
    n2, n1, n0 = comp.shape
    n = (n0, n1, n2)
    N = n0 * n1 * n2
    S7 = nq * N

    def sidx(j):
        return j[0] + n0 * (j[1] + n1 * j[2])

    ph = np.asarray(comp_phase)[comp.reshape(-1)]
    w = np.array([_w(D[p], dt, dx, eps) for p in ph])
    dec = np.array([1.0 if math.isinf(T2[p]) else math.exp(-dt / T2[p]) for p in ph])
    # collision (acts identically on Re and Im)
    C = np.zeros((S7, S7))
    for s in range(N):
        for i in range(nq):
            C[i * N + s, i * N + s] += 1.0 - w[s]
            for j in range(nq):
                C[i * N + s, j * N + s] += w[s] * Wl[i]
    Cr = np.kron(np.eye(2), C)
    inv_t2 = np.array([0.0 if math.isinf(T2[p]) else 1.0 / T2[p] for p in ph])
    mats = []
    F = 0.0
    gG0 = np.asarray(gG0, np.float64)
    for k in range(len(f)):
        S = np.zeros((2 * S7, 2 * S7))

        def add(dst, src, c, conj=False, scale=1.0):
            blk = scale * _cblock(c, conj)
            for pd in range(2):
                for ps in range(2):
                    S[pd * S7 + dst, ps * S7 + src] += blk[pd, ps]

        for s in range(N):
            j = (s % n0, (s // n0) % n1, s // (n0 * n1))
            cx = comp.reshape(-1)[s]
            for i in range(nq):
                src = [j[a] - E_DIR[i][a] for a in range(3)]
                crossed = [a for a in range(3) if not 0 <= src[a] < n[a]]
                terms = []      # (source flat index, coefficient, conj)
                if not crossed:
                    cs = comp.reshape(-1)[sidx(src)]
                    terms.append((i * N + sidx(src), 1.0 + 0j, False))
                else:
                    a = crossed[0]
                    if bc[a] == 0:
                        wsrc = list(src)
                        wsrc[a] %= n[a]
                        phi = n[a] * dx * gG0[a] * F
                        c = np.exp(1j * phi) if src[a] < 0 else np.exp(-1j * phi)
                        cs = comp.reshape(-1)[sidx(wsrc)]
                        terms.append((i * N + sidx(wsrc), c, False))
                    else:
                        cs = cx
                        ib = OPP[i]          # i is along axis a here
                        if gG0[a] != 0.0:
                            xn = j[a] * dx
                            xm = (j[a] - 1) * dx if src[a] < 0 else (j[a] + 1) * dx
                            th = gG0[a] * (xn + xm) * F
                            terms.append((ib * N + s, np.exp(-1j * th), True))
                        else:
                            terms.append((ib * N + s, 1.0 + 0j, False))
                kap = kappa[comp_phase[cx], comp_phase[cs]]
                if cs != cx and not math.isinf(kap):
                    if kap == 0.0:
                        t, r = 0.0, 1.0
                    else:
                        P = eps * dx / (2.0 * kap * dt)
                        t, r = 1.0 / (1.0 + P), P / (1.0 + P)
                    for (src_i, c, cj) in terms:
                        add(i * N + s, src_i, c, cj, t)
                    add(i * N + s, OPP[i] * N + s, 1.0 + 0j, False, r)
                else:
                    for (src_i, c, cj) in terms:
                        add(i * N + s, src_i, c, cj)
        if scheme == 1:
            # collision with dt w_i R M, R = -i (x.gG0) f_k - 1/T2
            Ck = Cr.copy()
            for s_ in range(N):
                j = (s_ % n0, (s_ // n0) % n1, s_ // (n0 * n1))
                xg = sum(gG0[a] * j[a] * dx for a in range(3))
                Rc = (-1j * xg * f[k] - inv_t2[s_]) * dt
                for i in range(nq):
                    for jj in range(nq):
                        blk = Wl[i] * _cblock(Rc)
                        for pd in range(2):
                            for ps in range(2):
                                Ck[pd * S7 + i * N + s_, ps * S7 + jj * N + s_] += blk[pd, ps]
            mats.append((S, Ck) if factors else S @ Ck)
            F += f[k] * dt
            continue
        # reaction
        R = np.zeros((2 * S7, 2 * S7))
        for s in range(N):
            j = (s % n0, (s // n0) % n1, s // (n0 * n1))
            xg = sum(gG0[a] * j[a] * dx for a in range(3))
            c = np.exp(-1j * xg * f[k] * dt) * dec[s]
            blk = _cblock(c)
            for i in range(nq):
                for pd in range(2):
                    for ps in range(2):
                        R[pd * S7 + i * N + s, ps * S7 + i * N + s] = blk[pd, ps]
        mats.append((R, S, Cr) if factors else R @ S @ Cr)
        F += f[k] * dt
    return mats


def dense_run(mats, N, lattice=0):
    """E_k for the uniform initial state, all steps."""
    _, Wl, nq = LATTICES[lattice]
    S7 = nq * N
    v = np.zeros(2 * S7)
    for i in range(nq):
        v[i * N:(i + 1) * N] = Wl[i]
    out = []
    for k in range(len(mats) + 1):
        out.append((v[:S7].sum() + 1j * v[S7:].sum()) / N)
        if k < len(mats):
            m = mats[k]
            if isinstance(m, tuple):
                for fac in reversed(m):
                    v = fac @ v
            else:
                v = m @ v
    return np.array(out)


def step_average_pgse(delta, Delta, dt, K):
    """Per-step averages of the PGSE effective waveform (+1 on [0, delta),
    -1 on [Delta, Delta + delta)) over [k dt, (k+1) dt)."""
    t0 = np.arange(K) * dt
    t1 = t0 + dt

    def cover(a, b):
        return np.clip(np.minimum(t1, b) - np.maximum(t0, a), 0.0, None) / dt

    # rounded so that fully covered steps are exactly +-1 and runs of equal
    # values can share one exponential in `slab_fv_reference`
    return np.round(cover(0.0, delta) - cover(Delta, Delta + delta), 12)


def slab_fv_reference(x_if, D, T2, kappa_if, gG, f, dt, x_eval, cells):
    """Bloch-Torrey solution M(x_eval, K dt) in 1D, M(x, 0) = 1, by finite
    volumes and exact matrix exponentials (an independent discretisation).

    Compartment c spans [x_if[c], x_if[c+1]] with diffusivity D[c] and
    relaxation T2[c]; the two outer ends are impermeable, interior interface
    c+1 has permeability kappa_if[c] (flux kappa (M_right - M_left)).  The
    gradient term is -i gG x f(t) M with f constant on each step.  `cells`
    cells per compartment; second order in the cell width.
    """
    import scipy.linalg as sla

    nc = len(D)
    xs, hs, cid = [], [], []
    for c in range(nc):
        h = (x_if[c + 1] - x_if[c]) / cells
        xs.append(x_if[c] + h * (np.arange(cells) + 0.5))
        hs.append(np.full(cells, h))
        cid.append(np.full(cells, c))
    xs, hs, cid = np.concatenate(xs), np.concatenate(hs), np.concatenate(cid)
    n = len(xs)
    Ldiff = np.zeros((n, n))
    for k in range(n - 1):
        cl, cr = cid[k], cid[k + 1]
        if cl == cr:
            cond = D[cl] / hs[k]                       # h equal within a compartment
        else:
            kap = kappa_if[cl]
            if kap == 0.0:
                continue
            cond = 1.0 / (hs[k] / (2 * D[cl]) + 1.0 / kap + hs[k + 1] / (2 * D[cr]))
        Ldiff[k, k] -= cond / hs[k]
        Ldiff[k, k + 1] += cond / hs[k]
        Ldiff[k + 1, k + 1] -= cond / hs[k + 1]
        Ldiff[k + 1, k] += cond / hs[k + 1]
    relax = np.array([0.0 if math.isinf(T2[c]) else 1.0 / T2[c] for c in cid])
    M = np.ones(n, np.complex128)
    # runs of equal waveform values share one exponential
    k = 0
    f = np.asarray(f, np.float64)
    while k < len(f):
        e = k
        while e < len(f) and f[e] == f[k]:
            e += 1
        A = Ldiff - np.diag(relax) - 1j * gG * f[k] * np.diag(xs)
        M = sla.expm(A * ((e - k) * dt)) @ M
        k = e
    # linear interpolation between cell centres of the same compartment
    out = np.zeros(len(x_eval), np.complex128)
    for t, x in enumerate(x_eval):
        c = int(np.searchsorted(x_if, x, side="right") - 1)
        idx = np.nonzero(cid == c)[0]
        xc = xs[idx]
        j = int(np.clip(np.searchsorted(xc, x) - 1, 0, len(xc) - 2))
        w_ = (x - xc[j]) / (xc[j + 1] - xc[j])
        out[t] = (1 - w_) * M[idx[j]] + w_ * M[idx[j + 1]]
    return out
