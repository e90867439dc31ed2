"""FP64 CPU oracle for the hybrid lattice Boltzmann Bloch-Torrey scheme.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (paper_1907_00908_amd); both only consume the seeded inputs of the
`workloads` package.

`simulate` runs the scheme one gradient direction at a time in the paper's
buffer-row formulation (see oracle.c for the steps and the readings of the
paper they take).  For a mirrored axis and a gradient that is neither normal
nor parallel to its faces the paper gives no rule (Sec. 2.4.4 sets that
case aside as needing a more involved rotation); the oracle then takes the plain
definition of a mirroring boundary -- the REV reflected across the face,
i.e. the medium doubled along that axis and tiled periodically -- and runs
the modified periodic condition on the doubled domain, averaging the signal
over the original REV only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_oracle.so")
_lib = None

PERIODIC, MIRROR = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_run.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P, P,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   P, P, P, P, P, P, P, P, P, ctypes.c_int32, ctypes.c_int32,
                                   P, P, ctypes.c_int32, ctypes.c_int32, P]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_memb_coeffs.argtypes = [ctypes.c_double] * 3 + [P]
        lib.oracle_memb_coeffs.restype = None
        lib.oracle_tau.argtypes = [ctypes.c_double] * 3 + [ctypes.c_int32]
        lib.oracle_tau.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _run_core(comp, comp_phase, n_phase, bc, off, dx, dt, D, T2, kappa, f, gG0,
              elo, ehi, threads, want_M, scheme=0, link_delta=None, tile=None, substeps=1,
              lattice=0, link_normal=None):
    lib = _load()
    comp = np.ascontiguousarray(comp, dtype=np.uint32)
    n2, n1, n0 = comp.shape
    n = np.array([n0, n1, n2], np.int32)
    cp = np.ascontiguousarray(comp_phase, dtype=np.uint8)
    bc = np.ascontiguousarray(bc, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.float64)
    D = np.ascontiguousarray(D, dtype=np.float64)
    T2 = np.ascontiguousarray(T2, dtype=np.float64)
    kappa = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
    f = np.ascontiguousarray(f, dtype=np.float64)
    gG0 = np.ascontiguousarray(gG0, dtype=np.float64)
    elo = np.ascontiguousarray(elo, dtype=np.int32)
    ehi = np.ascontiguousarray(ehi, dtype=np.int32)
    if len(f) % substeps:
        raise ValueError("len(f) must be a multiple of substeps")
    K = len(f) // substeps
    E = np.zeros(2 * (K + 1), np.float64)
    M = np.zeros(2 * comp.size, np.float64) if want_M else None
    if link_delta is not None:
        link_delta = np.ascontiguousarray(link_delta, dtype=np.float64)
        if link_delta.shape != (3,) + comp.shape:
            raise ValueError("link_delta must have shape (3, n2, n1, n0)")
    if link_normal is not None:
        if link_delta is None:
            raise ValueError("link_normal needs link_delta")
        link_normal = np.ascontiguousarray(link_normal, dtype=np.float64)
        if link_normal.shape != (3, 3) + comp.shape:
            raise ValueError("link_normal must have shape (3, 3, n2, n1, n0)")
    tile = None if tile is None else np.ascontiguousarray(tile, dtype=np.int32)
    rc = lib.oracle_run(_ptr(n), _ptr(comp), _ptr(cp), len(cp), int(n_phase), _ptr(bc),
                        _ptr(off), float(dx), float(dt), K, _ptr(D), _ptr(T2),
                        _ptr(kappa), _ptr(f), _ptr(gG0), _ptr(elo), _ptr(ehi),
                        _ptr(E), _ptr(M) if want_M else None, int(threads), int(scheme),
                        _ptr(link_delta) if link_delta is not None else None,
                        _ptr(tile) if tile is not None else None, int(substeps),
                        int(lattice), _ptr(link_normal) if link_normal is not None else None)
    if rc == -2:
        raise NotImplementedError("oblique gradient on a mirrored axis")
    if rc != 0:
        raise ValueError(f"oracle_run rejected its input (code {rc})")
    Ec = E[0::2] + 1j * E[1::2]
    Mc = (M[0::2] + 1j * M[1::2]).reshape(comp.shape) if want_M else None
    return Ec, Mc


def memb_coeffs(delta: float, kappa_dt: float, epsd_dx: float) -> np.ndarray:
    """{A_1, A_2, A_3, B_1, B_2, B_3} of the theta = 0 membrane condition
    (Eqs. B4a-B4c) for a membrane at `delta` (units of dx) from the
    receiving node."""
    out = np.zeros(6)
    _load().oracle_memb_coeffs(float(delta), float(kappa_dt), float(epsd_dx), _ptr(out))
    return out


D3Q7, D2Q5 = 0, 1


def tau(D: float, dt: float, dx: float, lattice: int = D3Q7) -> float:
    """Relaxation time the oracle uses (Eq. tau_def; eps_D = 1/4 for D3Q7,
    1/3 for D2Q5)."""
    return float(_load().oracle_tau(D, dt, dx, int(lattice)))


def needs_doubling(bc, gG0) -> bool:
    """True when a mirrored axis sees an oblique gradient (paper silent)."""
    g = np.asarray(gG0, dtype=np.float64)
    nz = g != 0.0
    for a in range(3):
        if bc[a] == MIRROR and nz[a] and nz.sum() > 1:
            return True
    return False


HYBRID, CLASSICAL = 0, 1


def simulate(comp, comp_phase, n_phase, bc, dx, dt, D, T2, kappa, f, gG0,
             threads: int = 1, mirror: str = "auto", want_M: bool = True,
             scheme: int = HYBRID, link_delta=None, substeps: int = 1,
             lattice: int = D3Q7, link_normal=None):
    """Run the scheme for one gradient vector.

    comp (n2, n1, n0) compartment ids, comp_phase [C], bc[3] (0 periodic,
    1 mirror), D/T2 [P], kappa [P, P], f [K], gG0 [3].
    mirror: "paper" uses the paper's buffer rule (axis-aligned gradients
    only), "double" reflects and doubles every mirrored axis and runs
    periodic, "auto" picks "paper" when it applies.
    scheme: HYBRID (the paper's split scheme) or CLASSICAL (reaction term in
    the collision, Eq. A12).  The conjugate mirror rule relies on an exact
    symmetry of the split reaction; with the classical scheme a mirrored
    axis with a gradient component always runs on the doubled domain.
    link_delta: None (half-link membranes at mid-link) or (3, n2, n1, n0)
    membrane positions along the +x, +y, +z links from each node (units of
    dx) for the general theta = 0 membrane condition (oracle.c).
    link_normal: None, or (3, 3, n2, n1, n0) unit normals of the membrane on
    each link (axis, component; either orientation) for the general
    condition at any angle (oracle.c; needs link_delta).
    substeps: m reaction sub-steps per step; f then holds K*m samples at
    dt/m (hybrid scheme only).
    lattice: D3Q7, or D2Q5 on a single layer (n2 = 1, gG0[2] = 0; the z
    axis is not a lattice axis and its boundary kind is ignored).
    Returns E [K+1] complex and M at t_K, complex (n2, n1, n0).
    """
    comp = np.asarray(comp)
    bc = [int(b) for b in bc]
    if lattice == D2Q5:
        bc[2] = PERIODIC
    if mirror == "auto":
        g = np.asarray(gG0, np.float64)
        classical_mirror = scheme == CLASSICAL and any(
            bc[a] == MIRROR and g[a] != 0.0 for a in range(3))
        mirror = "double" if (needs_doubling(bc, gG0) or classical_mirror) else "paper"
    if mirror == "paper" or MIRROR not in bc:
        n2, n1, n0 = comp.shape
        ld = None if link_delta is None else np.asarray(link_delta, np.float32)
        ln = None if link_normal is None else np.asarray(link_normal, np.float32)
        return _run_core(comp, comp_phase, n_phase, bc, [0.0, 0.0, 0.0], dx, dt,
                         D, T2, kappa, f, gG0, [0, 0, 0], [n0, n1, n2], threads, want_M,
                         scheme, ld, None, substeps, lattice, ln)
    if mirror != "double":
        raise ValueError("mirror must be 'auto', 'paper' or 'double'")
    # reflect the REV across the lower face of every mirrored axis: the
    # extended axis holds the mirror image at coordinates -N..-1 and the REV
    # at 0..N-1, and the doubled medium is tiled periodically
    ext = comp
    # positions are single precision on input (as the HIP library stores
    # them); complements 1 - d of the reflected copies are exact in FP64
    ld = None if link_delta is None else np.asarray(link_delta, np.float32).astype(np.float64)
    ln = None if link_normal is None else np.asarray(link_normal, np.float32).astype(np.float64)
    off = [0.0, 0.0, 0.0]
    lo = [0, 0, 0]
    hi = list(comp.shape[::-1])
    tile = list(comp.shape[::-1])
    for a in range(3):
        if bc[a] != MIRROR:
            continue
        ax = 2 - a                   # numpy axis of lattice axis a
        na = comp.shape[ax]
        ext = np.concatenate([np.flip(ext, axis=ax), ext], axis=ax)
        if ld is not None:
            # the image holds node n-1-k at k; its link k -> k+1 is the
            # original link n-2-k -> n-1-k seen from the other end
            img = np.flip(ld, axis=ax + 1).copy()
            sl = [slice(None)] * 4
            sl[0] = a
            sl[ax + 1] = slice(0, na - 1)
            src = [slice(None)] * 4
            src[0] = a
            src[ax + 1] = slice(1, na)
            img[tuple(sl)] = 1.0 - np.flip(ld, axis=ax + 1)[tuple(src)]
            sl[ax + 1] = slice(na - 1, na)
            img[tuple(sl)] = 0.5     # image of node 0 -> node 0: no membrane
            ld = np.concatenate([img, ld], axis=ax + 1)
        if ln is not None:
            # the reflected copy: normals mirrored in axis a (component a
            # negated), links indexed as for the positions above
            imn = np.flip(ln, axis=ax + 2).copy()
            imn[:, a] *= -1.0
            src = imn.copy()
            dst = [slice(None)] * 5
            dst[0] = a
            dst[ax + 2] = slice(0, na - 1)
            srs = [slice(None)] * 5
            srs[0] = a
            srs[ax + 2] = slice(1, na)
            imn[tuple(dst)] = src[tuple(srs)]
            # the image of node 0 -> node 0 joins one compartment: not read
            dst[ax + 2] = slice(na - 1, na)
            imn[tuple(dst)] = 0.0
            ln = np.concatenate([imn, ln], axis=ax + 2)
        off[a] = -float(na)
        lo[a], hi[a] = na, 2 * na
    bce = [PERIODIC] * 3
    E, M = _run_core(ext, comp_phase, n_phase, bce, off, dx, dt, D, T2, kappa, f,
                     gG0, lo, hi, threads, want_M, scheme, ld, tile, substeps, lattice, ln)
    if want_M:
        M = M[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]].copy()
    return E, M


def simulate_config(cfg: dict, q=None, threads: int = 1, mirror: str = "auto",
                    want_M: bool = False, scheme: int = None):
    """Run every q-sample (or the listed ones) of a workloads config."""
    qs = range(len(cfg["gG0"])) if q is None else q
    Es, Ms = [], []
    for i in qs:
        g = cfg["geoms"][int(cfg["q_geom"][i])]
        E, M = simulate(g.comp, g.comp_phase, g.n_phase, cfg["bc"], cfg["dx"], cfg["dt"],
                        cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"], cfg["gG0"][i],
                        threads=threads, mirror=mirror, want_M=want_M,
                        scheme=cfg.get("scheme", HYBRID) if scheme is None else scheme,
                        link_delta=getattr(g, "link_delta", None),
                        substeps=cfg.get("substeps", 1), lattice=cfg.get("lattice", D3Q7),
                        link_normal=getattr(g, "link_normal", None))
        Es.append(E)
        Ms.append(M)
    return np.array(Es), Ms
