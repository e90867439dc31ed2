"""Seeded compartment-label volumes (inputs only).

A geometry is a volume of compartment ids (uint32, array shape (n2, n1, n0),
x fastest) plus a table mapping each compartment to a phase (uint8).  A
phase carries one set of material parameters (D, T2); every lattice link
joining two different compartments carries a membrane whose permeability is
looked up by the pair of phases.  This is how the paper's piecewise-uniform
media with thin membranes (Sec. 2.1, Fig. 1) and its cell-to-cell membranes
in histology-derived domains (Sec. 3.6) are represented on a label volume.

Lattice node j along an axis sits at x = j*dx; a box of n nodes has length
L = n*dx (the node at n is the periodic image of node 0, Sec. 2.4.3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Geometry:
    comp: np.ndarray            # uint32, shape (n2, n1, n0)
    comp_phase: np.ndarray      # uint8, shape (C,)
    n_phase: int
    dx: float
    info: dict = field(default_factory=dict)
    # optional membrane positions on the links, (3, n2, n1, n0) float32 (see
    # `link_delta`); None: every membrane at mid-link
    link_delta: np.ndarray | None = None

    @property
    def shape_xyz(self):
        n2, n1, n0 = self.comp.shape
        return (n0, n1, n2)

    @property
    def n_sites(self) -> int:
        return int(self.comp.size)

    def phase_volume(self) -> np.ndarray:
        return self.comp_phase[self.comp]

    def phase_fractions(self) -> np.ndarray:
        pv = self.phase_volume()
        return np.bincount(pv.ravel(), minlength=self.n_phase) / pv.size


def _shape3(n):
    if np.isscalar(n):
        return (int(n),) * 3
    n = tuple(int(v) for v in n)
    if len(n) != 3:
        raise ValueError("n must be an int or (n0, n1, n2)")
    return n


def uniform(n, dx: float) -> Geometry:
    """Single compartment, single phase."""
    n0, n1, n2 = _shape3(n)
    comp = np.zeros((n2, n1, n0), dtype=np.uint32)
    return Geometry(comp, np.zeros(1, np.uint8), 1, float(dx),
                    {"kind": "uniform"})


def slabs(n, dx: float, cuts_x, phases=None) -> Geometry:
    """Slabs stacked along x: compartment c covers cuts_x[c-1] <= j0 < cuts_x[c].

    With a periodic x axis the last and first slab are also separated by the
    wrap link; a single cut list [] gives one slab whose only membrane is the
    wrap link when the two sides are given different compartments.
    """
    n0, n1, n2 = _shape3(n)
    cuts = [0] + sorted(int(c) for c in cuts_x) + [n0]
    comp1 = np.zeros(n0, dtype=np.uint32)
    for c in range(len(cuts) - 1):
        comp1[cuts[c]:cuts[c + 1]] = c
    comp = np.broadcast_to(comp1[None, None, :], (n2, n1, n0)).copy()
    nc = len(cuts) - 1
    ph = np.zeros(nc, np.uint8) if phases is None else np.asarray(phases, np.uint8)
    return Geometry(comp, ph, int(ph.max()) + 1, float(dx), {"kind": "slabs"})


def _relax_disks(rng, L, radii, gap, periodic, max_iter=20000):
    """Random positions, then push overlapping disks apart until every pair
    is separated by at least `gap` (or give up and drop offenders)."""
    n = len(radii)
    pos = rng.uniform(0.0, 1.0, size=(n, 2)) * np.asarray(L)
    r = np.asarray(radii)
    need = r[:, None] + r[None, :] + gap
    np.fill_diagonal(need, 0.0)
    Lv = np.asarray(L, dtype=np.float64)
    for _ in range(max_iter):
        d = pos[None, :, :] - pos[:, None, :]          # j - i
        if periodic:
            d -= Lv * np.round(d / Lv)
        dist = np.sqrt(np.sum(d * d, axis=-1))
        np.fill_diagonal(dist, np.inf)
        ov = need - dist
        np.fill_diagonal(ov, -1.0)
        if ov.max() <= 1e-7:
            return pos, np.ones(n, bool)
        m = ov > 0
        with np.errstate(invalid="ignore", divide="ignore"):
            u = d / dist[..., None]
        u[~m] = 0.0
        push = 0.5 * (ov * m)[..., None] * 1.05 * u
        # i moves away from j: -push; j receives +push from i
        disp = -push.sum(axis=1)
        pos += disp
        if periodic:
            pos %= Lv
        else:
            pos = np.clip(pos, 0.0, Lv)
    # could not separate everything: drop disks that still overlap
    keep = np.ones(n, bool)
    d = pos[None, :, :] - pos[:, None, :]
    if periodic:
        d -= Lv * np.round(d / Lv)
    dist = np.sqrt(np.sum(d * d, axis=-1))
    np.fill_diagonal(dist, np.inf)
    ov = need - dist
    for i in np.argsort(r):                             # smallest first
        if not keep[i]:
            continue
        if np.any((ov[i] > 1e-7) & keep):
            keep[i] = False
    return pos, keep


def _raster_disks(n0, n1, dx, pos, radii, periodic, ids):
    """2D label image (n1, n0): site (j0, j1) at (j0*dx, j1*dx)."""
    img = np.zeros((n1, n0), dtype=np.uint32)
    L = np.array([n0 * dx, n1 * dx])
    for (cx, cy), r, cid in zip(pos, radii, ids):
        shifts = [(0.0, 0.0)]
        if periodic:
            shifts = [(sx * L[0], sy * L[1]) for sx in (-1, 0, 1) for sy in (-1, 0, 1)]
        for sx, sy in shifts:
            x0, y0 = cx + sx, cy + sy
            i0 = max(0, int(math.floor((x0 - r) / dx)))
            i1 = min(n0 - 1, int(math.ceil((x0 + r) / dx)))
            k0 = max(0, int(math.floor((y0 - r) / dx)))
            k1 = min(n1 - 1, int(math.ceil((y0 + r) / dx)))
            if i0 > i1 or k0 > k1:
                continue
            xs = np.arange(i0, i1 + 1) * dx - x0
            ys = np.arange(k0, k1 + 1) * dx - y0
            inside = (xs[None, :] ** 2 + ys[:, None] ** 2) < r * r
            sub = img[k0:k1 + 1, i0:i1 + 1]
            sub[inside] = cid
    return img


def cylinders_z(n, dx: float, seed: int, vf_target: float = 0.6,
                gamma_shape: float = 4.0, mean_r: float = 1.0,
                periodic: bool = True, gap: float | None = None) -> Geometry:
    """Parallel cylinders along z in an extracellular matrix.

    Radii ~ Gamma(shape, mean) redrawn below 2*dx; disks are drawn until
    their area reaches the target, placed at random and relaxed apart so that
    surfaces are at least `gap` (default dx) apart, largest first when some
    have to be dropped.  Phase 0 = extracellular, phase 1 = intracellular;
    each cylinder is its own compartment (ids 1..).  With gap >= dx no two
    cylinders share a lattice link, so every membrane link is in/ex.
    """
    n0, n1, n2 = _shape3(n)
    rng = np.random.default_rng(seed)
    gap = dx if gap is None else float(gap)
    L = (n0 * dx, n1 * dx)
    target = vf_target * L[0] * L[1]
    radii = []
    area = 0.0
    scale = mean_r / gamma_shape
    while area < target:
        r = rng.gamma(gamma_shape, scale)
        while r < 2.0 * dx:
            r = rng.gamma(gamma_shape, scale)
        radii.append(r)
        area += math.pi * r * r
    radii = np.sort(np.asarray(radii))[::-1]
    # placement always uses periodic distances; a non-periodic (mirror) box
    # then simply cuts the cylinders that cross its faces
    pos, keep = _relax_disks(rng, L, radii, gap, True)
    pos, radii = pos[keep], radii[keep]
    ids = np.arange(1, len(radii) + 1, dtype=np.uint32)
    img = _raster_disks(n0, n1, dx, pos, radii, periodic, ids)
    comp = np.broadcast_to(img[None, :, :], (n2, n1, n0)).copy()
    comp_phase = np.ones(len(radii) + 1, np.uint8)
    comp_phase[0] = 0
    g = Geometry(comp, comp_phase, 2, float(dx),
                 {"kind": "cylinders_z", "seed": seed, "n_cyl": int(len(radii)),
                  "vf_target": vf_target, "periodic": periodic})
    # analytic surfaces: (x-c)^T A (x-c) < 1 inside, A_zz = 0 for a z-cylinder
    g.info["shapes"] = {"periodic": (periodic, periodic, False),
                        "items": [(int(cid), np.array([cx, cy, 0.0]),
                                   np.diag([1.0 / (r * r), 1.0 / (r * r), 0.0]))
                                  for (cx, cy), r, cid in zip(pos, radii, ids)]}
    g.info["vf_voxel"] = float(g.phase_fractions()[1])
    return g


def cylinders_spheres(n, dx: float, seed: int, vf_cyl: float = 0.4,
                      vf_sph: float = 0.15, r_sph=(2.0, 6.0)) -> Geometry:
    """Periodic z-cylinders (as `cylinders_z`) to vf_cyl, then spheres with
    radius ~ U(r_sph) placed without mutual overlap until they add vf_sph;
    a sphere replaces whatever it covers.  Phases: 0 extracellular,
    1 cylinder interior, 2 sphere interior."""
    n0, n1, n2 = _shape3(n)
    base = cylinders_z((n0, n1, n2), dx, seed, vf_target=vf_cyl, periodic=True)
    rng = np.random.default_rng(seed + 7919)
    comp = base.comp.copy()
    nc = len(base.comp_phase)
    L = np.array([n0, n1, n2], dtype=np.float64) * dx
    target = vf_sph * float(np.prod(L))
    placed = []
    vol = 0.0
    tries = 0
    while vol < target and tries < 200000:
        tries += 1
        r = rng.uniform(*r_sph)
        c = rng.uniform(0.0, 1.0, 3) * L
        ok = True
        for (c2, r2) in placed:
            d = c - c2
            d -= L * np.round(d / L)
            if np.sqrt(np.dot(d, d)) < r + r2 + dx:
                ok = False
                break
        if ok:
            placed.append((c, r))
            vol += 4.0 / 3.0 * math.pi * r ** 3
    ax = [np.arange(m) * dx for m in (n0, n1, n2)]
    for s, (c, r) in enumerate(placed):
        cid = nc + s
        sl, coords = [], []
        for a in range(3):
            lo = int(math.floor((c[a] - r) / dx))
            hi = int(math.ceil((c[a] + r) / dx))
            idx = np.arange(lo, hi + 1)
            coords.append(idx * dx - c[a])
            sl.append(np.mod(idx, (n0, n1, n2)[a]))
        inside = (coords[2][:, None, None] ** 2 + coords[1][None, :, None] ** 2
                  + coords[0][None, None, :] ** 2) < r * r
        zz, yy, xx = np.nonzero(inside)
        comp[sl[2][zz], sl[1][yy], sl[0][xx]] = cid
    comp_phase = np.concatenate([base.comp_phase,
                                 np.full(len(placed), 2, np.uint8)])
    g = Geometry(comp, comp_phase, 3, float(dx),
                 {"kind": "cylinders_spheres", "seed": seed,
                  "n_cyl": base.info["n_cyl"], "n_sph": len(placed)})
    g.info["shapes"] = {"periodic": (True, True, True),
                        "items": list(base.info["shapes"]["items"])
                        + [(nc + s, c.copy(), np.eye(3) / (r * r))
                           for s, (c, r) in enumerate(placed)]}
    fr = g.phase_fractions()
    g.info["vf_voxel"] = [float(v) for v in fr]
    return g


def _rand_rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ellipsoid_cells(n, dx: float, seed: int, vf_target: float = 0.5,
                    semi=(3.0, 8.0), max_tries: int = 20000) -> Geometry:
    """Randomly oriented ellipsoidal cells with a concentric nucleus of half
    the semi-axes, periodic box, at least one empty voxel between cells.

    Phases: 0 extracellular, 1 cytoplasm, 2 nucleus.  Cell c has cytoplasm
    compartment 2c+1 and nucleus compartment 2c+2.
    """
    n0, n1, n2 = _shape3(n)
    dims = (n0, n1, n2)
    rng = np.random.default_rng(seed)
    comp = np.zeros((n2, n1, n0), dtype=np.uint32)
    occ = np.zeros((n2, n1, n0), dtype=bool)      # cells dilated by one voxel
    L = np.array(dims, dtype=np.float64) * dx
    target = vf_target * comp.size
    filled = 0
    ncell = 0
    tries = 0
    shapes = []
    while filled < target and tries < max_tries:
        tries += 1
        ax = rng.uniform(semi[0], semi[1], 3)
        R = _rand_rotation(rng)
        c = rng.uniform(0.0, 1.0, 3) * L
        # quick rejection: centre voxel already taken
        ci = [int(round(c[a] / dx)) % dims[a] for a in range(3)]
        if occ[ci[2], ci[1], ci[0]]:
            continue
        A = R @ np.diag(1.0 / ax ** 2) @ R.T        # x^T A x < 1 inside
        ext = np.sqrt(np.diag(np.linalg.inv(A)))     # bounding half-widths
        idx, rel = [], []
        for a in range(3):
            lo = int(math.floor((c[a] - ext[a]) / dx)) - 1
            hi = int(math.ceil((c[a] + ext[a]) / dx)) + 1
            j = np.arange(lo, hi + 1)
            idx.append(np.mod(j, dims[a]))
            rel.append(j * dx - c[a])
        X = rel[0][None, None, :]
        Y = rel[1][None, :, None]
        Z = rel[2][:, None, None]
        qf = (A[0, 0] * X * X + A[1, 1] * Y * Y + A[2, 2] * Z * Z
              + 2 * A[0, 1] * X * Y + 2 * A[0, 2] * X * Z + 2 * A[1, 2] * Y * Z)
        inside = qf < 1.0
        if not inside.any():
            continue
        sub = np.ix_(idx[2], idx[1], idx[0])
        if np.any(occ[sub] & inside):
            continue
        nuc = qf < 0.25                                # half semi-axes
        block = comp[sub]
        block[inside] = 2 * ncell + 1
        block[nuc] = 2 * ncell + 2
        comp[sub] = block
        dil = inside.copy()
        for a in range(3):
            dil |= np.roll(inside, 1, axis=a) | np.roll(inside, -1, axis=a)
        o = occ[sub]
        o |= dil
        occ[sub] = o
        filled += int(inside.sum())
        shapes.append((2 * ncell + 1, c.copy(), A))
        shapes.append((2 * ncell + 2, c.copy(), 4.0 * A))
        ncell += 1
    comp_phase = np.zeros(2 * ncell + 1, np.uint8)
    comp_phase[1::2] = 1
    comp_phase[2::2] = 2
    g = Geometry(comp, comp_phase, 3, float(dx),
                 {"kind": "ellipsoid_cells", "seed": seed, "n_cell": ncell,
                  "shapes": {"periodic": (True, True, True), "items": shapes}})
    g.info["vf_voxel"] = [float(v) for v in g.phase_fractions()]
    return g


def tile_xy(g: Geometry, rx: int, ry: int) -> Geometry:
    """rx x ry periodic copies of a geometry that is periodic in x and y
    (compartment ids kept: a cell cut by the tile border continues in the
    next copy as the same compartment)."""
    comp = np.tile(g.comp, (1, ry, rx))
    info = {"kind": g.info.get("kind", "?") + "_tiled", "tile_of": (g, rx, ry)}
    return Geometry(comp, g.comp_phase.copy(), g.n_phase, g.dx, info)


def _link_crossings(g: Geometry):
    """Crossing positions and unit normals of the analytic surfaces on the
    lattice links (see link_delta and link_normal)."""
    n2, n1, n0 = g.comp.shape
    dims = (n0, n1, n2)
    out = np.full((3, n2, n1, n0), 0.5, np.float32)
    nrm = np.zeros((3, 3, n2, n1, n0), np.float32)
    for a in range(3):
        nrm[a, a] = 1.0
    shp = g.info.get("shapes")
    if not shp:
        return out, nrm
    dx = g.dx
    L = np.array(dims, np.float64) * dx
    per = np.array(shp["periodic"], bool)
    items = shp["items"]
    ncomp = len(g.comp_phase)
    shape_of = np.full(ncomp, -1, np.int64)
    for k, (cid, _, _) in enumerate(items):
        shape_of[cid] = k
    C = np.array([it[1] for it in items], np.float64).reshape(-1, 3)
    A = np.array([it[2] for it in items], np.float64).reshape(-1, 3, 3)
    for a in range(3):
        nb = np.roll(g.comp, -1, axis=2 - a)             # comp of node j + e_a
        link = g.comp != nb
        if not per[a]:
            # the link beyond the last node is not a lattice link
            sl = [slice(None)] * 3
            sl[2 - a] = slice(dims[a] - 1, dims[a])
            link[tuple(sl)] = False
        z, y, x = np.nonzero(link)
        if len(x) == 0:
            continue
        p0 = np.stack([x, y, z], axis=1) * dx
        best = np.full(len(x), 0.5)
        bestn = np.zeros((len(x), 3))
        bestn[:, a] = 1.0
        found = np.zeros(len(x), bool)
        for side in (g.comp[z, y, x], nb[z, y, x]):
            k = shape_of[side]
            ok = k >= 0
            if not ok.any():
                continue
            kk = k[ok]
            c = C[kk]
            d = p0[ok] - c
            d = np.where(per[None, :], d - L * np.round(d / L), d)   # nearest image
            Ak = A[kk]
            Ad = np.einsum("nij,nj->ni", Ak, d)
            qa = dx * dx * Ak[:, a, a]
            qb = 2.0 * dx * Ad[:, a]
            qc = np.einsum("ni,ni->n", d, Ad) - 1.0
            q1 = qa + qb + qc
            in0, in1 = qc < 0.0, q1 < 0.0
            one = (in0 != in1) & (qa > 0.0)
            disc = np.sqrt(np.maximum(qb * qb - 4.0 * qa * qc, 0.0))
            with np.errstate(divide="ignore", invalid="ignore"):
                t = np.where(in0, (-qb + disc) / (2.0 * qa), (-qb - disc) / (2.0 * qa))
            # the surface (p - c).A(p - c) = 1 has the normal A (p - c)
            pc = d + np.where(np.isfinite(t), t, 0.0)[:, None] * dx * np.eye(3)[a][None, :]
            gn = np.einsum("nij,nj->ni", Ak, pc)
            gl = np.linalg.norm(gn, axis=1)
            use = one & ~found[ok] & (gl > 0.0)
            idx = np.nonzero(ok)[0][use]
            best[idx] = t[use]
            bestn[idx] = gn[use] / gl[use][:, None]
            found[idx] = True
        out[a, z, y, x] = np.clip(best, 1e-4, 1.0 - 1e-4).astype(np.float32)
        nrm[a, :, z, y, x] = bestn.astype(np.float32)   # advanced index first: (links, 3)
    return out, nrm


def link_delta(g: Geometry) -> np.ndarray:
    """Where each membrane cuts its lattice link, from the analytic surfaces
    the geometry was rasterised from.

    Returns float32 (3, n2, n1, n0): entry [a, j2, j1, j0] is the distance,
    in units of dx, from node j to the surface on the link j -> j + e_a (the
    last node of a periodic axis links to node 0).  Links that join two
    compartments get the crossing of the surface that has exactly one of the
    two nodes inside (clamped to [1e-4, 1 - 1e-4]); every other entry, and
    every entry of a geometry without analytic surfaces, is 0.5 (the
    mid-link position).
    """
    if "tile_of" in g.info:
        base, rx, ry = g.info["tile_of"]
        return np.tile(link_delta(base), (1, 1, ry, rx))
    return _link_crossings(g)[0]


def link_normal(g: Geometry) -> np.ndarray:
    """Unit normals of the analytic surfaces where they cut the lattice
    links (the gradient of the quadric at the crossing of link_delta).

    Returns float32 (3, 3, n2, n1, n0): entry [a, c, j2, j1, j0] is
    component c of the normal on the link j -> j + e_a, pointing out of the
    shape; links without a crossing (and geometries without analytic
    surfaces) get e_a, i.e. a membrane normal to the link."""
    if "tile_of" in g.info:
        base, rx, ry = g.info["tile_of"]
        return np.tile(link_normal(base), (1, 1, 1, ry, rx))
    if "link_normal" in g.info:
        return g.info["link_normal"]
    return _link_crossings(g)[1]


def angled_slabs_2d(n: int, dx: float, bounds, tan_phi=(1, 2), phases=None) -> Geometry:
    """Single-layer (n x n x 1) periodic box crossed by straight membranes
    along the lines x.nhat = s (mod P), nhat = (q, p)/sqrt(p^2 + q^2) for
    tan_phi = (p, q) (the normal makes the angle atan(p/q) with x), P the
    period of the pattern in the box (P = L / sqrt(p^2 + q^2), L = n dx).
    bounds: increasing positions s_0 < s_1 < ... in [0, P); compartment c
    spans [s_{c-1}, s_c) and compartment 0 the rest.  Carries the exact
    membrane positions of every link (link_delta)."""
    p, q = tan_phi
    nrm = math.hypot(p, q)
    nh = np.array([q / nrm, p / nrm])
    L = n * dx
    P = L / nrm
    b = np.asarray(bounds, np.float64)
    j = np.arange(n)
    X, Y = np.meshgrid(j * dx, j * dx)            # (n1, n0): Y rows, X columns

    def comp_at(s):
        s = np.mod(s, P)
        c = np.zeros(s.shape, np.uint32)
        for k in range(1, len(b)):
            c[(s >= b[k - 1]) & (s < b[k])] = k
        return c

    s0 = X * nh[0] + Y * nh[1]
    comp2 = comp_at(s0)
    comp = comp2[None, :, :].copy()
    nc = len(b)
    ph = np.arange(nc, dtype=np.uint8) if phases is None else np.asarray(phases, np.uint8)
    ld = np.full((3, 1, n, n), 0.5, np.float32)
    for a, step in ((0, np.array([dx, 0.0])), (1, np.array([0.0, dx]))):
        ds = step @ nh                               # s increment along the link (> 0)
        s_lo = np.mod(s0, P)
        for k in range(len(b)):
            # first crossing of the line s = b_k (mod P) in (0, ds]
            t = np.mod(b[k] - s_lo, P) / ds
            hit = (t > 0) & (t < 1)
            ld[a, 0][hit] = np.clip(t[hit], 1e-4, 1 - 1e-4)
    nrm3 = np.zeros((3, 3, 1, n, n), np.float32)
    nrm3[:, 0] = nh[0]
    nrm3[:, 1] = nh[1]
    g = Geometry(comp, ph, int(ph.max()) + 1, float(dx),
                 {"kind": "angled_slabs_2d", "link_normal": nrm3})
    g.link_delta = ld
    return g
