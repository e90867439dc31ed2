"""Python binding of libbtlbm (hybrid LBM Bloch-Torrey solver for gfx950).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libbtlbm.so.  The `btl_*` functions below mirror the C ABI of
include/btlbm.h one to one (the names are listed in EXPORTED).  `Simulator`
wraps them with torch tensors for device memory and the current torch
stream.

There is no CPU fallback: if libbtlbm.so is missing or fails to load, every
call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbtlbm.so")

BTL_OK, BTL_E_INVAL, BTL_E_UNSUPPORTED, BTL_E_NOMEM, BTL_E_HIP, BTL_E_NONFINITE = range(6)
BTL_PERIODIC, BTL_MIRROR = 0, 1
BTL_F64, BTL_F32 = 0, 1
BTL_HYBRID, BTL_CLASSICAL = 0, 1
BTL_D3Q7, BTL_D2Q5 = 0, 1

EXPORTED = ("btl_create", "btl_forward", "btl_forward_noalloc", "btl_backward",
            "btl_get_backward_stats", "btl_get_backward_timing", "btl_set_scheme", "btl_set_lattice", "btl_set_substeps",
            "btl_set_grad_gG0", "btl_autotune", "btl_set_launch", "btl_set_adjoint_launch",
            "btl_set_memory_budget", "btl_set_graphs", "btl_get_launch", "btl_synchronize",
            "btl_destroy", "btl_last_error")


class BtlError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"btl status {status}: {msg}")
        self.status = status


class btl_geom(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double),
                ("bc", ctypes.c_int32 * 3), ("n_comp", ctypes.c_int32),
                ("comp_id", ctypes.c_void_p), ("comp_phase", ctypes.c_void_p),
                ("n_phase", ctypes.c_int32), ("link_delta", ctypes.c_void_p),
                ("link_normal", ctypes.c_void_p)]


_lib = None


def load_library(path: str = None):
    """Load libbtlbm.so and declare its signatures (raises if missing).

    The environment variable BTLBM_LIBRARY may name another build of the
    same library (for example one compiled with different tile options)."""
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        path = os.environ.get("BTLBM_LIBRARY", LIB_PATH)
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1907_00908_amd.build`")
    lib = ctypes.CDLL(path)
    P, i32, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.btl_create.argtypes = [ctypes.POINTER(btl_geom), i32, i32, ctypes.POINTER(P)]
    lib.btl_create.restype = ctypes.c_int
    lib.btl_forward.argtypes = [P, d, i32, P, P, P, i32, P, P, P, P, P, i32, P]
    lib.btl_forward.restype = ctypes.c_int
    lib.btl_forward_noalloc.argtypes = [P, d, i32, P, P, P, i32, P, P, P, P, P, P]
    lib.btl_forward_noalloc.restype = ctypes.c_int
    lib.btl_backward.argtypes = [P, P, P, P, P, P, P, P]
    lib.btl_backward.restype = ctypes.c_int
    lib.btl_get_backward_stats.argtypes = [P, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.btl_get_backward_stats.restype = ctypes.c_int
    lib.btl_get_backward_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64)]
    lib.btl_get_backward_timing.restype = ctypes.c_int
    lib.btl_set_launch.argtypes = [P, i32, i32, i32]
    lib.btl_set_launch.restype = ctypes.c_int
    lib.btl_set_adjoint_launch.argtypes = [P, i32, i32]
    lib.btl_set_adjoint_launch.restype = ctypes.c_int
    lib.btl_set_memory_budget.argtypes = [P, ctypes.c_int64]
    lib.btl_set_memory_budget.restype = ctypes.c_int
    lib.btl_set_graphs.argtypes = [P, i32]
    lib.btl_set_graphs.restype = ctypes.c_int
    lib.btl_synchronize.argtypes = [P, P]
    lib.btl_synchronize.restype = ctypes.c_int
    lib.btl_set_scheme.argtypes = [P, i32]
    lib.btl_set_scheme.restype = ctypes.c_int
    lib.btl_set_lattice.argtypes = [P, i32]
    lib.btl_set_lattice.restype = ctypes.c_int
    lib.btl_set_substeps.argtypes = [P, i32]
    lib.btl_set_substeps.restype = ctypes.c_int
    lib.btl_set_grad_gG0.argtypes = [P, i32]
    lib.btl_set_grad_gG0.restype = ctypes.c_int
    lib.btl_autotune.argtypes = [P, i32, i32, P]
    lib.btl_autotune.restype = ctypes.c_int
    lib.btl_get_launch.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
    lib.btl_get_launch.restype = ctypes.c_int
    lib.btl_destroy.argtypes = [P]
    lib.btl_destroy.restype = None
    lib.btl_last_error.argtypes = [P]
    lib.btl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(st, handle):
    if st != BTL_OK:
        msg = load_library().btl_last_error(handle)
        raise BtlError(st, msg.decode() if msg else "")


# ---- one-to-one wrappers of the C ABI -------------------------------------

def btl_create(geoms, prec: int):
    """geoms: list of objects with comp (n2,n1,n0) uint32, comp_phase uint8,
    n_phase, dx, a `bc` list and optionally link_delta (3, n2, n1, n0)
    float32 membrane positions (None: half-link membranes) and link_normal
    (3, 3, n2, n1, n0) float32 membrane normals (None: membranes normal to
    the links).  Returns the handle."""
    lib = load_library()
    arr = (btl_geom * len(geoms))()
    keep = []
    for i, g in enumerate(geoms):
        comp = np.ascontiguousarray(g.comp, dtype=np.uint32)
        cp = np.ascontiguousarray(g.comp_phase, dtype=np.uint8)
        keep += [comp, cp]
        n2, n1, n0 = comp.shape
        arr[i].n[:] = [n0, n1, n2]
        arr[i].dx = float(g.dx)
        arr[i].bc[:] = [int(b) for b in g.bc]
        arr[i].n_comp = len(cp)
        arr[i].comp_id = _np_ptr(comp)
        arr[i].comp_phase = _np_ptr(cp)
        arr[i].n_phase = int(g.n_phase)
        ld = getattr(g, "link_delta", None)
        if ld is not None:
            ld = np.ascontiguousarray(ld, dtype=np.float32)
            if ld.shape != (3,) + comp.shape:
                raise ValueError("link_delta must have shape (3, n2, n1, n0)")
            keep.append(ld)
            arr[i].link_delta = _np_ptr(ld)
        ln = getattr(g, "link_normal", None)
        if ln is not None:
            ln = np.ascontiguousarray(ln, dtype=np.float32)
            if ln.shape != (3, 3) + comp.shape:
                raise ValueError("link_normal must have shape (3, 3, n2, n1, n0)")
            keep.append(ln)
            arr[i].link_normal = _np_ptr(ln)
    h = ctypes.c_void_p()
    _check(lib.btl_create(arr, len(geoms), int(prec), ctypes.byref(h)), None)
    return h


def _forward_args(K, D, T2, kappa, Q, q_geom, gG0, f, substeps):
    if len(f) < int(K) * int(substeps):
        raise ValueError("f needs K * substeps samples")
    D = np.ascontiguousarray(D, np.float64)
    T2 = np.ascontiguousarray(T2, np.float64)
    kappa = np.ascontiguousarray(kappa, np.float64).reshape(-1)
    q_geom = np.ascontiguousarray(q_geom, np.int32)
    gG0 = np.ascontiguousarray(gG0, np.float64).reshape(-1)
    f = np.ascontiguousarray(f, np.float64)
    if q_geom.size < int(Q) or gG0.size < 3 * int(Q):
        raise ValueError("q_geom needs Q entries and gG0 Q x 3")
    if D.size != T2.size or kappa.size != D.size * D.size:
        raise ValueError("D and T2 need n_phase values, kappa n_phase x n_phase")
    return D, T2, kappa, q_geom, gG0, f


def btl_forward(h, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E_ptr, M_ptr,
                ckpt_every, stream_ptr, substeps=1):
    """f must hold K * substeps samples (substeps as set on the handle)."""
    lib = load_library()
    D, T2, kappa, q_geom, gG0, f = _forward_args(K, D, T2, kappa, Q, q_geom, gG0, f, substeps)
    st = lib.btl_forward(h, float(dt), int(K), _np_ptr(D), _np_ptr(T2), _np_ptr(kappa),
                         int(Q), _np_ptr(q_geom), _np_ptr(gG0), _np_ptr(f),
                         ctypes.c_void_p(E_ptr), ctypes.c_void_p(M_ptr) if M_ptr else None,
                         int(ckpt_every), ctypes.c_void_p(stream_ptr) if stream_ptr else None)
    _check(st, h)


def btl_forward_noalloc(h, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E_ptr, M_ptr,
                        stream_ptr, substeps=1):
    """btl_forward without tape, all internal device buffers in the
    library's fixed device scratch (no allocation)."""
    lib = load_library()
    D, T2, kappa, q_geom, gG0, f = _forward_args(K, D, T2, kappa, Q, q_geom, gG0, f, substeps)
    st = lib.btl_forward_noalloc(h, float(dt), int(K), _np_ptr(D), _np_ptr(T2),
                                 _np_ptr(kappa), int(Q), _np_ptr(q_geom), _np_ptr(gG0),
                                 _np_ptr(f), ctypes.c_void_p(E_ptr),
                                 ctypes.c_void_p(M_ptr) if M_ptr else None,
                                 ctypes.c_void_p(stream_ptr) if stream_ptr else None)
    _check(st, h)


def btl_backward(h, dLdE_ptr, dD_ptr, dT2_ptr, dkappa_ptr, df_ptr, dgG0_ptr, stream_ptr):
    lib = load_library()
    V = lambda p: ctypes.c_void_p(p) if p else None  # noqa: E731
    _check(lib.btl_backward(h, V(dLdE_ptr), V(dD_ptr), V(dT2_ptr), V(dkappa_ptr),
                            V(df_ptr), V(dgG0_ptr), V(stream_ptr)), h)


def btl_get_backward_stats(h):
    """(forward steps recomputed, groups of q-samples, snapshots per group)
    of the last btl_backward."""
    lib = load_library()
    a, b, c = ctypes.c_int64(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib.btl_get_backward_stats(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), h)
    return int(a.value), int(b.value), int(c.value)


def btl_get_backward_timing(h):
    """(milliseconds, steps) of the adjoint-step launches of the last
    btl_backward (uniform tape)."""
    lib = load_library()
    ms, n = ctypes.c_double(0.0), ctypes.c_int64(0)
    _check(lib.btl_get_backward_timing(h, ctypes.byref(ms), ctypes.byref(n)), h)
    return float(ms.value), int(n.value)


def btl_set_launch(h, tile_shape, zc, xcd):
    _check(load_library().btl_set_launch(h, int(tile_shape), int(zc), int(xcd)), h)


def btl_set_adjoint_launch(h, zc, xcd):
    _check(load_library().btl_set_adjoint_launch(h, int(zc), int(xcd)), h)


def btl_set_memory_budget(h, nbytes):
    _check(load_library().btl_set_memory_budget(h, int(nbytes)), h)


def btl_set_graphs(h, on):
    _check(load_library().btl_set_graphs(h, int(on)), h)


def btl_synchronize(h, stream_ptr):
    lib = load_library()
    _check(lib.btl_synchronize(h, ctypes.c_void_p(stream_ptr) if stream_ptr else None), h)


def btl_set_scheme(h, scheme):
    _check(load_library().btl_set_scheme(h, int(scheme)), h)


def btl_set_lattice(h, lattice):
    _check(load_library().btl_set_lattice(h, int(lattice)), h)


def btl_set_substeps(h, m):
    _check(load_library().btl_set_substeps(h, int(m)), h)


def btl_set_grad_gG0(h, on):
    _check(load_library().btl_set_grad_gG0(h, int(on)), h)


def btl_autotune(h, Q, K_probe, stream_ptr):
    lib = load_library()
    _check(lib.btl_autotune(h, int(Q), int(K_probe),
                            ctypes.c_void_p(stream_ptr) if stream_ptr else None), h)


def btl_get_launch(h):
    """(tile_shape, zc, xcd) of the simulator's forwards (see the header)."""
    lib = load_library()
    v = [ctypes.c_int32(0) for _ in range(3)]
    _check(lib.btl_get_launch(h, *[ctypes.byref(x) for x in v]), h)
    return tuple(int(x.value) for x in v)


def btl_destroy(h):
    load_library().btl_destroy(h)


def btl_last_error(h):
    m = load_library().btl_last_error(h)
    return m.decode() if m else ""


# ---- torch-facing convenience ----------------------------------------------

class _GeomBC:
    """A workloads.Geometry together with its per-axis outer boundary."""

    def __init__(self, g, bc):
        self.comp, self.comp_phase = g.comp, g.comp_phase
        self.n_phase, self.dx, self.bc = g.n_phase, g.dx, list(bc)
        self.link_delta = getattr(g, "link_delta", None)
        self.link_normal = getattr(g, "link_normal", None)


class Simulator:
    """Owns one btl_sim.  Device memory for E and M_final comes from torch."""

    def __init__(self, geoms, bc, prec: str = "f32", scheme: int = BTL_HYBRID,
                 substeps: int = 1, lattice: int = BTL_D3Q7, grad_gG0: bool = False,
                 launch=None, adjoint_launch=None, mem_budget: int = 0, graphs: bool = True):
        """launch: (tile_shape, zc, xcd) for btl_set_launch; adjoint_launch:
        (zc, xcd) for btl_set_adjoint_launch; mem_budget: bytes for
        btl_set_memory_budget (0: none); graphs: btl_set_graphs."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Simulator needs a HIP device")
        self.torch = torch
        self.prec = BTL_F32 if prec == "f32" else BTL_F64
        self.geoms = list(geoms)
        bcs = bc if isinstance(bc[0], (list, tuple)) else [bc] * len(self.geoms)
        self._h = btl_create([_GeomBC(g, b) for g, b in zip(self.geoms, bcs)], self.prec)
        if scheme != BTL_HYBRID:
            btl_set_scheme(self._h, scheme)
        if lattice != BTL_D3Q7:
            btl_set_lattice(self._h, lattice)
        self.substeps = int(substeps)
        if self.substeps != 1:
            btl_set_substeps(self._h, self.substeps)
        self.grad_gG0 = bool(grad_gG0)
        if self.grad_gG0:
            btl_set_grad_gG0(self._h, 1)
        if launch is not None:
            btl_set_launch(self._h, *launch)
        if adjoint_launch is not None:
            btl_set_adjoint_launch(self._h, *adjoint_launch)
        if mem_budget:
            btl_set_memory_budget(self._h, mem_budget)
        if not graphs:
            btl_set_graphs(self._h, 0)
        # number of forwards so far, and which of them holds the adjoint tape
        # (with its q-sample count and steps: the sizes btl_backward reads
        # and writes)
        self._n_forward = 0
        self.tape_id = None
        self._tape_QK = None

    def set_grad_gG0(self, on: bool):
        """Plan taped forwards for the gamma G0 gradient (btl_set_grad_gG0)."""
        if bool(on) != self.grad_gG0:
            btl_set_grad_gG0(self._h, 1 if on else 0)
            self.grad_gG0 = bool(on)

    def close(self):
        if self._h is not None:
            btl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, dt, D, T2, kappa, f, gG0, q_geom=None, want_M=False,
                ckpt_every=0, noalloc=False):
        """Returns E (Q, K+1) complex128 torch tensor on the device (and M).
        noalloc: run through btl_forward_noalloc (no tape, the library's
        fixed device scratch; E and M still come from torch)."""
        torch = self.torch
        gG0 = np.ascontiguousarray(gG0, np.float64).reshape(-1, 3)
        Q = gG0.shape[0]
        q_geom = np.zeros(Q, np.int32) if q_geom is None else np.asarray(q_geom, np.int32)
        P = self.geoms[0].n_phase
        if q_geom.shape != (Q,):
            raise ValueError("q_geom needs one geometry index per q-sample")
        if np.size(D) != P or np.size(T2) != P or np.size(kappa) != P * P:
            raise ValueError("D and T2 need n_phase values, kappa n_phase x n_phase")
        if len(f) % self.substeps:
            raise ValueError("len(f) must be a multiple of the reaction sub-steps")
        K = len(f) // self.substeps
        dev = torch.device("cuda", torch.cuda.current_device())
        E = torch.empty((Q, K + 1, 2), dtype=torch.float64, device=dev)
        M = None
        if want_M:
            tot = sum(self.geoms[int(g)].comp.size for g in q_geom)
            dt_ = torch.float32 if self.prec == BTL_F32 else torch.float64
            M = torch.empty((tot, 2), dtype=dt_, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        if noalloc:
            if ckpt_every:
                raise ValueError("btl_forward_noalloc keeps no adjoint tape")
            btl_forward_noalloc(self._h, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E.data_ptr(),
                                M.data_ptr() if M is not None else 0, stream, self.substeps)
        else:
            self.tape_id = None
            self._tape_QK = None
            btl_forward(self._h, dt, K, D, T2, kappa, Q, q_geom, gG0, f, E.data_ptr(),
                        M.data_ptr() if M is not None else 0, ckpt_every, stream,
                        self.substeps)
            self._n_forward += 1
            if ckpt_every > 0 and K > 0:
                self.tape_id = self._n_forward
                self._tape_QK = (Q, K)
        Ec = torch.view_as_complex(E)
        if not want_M:
            return Ec
        Ms, off = [], 0
        Mc = torch.view_as_complex(M)
        for g in q_geom:
            sh = self.geoms[int(g)].comp.shape
            n = int(np.prod(sh))
            Ms.append(Mc[off:off + n].reshape(sh))
            off += n
        return Ec, Ms


    def backward(self, dLdE, P: int = None, K: int = None, grad_gG0: bool = False):
        """Gradients of a real loss from dL/dE (torch (Q, K+1, 2) float64 on
        the device: dL/dRe E, dL/dIm E) for the last forward that kept a tape.
        The sizes come from that forward (P, K, when given, must match it).
        Returns device tensors dD [P], dT2 [P], dkappa [P, P], df
        [K * substeps] (one entry per waveform sample), and with grad_gG0 also
        dgG0 [Q, 3]."""
        torch = self.torch
        if self._tape_QK is None:
            raise RuntimeError("no adjoint tape: run forward with ckpt_every > 0 first")
        Q, Kt = self._tape_QK
        Pt = self.geoms[0].n_phase
        if (P is not None and int(P) != Pt) or (K is not None and int(K) != Kt):
            raise ValueError(f"the taped forward has n_phase {Pt} and K {Kt}")
        P, K = Pt, Kt
        if tuple(dLdE.shape) != (Q, K + 1, 2):
            raise ValueError(f"dLdE must have shape ({Q}, {K + 1}, 2)")
        dev = dLdE.device
        g = dLdE.detach().to(torch.float64).contiguous()
        dD = torch.empty(P, dtype=torch.float64, device=dev)
        dT2 = torch.empty(P, dtype=torch.float64, device=dev)
        dk = torch.empty((P, P), dtype=torch.float64, device=dev)
        nf = K * self.substeps
        df = torch.empty(max(nf, 1), dtype=torch.float64, device=dev)
        dG = torch.empty((Q, 3), dtype=torch.float64, device=dev) if grad_gG0 else None
        stream = torch.cuda.current_stream().cuda_stream
        btl_backward(self._h, g.data_ptr(), dD.data_ptr(), dT2.data_ptr(), dk.data_ptr(),
                     df.data_ptr(), dG.data_ptr() if grad_gG0 else None, stream)
        if grad_gG0:
            return dD, dT2, dk, df[:nf], dG
        return dD, dT2, dk, df[:nf]


def _bt_function():
    import torch

    class BlochTorreySignal(torch.autograd.Function):
        """E = signal(D, T2, kappa, f) as a real (Q, K+1, 2) tensor, with the
        hand-written adjoint of libbtlbm as its backward.

        forward(D [P], T2 [P], kappa [P, P], f [K], sim, dt, gG0 [Q, 3],
        q_geom [Q], ckpt_every).  The parameters may live on any device; the
        returned gradients are placed on the parameter's device.  gG0 may be
        a tensor: it gets a gradient when it requires one."""

        @staticmethod
        def forward(ctx, D, T2, kappa, f, sim, dt, gG0, q_geom, ckpt_every):
            Dn = D.detach().cpu().double().numpy()
            T2n = T2.detach().cpu().double().numpy()
            kn = kappa.detach().cpu().double().numpy()
            fn = f.detach().cpu().double().numpy()
            if torch.is_tensor(gG0):
                ctx.gdev = gG0.device
                if gG0.requires_grad:
                    sim.set_grad_gG0(True)
                gG0 = gG0.detach().cpu().double().numpy()
            else:
                ctx.gdev = None
            gG0 = np.ascontiguousarray(gG0, np.float64).reshape(-1, 3)
            E = sim.forward(dt, Dn, T2n, kn, fn, gG0, q_geom, ckpt_every=max(1, int(ckpt_every)))
            ctx.sim = sim
            ctx.tape_id = sim.tape_id
            ctx.P = len(Dn)
            ctx.K = len(fn) // sim.substeps
            ctx.devs = (D.device, T2.device, kappa.device, f.device)
            return torch.view_as_real(E).clone()

        @staticmethod
        def backward(ctx, gE):
            if ctx.sim.tape_id is None or ctx.sim.tape_id != ctx.tape_id:
                raise RuntimeError("the simulator ran another forward after this one: its "
                                   "adjoint tape is gone (use one Simulator per pending backward)")
            want_g = ctx.gdev is not None and ctx.needs_input_grad[6]
            out = ctx.sim.backward(gE, ctx.P, ctx.K, grad_gG0=want_g)
            dD, dT2, dk, df = out[:4]
            dG = out[4].to(ctx.gdev) if want_g else None
            d0, d1, d2, d3 = ctx.devs
            return (dD.to(d0), dT2.to(d1), dk.to(d2), df.to(d3),
                    None, None, dG, None, None)

    return BlochTorreySignal


_BTS = None


def bloch_torrey_signal(D, T2, kappa, f, sim, dt, gG0, q_geom=None, ckpt_every=100):
    """Differentiable signal (see BlochTorreySignal)."""
    global _BTS
    if _BTS is None:
        _BTS = _bt_function()
    import torch
    if not torch.is_tensor(gG0):
        gG0 = np.ascontiguousarray(gG0, np.float64).reshape(-1, 3)
    if q_geom is None:
        q_geom = np.zeros(len(gG0), np.int32)
    return _BTS.apply(D, T2, kappa, f, sim, dt, gG0, q_geom, ckpt_every)


def simulate_config(cfg: dict, prec: str = "f32", want_M: bool = False, scheme=None,
                    **options):
    """Run a workloads config on the GPU: returns E (Q, K+1) complex (and M).
    The scheme is `scheme`, else the config's "scheme" entry, else hybrid;
    the config's "substeps" entry (default 1) sets reaction sub-steps and its
    "lattice" entry (default D3Q7) the lattice.  options go to Simulator
    (launch, mem_budget, graphs, ...)."""
    if scheme is None:
        scheme = cfg.get("scheme", BTL_HYBRID)
    sim = Simulator(cfg["geoms"], cfg["bc"], prec, scheme, cfg.get("substeps", 1),
                    cfg.get("lattice", BTL_D3Q7), **options)
    try:
        out = sim.forward(cfg["dt"], cfg["D"], cfg["T2"], cfg["kappa"], cfg["f"],
                          cfg["gG0"], cfg["q_geom"], want_M=want_M)
        sim.torch.cuda.synchronize()
        return out
    finally:
        sim.close()
