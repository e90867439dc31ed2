"""Host-side validation of btl_create: every refusal below happens before
the library makes a device call, so these run without a GPU.  The
geometry structs are built by hand to reach the checks directly."""
import ctypes

import numpy as np
import pytest

import paper_1907_00908_amd as btl


def _geom(n=(4, 4, 4), dx=0.5, bc=(0, 0, 0), comp=None, comp_phase=None, n_phase=1,
          n_comp=None, keep=None):
    comp = np.zeros(int(np.prod(n)), np.uint32) if comp is None else comp
    comp_phase = np.zeros(1, np.uint8) if comp_phase is None else comp_phase
    keep.extend([comp, comp_phase])
    g = btl.btl_geom()
    g.n[:] = list(n)
    g.dx = dx
    g.bc[:] = list(bc)
    g.n_comp = len(comp_phase) if n_comp is None else n_comp
    g.comp_id = comp.ctypes.data
    g.comp_phase = comp_phase.ctypes.data
    g.n_phase = n_phase
    g.link_delta = None
    g.link_normal = None
    return g


def _create(geoms, prec=btl.BTL_F32):
    lib = btl.load_library()
    arr = (btl.btl_geom * len(geoms))(*geoms)
    h = ctypes.c_void_p()
    st = lib.btl_create(arr, len(geoms), prec, ctypes.byref(h))
    return st, btl.btl_last_error(None), h


@pytest.mark.parametrize("case,word", [
    (dict(dx=0.0), "dx"),
    (dict(dx=float("inf")), "dx"),
    (dict(n_phase=0), "n_phase"),
    (dict(n_phase=9), "n_phase"),
    (dict(n=(1, 4, 4)), ">= 2 sites"),
    (dict(n=(4, 4, 0)), ">= 2 sites"),
    (dict(bc=(0, 2, 0)), "bc"),
    (dict(n=(2048, 2048, 65)), "too large"),      # 2.7e8 sites: beyond the 32-bit offsets
    (dict(comp_phase=np.array([1], np.uint8)), "comp_phase"),
    (dict(n_comp=0), "comp_id/comp_phase"),
])
def test_create_refuses_bad_geometry(case, word):
    keep = []
    if "n" in case and np.prod(case["n"]) > 1 << 20:
        # the size check comes before any read of the site labels
        case = dict(case, comp=np.zeros(1, np.uint32))
    st, msg, h = _create([_geom(keep=keep, **case)])
    assert st == btl.BTL_E_INVAL, (case, msg)
    assert word in msg, msg
    assert not h.value


def test_create_refuses_label_out_of_range_and_mixed_geometries():
    keep = []
    comp = np.zeros(64, np.uint32)
    comp[17] = 2                                          # only compartments 0, 1 exist
    st, msg, _ = _create([_geom(comp=comp, comp_phase=np.zeros(2, np.uint8), keep=keep)])
    assert st == btl.BTL_E_INVAL and "comp_id" in msg
    st, msg, _ = _create([_geom(keep=keep), _geom(dx=0.25, keep=keep)])
    assert st == btl.BTL_E_INVAL and "share dx" in msg
    st, msg, _ = _create([_geom(keep=keep), _geom(n_phase=2, comp_phase=np.zeros(1, np.uint8),
                                                  keep=keep)])
    assert st == btl.BTL_E_INVAL and "share dx and n_phase" in msg
    st, msg, _ = _create([_geom(keep=keep)], prec=7)
    assert st == btl.BTL_E_INVAL and "prec" in msg
    lib = btl.load_library()
    assert lib.btl_create(None, 1, btl.BTL_F32, ctypes.byref(ctypes.c_void_p())) == btl.BTL_E_INVAL
    assert lib.btl_create((btl.btl_geom * 1)(_geom(keep=keep)), 1, btl.BTL_F32, None) == btl.BTL_E_INVAL


def test_null_handle_calls_are_refused():
    lib = btl.load_library()
    for name, args in [("btl_forward", (None, 0.01, 1, None, None, None, 1, None, None, None,
                                        None, None, 0, None)),
                       ("btl_backward", (None,) * 8),
                       ("btl_set_scheme", (None, 0)), ("btl_set_lattice", (None, 0)),
                       ("btl_set_substeps", (None, 1)), ("btl_set_grad_gG0", (None, 0)),
                       ("btl_autotune", (None, 1, 1, None)),
                       ("btl_forward_noalloc", (None, 0.01, 1, None, None, None, 1, None, None,
                                                None, None, None, None)),
                       ("btl_set_launch", (None, 0, 0, 0)),
                       ("btl_set_adjoint_launch", (None, 0, 0)),
                       ("btl_set_memory_budget", (None, 0)), ("btl_set_graphs", (None, 1)),
                       ("btl_synchronize", (None, None))]:
        assert getattr(lib, name)(*args) == btl.BTL_E_INVAL, name
    v = ctypes.c_int32()
    assert lib.btl_get_launch(None, ctypes.byref(v), ctypes.byref(v), ctypes.byref(v)) == btl.BTL_E_INVAL
    v64 = ctypes.c_int64()
    assert lib.btl_get_backward_stats(None, ctypes.byref(v64), ctypes.byref(v),
                                      ctypes.byref(v)) == btl.BTL_E_INVAL
    vd = ctypes.c_double()
    assert lib.btl_get_backward_timing(None, ctypes.byref(vd), ctypes.byref(v64)) == btl.BTL_E_INVAL
    lib.btl_destroy(None)                                  # a no-op
