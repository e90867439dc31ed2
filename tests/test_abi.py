"""The C ABI: the library loads and exports every function the header
declares, and the Python binding mirrors them by name (no GPU calls)."""
import os
import re

import paper_1907_00908_amd as btl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "btlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(btl_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_exported_set():
    assert _declared() == sorted(btl.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = btl.load_library()
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_mirrors_names():
    for name in _declared():
        assert callable(getattr(btl, name)), name


def test_create_rejects_bad_geometry_without_touching_the_gpu():
    # validation happens before any device call
    import numpy as np

    class G:
        comp = np.zeros((2, 2, 2), np.uint32)
        comp_phase = np.zeros(1, np.uint8)
        n_phase = 1
        dx = -1.0
        bc = [0, 0, 0]
    try:
        btl.btl_create([G()], btl.BTL_F32)
    except btl.BtlError as e:
        assert e.status == btl.BTL_E_INVAL
        assert "dx" in str(e)
    else:
        raise AssertionError("negative dx accepted")


def test_binding_refuses_short_q_arrays_before_the_call():
    # the C side reads Q geometry indices and Q x 3 gradients through plain
    # pointers; the binding checks the arrays cover them
    import numpy as np
    import pytest
    inf = float("inf")
    with pytest.raises(ValueError):
        btl.btl_forward(None, 0.01, 1, [1.0], [1.0], [[inf]], 2, [0], np.zeros(6),
                        np.zeros(1), 0, 0, 0, 0)
    with pytest.raises(ValueError):
        btl.btl_forward(None, 0.01, 1, [1.0], [1.0], [[inf]], 2, [0, 0], np.zeros(3),
                        np.zeros(1), 0, 0, 0, 0)
