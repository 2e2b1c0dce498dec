"""CPU checks of the boundary: the library loads and exports every symbol the
header declares; the binding's structure layouts match the header's."""
import ctypes
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2606_21791_amd import binding
    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(binding.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(binding.EXPORTED) <= set(names)


def test_struct_layouts():
    from paper_2606_21791_amd import binding as b
    assert ctypes.sizeof(b.SgScene) == 6 * 8 * 3 + 16
    assert ctypes.sizeof(b.SgCamera) == 8 * 18 + 8
    assert ctypes.sizeof(b.SgRaster) == 4 * 9
    assert ctypes.sizeof(b.SgBox) == 8 + 12 * 8
    assert b.SITE_DTYPE.itemsize == 8 and b.METRICS_DTYPE.itemsize == 72


def test_invalid_arguments_are_rejected_without_a_gpu():
    from paper_2606_21791_amd import binding as b
    h = ctypes.c_void_p()
    # a NULL out pointer is rejected before any device call
    assert b.LIB.sg_ctx_create(0, 0, None) == b.SG_E_INVAL
    assert b.LIB.sg_cast(None, None, None, 0, 0, 0, None) == b.SG_E_INVAL
