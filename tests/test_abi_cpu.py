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
    assert b.SITE_DTYPE.itemsize == 8 and b.METRICS_DTYPE.itemsize == 88


def test_binding_layouts_match_the_header(tmp_path):
    """Every ABI structure the binding declares has the C compiler's size and
    field offsets (the header compiled with g++)."""
    import subprocess
    from paper_2606_21791_amd import binding as b
    exe = tmp_path / "abi_layout"
    subprocess.run(["g++", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "abi_layout.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    c = {k: int(v) for k, v in (line.split() for line in out.splitlines())}
    ct = {"sg_scene": b.SgScene, "sg_camera": b.SgCamera, "sg_raster": b.SgRaster, "sg_box": b.SgBox,
          "sg_campaign_cfg": b.SgCampaignCfg, "sg_tune_t": b.SgTune, "sg_serve_config": b.SgServeConfig,
          "sg_request": b.SgRequest, "sg_result": b.SgResult, "sg_serve_stats_t": b.SgServeStats}
    npd = {"sg_site": b.SITE_DTYPE, "sg_variant": b.VARIANT_DTYPE, "sg_metrics_t": b.METRICS_DTYPE}
    checked = 0
    for key, val in c.items():
        name, _, field = key.partition(".")
        if name in ct:
            got = ctypes.sizeof(ct[name]) if not field else getattr(ct[name], field).offset
        else:
            got = npd[name].itemsize if not field else npd[name].fields[field][1]
        assert got == val, (key, got, val)
        checked += 1
    assert checked >= 60


def test_invalid_arguments_are_rejected_without_a_gpu():
    from paper_2606_21791_amd import binding as b
    h = ctypes.c_void_p()
    # a NULL out pointer is rejected before any device call
    assert b.LIB.sg_ctx_create(0, 0, None) == b.SG_E_INVAL
    assert b.LIB.sg_cast(None, None, None, 0, 0, 0, None) == b.SG_E_INVAL
