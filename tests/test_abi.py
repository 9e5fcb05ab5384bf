"""The C-ABI library loads, exports every declared symbol, and validates
configurations on the host (no GPU needed: dem_workspace_size does no device work)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1705_03850_amd import dem
from paper_1705_03850_amd.inputs import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "dem.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(dem_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(dem.symbols())


def test_library_exports_every_declared_symbol():
    L = dem.load()
    out = subprocess.run(["nm", "-D", "--defined-only", dem.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dem_\w+)", out))
    for name in declared_symbols():
        assert name in exported, name
        assert hasattr(L, name)


def ws_size(cfgs):
    L = dem.load()
    arr = (dem.Config * len(cfgs))(*cfgs)
    b = ctypes.c_size_t()
    rc = L.dem_batch_workspace_size(len(cfgs), arr, ctypes.byref(b))
    return rc, b.value


def test_workspace_size_scales_with_particles():
    s = W.plain_fcc()
    rc, b1 = ws_size([dem.make_config(s)])
    assert rc == dem.DEM_OK and b1 > 0
    s2 = s.copy()
    s2.r = np.concatenate([s.r, s.r]); s2.x = np.concatenate([s.x, s.x])
    rc, b2 = ws_size([dem.make_config(s2)])
    assert rc == dem.DEM_OK and b2 > b1
    rc, b3 = ws_size([dem.make_config(s), dem.make_config(s)])
    assert rc == dem.DEM_OK and b3 >= 2 * b1 - 65536


@pytest.mark.parametrize("field,value,code", [
    ("e", 0.0, dem.DEM_ERR_ARG), ("e", 1.2, dem.DEM_ERR_ARG), ("mu", -0.1, dem.DEM_ERR_ARG),
    ("E", 0.0, dem.DEM_ERR_ARG), ("nu", 0.5, dem.DEM_ERR_ARG), ("rho", -1.0, dem.DEM_ERR_ARG),
])
def test_material_validation(field, value, code):
    c = dem.make_config(W.plain_fcc())
    setattr(c.mat[0], field, value)
    assert ws_size([c])[0] == code


def test_config_validation():
    base = W.plain_fcc()
    c = dem.make_config(base); c.dt = 0.0
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    c = dem.make_config(base); c.skin = 0.0
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    c = dem.make_config(base); c.k_max = 64
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    c = dem.make_config(base); c.block = 96
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    c = dem.make_config(base); c.cell = 1e-3           # smaller than 2 r_max + skin
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    small = base.copy(); small.hi = (4e-3, 20e-3, 60e-3)   # periodic x shorter than two cut-offs
    assert ws_size([dem.make_config(small)])[0] == dem.DEM_ERR_DOMAIN
    c = dem.make_config(base); c.hi[2] = c.lo[2]
    assert ws_size([c])[0] == dem.DEM_ERR_ARG
    a, b = dem.make_config(base), dem.make_config(base)
    a.block, b.block = 64, 128
    assert ws_size([a, b])[0] == dem.DEM_ERR_ARG
