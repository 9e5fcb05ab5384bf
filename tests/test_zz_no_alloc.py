"""dem_init_noalloc: a context whose workspace is the library's static device
array (for callers that cannot allocate device memory) steps exactly as a
context over a caller workspace, call after call, and a system too large for
the array is refused before any device work."""
import ctypes

import numpy as np
import pytest

from paper_1705_03850_amd import dem
from paper_1705_03850_amd.inputs import workloads as W


def test_noalloc_refuses_oversized_system():
    """Checked on the host before any device call (runs without a GPU)."""
    L = dem.load()
    cfg = dem.make_config(W.plain_fcc())
    cfg.n = 200_000                                    # about 0.5 GB of workspace at k_max = 32
    need = ctypes.c_size_t()
    assert L.dem_workspace_size(ctypes.byref(cfg), ctypes.byref(need)) == dem.DEM_OK
    assert need.value > 64 << 20
    ctx = ctypes.c_void_p()
    rc = L.dem_init_noalloc(ctypes.byref(ctx), ctypes.byref(cfg), None)
    assert rc == dem.DEM_ERR_CAPACITY and not ctx.value
    assert b"static workspace" in L.dem_last_error(None)


def _run(system, static, steps):
    g = dem.DemSystem(system, static_workspace=static)
    g.prime()
    g.step(steps)
    h = g.host()
    a, b = g.export_neighbors()
    stats = g.stats()
    g.close()
    return h, a, b, stats


@pytest.mark.gpu
def test_noalloc_equals_dem_init_twice():
    """Two static contexts in a row, the second smaller, each against a context
    over a caller workspace on the same input: state, list and counters agree
    bit for bit (the second also shows that the array's leftovers from the
    first do not leak into it)."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for system, steps in ((W.plain_fcc(), 150), (W.chute_adjoint(seed=9, n=600, Lx=14e-3, Ly=10e-3), 120)):
        ref = _run(system, False, steps)
        got = _run(system, True, steps)
        for key in ("id", "x", "v", "w", "f", "t"):
            assert np.array_equal(ref[0][key], got[0][key]), (system.name, key)
        assert np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])
        assert ref[3] == got[3]
        assert ref[3]["steps"] == steps and ref[3]["contacts"] > 0


@pytest.mark.gpu
def test_noalloc_one_context_per_device():
    """While a static context lives, a second one on the device is refused;
    after dem_destroy the array is free again."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.plain_fcc()
    g = dem.DemSystem(s, static_workspace=True)
    with pytest.raises(dem.DemError) as e:
        dem.DemSystem(s, static_workspace=True)
    assert e.value.code == dem.DEM_ERR_STATE
    g.close()
    g2 = dem.DemSystem(s, static_workspace=True)
    g2.prime()
    g2.step(10)
    g2.close()
