"""The library's reverse-mode contact arithmetic (contact_vjp in dem_core.h),
built for the host, against central differences of the library's own forward
(contact_force) on random pair and wall contacts, sticking and sliding, with
and without the history update.  CPU only: it checks the hand-written adjoint
of Eq. (3)-(6) before any kernel uses it."""
import ctypes
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "contact_check.cpp")
CORE = os.path.join(os.path.dirname(HERE), "paper_1705_03850_amd", "csrc", "dem_core.h")
OUT = os.path.join(HERE, "native", "_build", "libcontact_check.so")

_dp = ctypes.POINTER(ctypes.c_double)


def _lib():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    newest = max(os.path.getmtime(SRC), os.path.getmtime(CORE))
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < newest:
        os.makedirs(os.path.dirname(OUT), exist_ok=True)
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               SRC, "-o", OUT + ".tmp"], stderr=subprocess.DEVNULL)
        os.replace(OUT + ".tmp", OUT)
    L = ctypes.CDLL(OUT)
    L.host_contact_force.argtypes = [_dp, _dp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _dp]
    L.host_contact_vjp.argtypes = [_dp, _dp, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
    return L


def _p(a):
    return a.ctypes.data_as(_dp)


def folded_coef(E=5e6, nu=0.25, e=0.9, mu=0.5):
    Es = E / (2 * (1 - nu * nu))
    Gs = E / (4 * (2 - nu) * (1 + nu))
    le = math.log(e)
    beta = le / math.sqrt(le * le + math.pi ** 2)
    return np.array([4 / 3 * Es, 8 * Gs, -beta * math.sqrt(20 / 3 * Es), -beta * math.sqrt(80 / 3 * Gs), mu])


def forward(L, inp, xi, wall, coef, dt, update):
    out = np.zeros(10)
    ok = L.host_contact_force(_p(inp), _p(xi), int(wall), _p(coef), dt, int(update), _p(out))
    return ok, out


def scalar(L, inp, xi, wall, coef, dt, update, seeds):
    ok, out = forward(L, inp, xi, wall, coef, dt, update)
    assert ok
    s = seeds[0:3] @ out[0:3] + seeds[3:6] @ out[3:6]
    if update:
        s += seeds[6:9] @ out[6:9]
    return s, out[9]


def make_case(rng, wall, slip):
    ra, rb = rng.uniform(0.9e-3, 1.1e-3, 2)
    ma, mb = (4 / 3 * math.pi * 2500 * r ** 3 for r in (ra, rb))
    frac = rng.uniform(2e-4, 5e-3)
    if wall:
        d = np.array([0.0, 0.0, ra * (1 - frac)])
    else:
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d = u * (ra + rb) * (1 - frac)
    vr = rng.normal(0, 0.05, 3)
    ws = rng.normal(0, 0.05, 3)
    n = d / np.linalg.norm(d)
    t = rng.normal(size=3)
    t -= (t @ n) * n
    t /= np.linalg.norm(t)
    delta = (ra if wall else ra + rb) * frac
    xi = t * delta * (0.5 if slip else 0.01) + n * delta * 0.01 * rng.normal()
    inp = np.array([*d, ra, rb, ma, mb, *vr, *ws])
    return inp, xi


@pytest.mark.parametrize("wall", [False, True])
@pytest.mark.parametrize("update", [0, 1])
@pytest.mark.parametrize("slip", [False, True])
def test_contact_vjp_matches_central_differences(wall, update, slip):
    L = _lib()
    rng = np.random.default_rng(100 + 4 * int(wall) + 2 * update + int(slip))
    coef = folded_coef()
    dt = 1e-6
    checked = 0
    for trial in range(12):
        inp, xi = make_case(rng, wall, slip)
        seeds = rng.normal(size=9)
        s0, flag = scalar(L, inp, xi, wall, coef, dt, update, seeds)
        if bool(flag) != slip:
            continue
        out = np.zeros(17)
        assert L.host_contact_vjp(_p(inp), _p(xi), int(wall), _p(coef), dt, update, _p(seeds), _p(out)) == 1
        # variables: d (wall: z only), v_r, w_s, xi, coefficients
        groups = [("d", inp, [2] if wall else [0, 1, 2], out[0:3] if not wall else out[2:3]),
                  ("vr", inp, [7, 8, 9], out[3:6]), ("ws", inp, [10, 11, 12], out[6:9]),
                  ("xi", xi, [0, 1, 2], out[9:12]), ("coef", coef, [0, 1, 2, 3, 4], out[12:17])]
        for name, arr, idx, got in groups:
            scale = np.abs(arr[idx]).max() if name != "coef" else None
            for m, k in enumerate(idx):
                h = 1e-6 * (scale if scale else abs(arr[k]))
                if name == "d":
                    h = 1e-9 * np.linalg.norm(inp[0:3])
                if h == 0.0:
                    h = 1e-12
                keep = arr[k]
                arr[k] = keep + h
                sp, fp = scalar(L, inp, xi, wall, coef, dt, update, seeds)
                arr[k] = keep - h
                sm, fm = scalar(L, inp, xi, wall, coef, dt, update, seeds)
                arr[k] = keep
                if fp != fm:
                    continue   # a Coulomb switch inside the difference step
                fd = (sp - sm) / (2 * h)
                tol = 2e-5 * max(abs(fd), abs(got[m])) + 1e-9 * abs(s0) / max(abs(keep), h)
                assert abs(fd - got[m]) <= tol, (name, k, fd, got[m], wall, update, slip)
                checked += 1
        if not update:
            assert np.all(out[9:12] == out[9:12])
    assert checked > 40


def test_contact_vjp_mirror_exact():
    """With a and b swapped and the seeds mirrored, every adjoint flips sign
    exactly (separation, relative velocity, history) or stays the same (w_s and
    the coefficients): the pair adjoint held by both particles agrees bit for bit."""
    L = _lib()
    rng = np.random.default_rng(7)
    coef = folded_coef()
    for slip in (False, True):
        for _ in range(20):
            inp, xi = make_case(rng, False, slip)
            seeds = rng.normal(size=9)
            a = np.zeros(17)
            assert L.host_contact_vjp(_p(inp), _p(xi), 0, _p(coef), 1e-6, 1, _p(seeds), _p(a)) == 1
            mir = inp.copy()
            mir[0:3] = -inp[0:3]
            mir[3], mir[4] = inp[4], inp[3]
            mir[5], mir[6] = inp[6], inp[5]
            mir[7:10] = -inp[7:10]
            ms = seeds.copy()
            ms[0:3] = -seeds[0:3]
            ms[6:9] = -seeds[6:9]
            b = np.zeros(17)
            assert L.host_contact_vjp(_p(mir), _p(-xi), 0, _p(coef), 1e-6, 1, _p(ms), _p(b)) == 1
            assert np.array_equal(b[0:6], -a[0:6])
            assert np.array_equal(b[6:9], a[6:9])
            assert np.array_equal(b[9:12], -a[9:12])
            assert np.array_equal(b[12:17], a[12:17])


def test_no_contact_writes_nothing():
    L = _lib()
    inp = np.array([3e-3, 0, 0, 1e-3, 1e-3, 1e-5, 1e-5, 0, 0, 0, 0, 0, 0], float)
    out = np.full(17, 7.0)
    assert L.host_contact_vjp(_p(inp), _p(np.zeros(3)), 0, _p(folded_coef()), 1e-6, 1, _p(np.ones(9)), _p(out)) == 0
    assert np.all(out == 7.0)
