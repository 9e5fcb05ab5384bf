"""Tiny hand-built systems for closed-form checks (test helpers only)."""
import math

import numpy as np

from paper_1705_03850_amd.inputs.workloads import G0, MAT_A, Material, System


def mat(E=5e6, nu=0.25, rho=2500.0, e=0.9, mu=0.5):
    return Material(E=E, nu=nu, rho=rho, e=e, mu=mu)


def sphere_mass(r, rho):
    return 4.0 / 3.0 * math.pi * rho * r ** 3


def e_star(m1, m2):
    return 1.0 / ((1 - m1.nu ** 2) / m1.E + (1 - m2.nu ** 2) / m2.E)


def g_star(m1, m2):
    return 1.0 / (2 * (2 - m1.nu) * (1 + m1.nu) / m1.E + 2 * (2 - m2.nu) * (1 + m2.nu) / m2.E)


def two_spheres(v0=1.0, r1=1e-3, r2=1e-3, m1=None, m2=None, gap=1e-6):
    """Head-on approach along x at relative speed v0 (no gravity, no wall, open box)."""
    m1 = m1 or MAT_A
    m2 = m2 or m1
    mats = [m1] if m2 is m1 else [m1, m2]
    x = np.array([[-(r1 + gap / 2), 0.0, 0.0], [r2 + gap / 2, 0.0, 0.0]])
    # equal and opposite momenta: zero centre-of-mass velocity
    ma, mb = sphere_mass(r1, m1.rho), sphere_mass(r2, m2.rho)
    va = v0 * mb / (ma + mb)
    vb = -v0 * ma / (ma + mb)
    v = np.array([[va, 0.0, 0.0], [vb, 0.0, 0.0]])
    return System(x=x, v=v, w=np.zeros((2, 3)), r=np.array([r1, r2]),
                  type=np.array([0, 0 if m2 is m1 else 1], np.int32), id=np.array([0, 1], np.int32),
                  materials=mats, lo=(-20e-3, -20e-3, -20e-3), hi=(20e-3, 20e-3, 20e-3), periodic=(0, 0, 0),
                  wall_z0=0, g=(0.0, 0.0, 0.0), dt=1e-6, skin=0.1e-3, steps=0, name="two_spheres")


def sphere_on_wall(z, r=1e-3, m=None, v=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), g=(0.0, 0.0, -G0)):
    m = m or MAT_A
    return System(x=np.array([[0.0, 0.0, z]]), v=np.array([list(v)], float), w=np.array([list(w)], float),
                  r=np.array([r]), type=np.array([0], np.int32), id=np.array([7], np.int32), materials=[m],
                  lo=(-20e-3, -20e-3, 0.0), hi=(20e-3, 20e-3, 20e-3), periodic=(0, 0, 0), wall_z0=1, g=g,
                  dt=1e-6, skin=0.1e-3, steps=0, name="sphere_on_wall")
