"""Seeded input generators shared by the oracle tests and the GPU path."""
from .workloads import (Material, System, MAT_A, MAT_B, plain_fcc, settled_bed, chute_two_level,  # noqa: F401
                        batch_systems, chute_adjoint, deposit, bed, chute_gravity, build_deposit)
