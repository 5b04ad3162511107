"""Seeded synthetic inputs for the GSPM time step.

This package builds inputs only: node coordinates, tetrahedral connectivity,
material tags, material constants and initial fields.  It holds none of the
time-step arithmetic, so both the CPU oracle and the HIP library can take their
inputs from it without sharing any of the method.
"""
from .mesh import Mesh, kuhn_cube, random_rotation, tag_inclusions, Inclusion
from .cases import (Case, MATERIAL_FEGA, cube10_random, cube47_sphere,
                    cube100_ellipsoids, cube144_ellipsoids, small_cube, warm_start_training, CASES)

__all__ = ["Mesh", "kuhn_cube", "random_rotation", "tag_inclusions", "Inclusion",
           "Case", "MATERIAL_FEGA", "cube10_random", "cube47_sphere",
           "cube100_ellipsoids", "cube144_ellipsoids", "small_cube", "warm_start_training", "CASES"]
