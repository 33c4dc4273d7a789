"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws numbers and builds initial fields and geometries; it
holds none of the lattice Boltzmann arithmetic (no weights, no moments, no
equilibria).  Every generator takes an explicit seed (numpy PCG64)."""
from .workloads import *  # noqa: F401,F403
