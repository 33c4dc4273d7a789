"""Shared helpers of the GPU parity tests: run the same seeded problem through
the HIP library (via the C ABI binding) and through the FP64 oracle."""
from __future__ import annotations

import numpy as np

from oracle import rmrt_oracle as O

WALLS = {"y": O.WALL_YM | O.WALL_YP, "z": O.WALL_ZM | O.WALL_ZP, "yz": O.WALL_YM | O.WALL_YP | O.WALL_ZM | O.WALL_ZP}


def random_fields(m: O.Model, seed: int, du=0.02, drho=1e-3):
    """Smooth-plus-noise initial fields (seeded) for a model's grid."""
    rng = np.random.default_rng(seed)
    x, y, z = m.xyz
    nx, ny, nz = m.shape
    kx, ky, kz = 2 * np.pi / nx, 2 * np.pi / ny, 2 * np.pi / max(nz, 1)
    base = np.stack([np.sin(kx * x + 0.3) * np.cos(ky * y), np.cos(kx * x) * np.sin(ky * y + 0.1),
                     np.sin(kz * z + 0.2) * np.cos(kx * x)])[: m.d]
    u = du * (base + 0.3 * rng.uniform(-1, 1, size=(m.d, m.N)))
    rho = m.rho0 + drho * rng.uniform(-1, 1, size=m.N) if m.nse else rng.uniform(0.0, 1.0, size=m.N)
    return rho, u


def circle_mask(n, center, radius):
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (i - center[0]) ** 2 + (j - center[1]) ** 2
    return (r2.reshape(-1) <= radius**2)


def rel_err(a, b, scale=None):
    scale = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / scale)
