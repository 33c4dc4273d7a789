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


# ---------------------------------------------------------------------------
# Light cones: after k steps a node's populations depend only on the initial
# state within k nodes per axis (|e_ja| <= 1 and the collision is local), so
# the oracle can evolve a (2k+1)-wide sub-box around the node instead of the
# whole domain.  Cut faces of the sub-box are bounce-back walls; the wrong
# data they give travels one node per step and never reaches the centre.  (A
# cut face must not wrap: next to a wall face its wrapped populations would
# land on the wall row, inside the cone.)  Faces of the domain that are walls
# stay walls, and an axis the domain is at most 2k+1 nodes long on is kept
# whole with its own boundary.  The cone narrows as steps are taken, so the
# box is cropped in stages.
# ---------------------------------------------------------------------------

def _axis_window(n, centre, half, wall_lo, wall_hi):
    """Indices of a window of half-width `half` around `centre` on an axis of n
    nodes (wrapping through a periodic face), the window's wall flags (a cut
    face is a wall) and the centre's position in it."""
    if n <= 2 * half + 1:
        return np.arange(n), wall_lo, wall_hi, centre
    lo, hi = centre - half, centre + half
    if wall_lo:
        lo = max(lo, 0)
    if wall_hi:
        hi = min(hi, n - 1)
    return np.arange(lo, hi + 1) % n, True, True, centre - lo


def lightcone_oracle(prm, rho, u, node, k):
    """Oracle populations (q,) at `node` = (x, y, z) after k steps of the domain
    with parameters prm (its n and wall_faces) from the initial fields rho (N,)
    and u (d, N) or None, evolving only the node's light cone."""
    n = [int(v) for v in prm["n"]]
    walls = int(prm.get("wall_faces", 0))
    d = 2 if n[2] == 1 and prm.get("lattice", "Q9") in ("Q9", "Q5") else 3
    # current box: global indices per axis, wall flags, the node's position
    idx = [np.arange(n[a]) for a in range(3)]
    wlo = [bool(walls & (1 << (2 * a))) for a in range(3)]
    whi = [bool(walls & (1 << (2 * a + 1))) for a in range(3)]
    pos = list(node)
    f = None
    left = k
    while True:
        half = left
        sub_idx, sub_lo, sub_hi, sub_pos = [], [], [], []
        for a in range(3):
            if a >= d:
                sub_idx.append(np.arange(1)), sub_lo.append(False), sub_hi.append(False), sub_pos.append(0)
                continue
            w, l, h, p = _axis_window(len(idx[a]), pos[a], half, wlo[a], whi[a])
            sub_idx.append(w), sub_lo.append(l), sub_hi.append(h), sub_pos.append(p)
        shape = [len(w) for w in sub_idx]
        # node indices (x-fastest) of the sub-box within the current box
        Z, Y, X = np.meshgrid(sub_idx[2], sub_idx[1], sub_idx[0], indexing="ij")
        cur_n = [len(i) for i in idx]
        lin = (X + cur_n[0] * (Y + cur_n[1] * Z)).reshape(-1)
        sub_walls = sum((1 << (2 * a)) * sub_lo[a] + (1 << (2 * a + 1)) * sub_hi[a] for a in range(3))
        m = O.Model(dict(prm, n=tuple(shape), wall_faces=sub_walls))
        if f is None:
            uu = None if u is None else np.asarray(u).reshape(-1, len(rho))[:, lin]
            f = m.init(np.asarray(rho)[lin], uu)
        else:
            f = f[:, lin]
        # carry the global coordinates along
        idx = [idx[a][sub_idx[a]] for a in range(3)]
        wlo, whi, pos = sub_lo, sub_hi, sub_pos
        if left == 0:
            break
        s = max(1, (left + 1) // 2)
        f = m.step(f, s)
        left -= s
    centre = pos[0] + shape[0] * (pos[1] + shape[1] * pos[2])
    return f[:, centre], m
