"""Seeded initial fields, domain lists and geometries.

Positions: node (i, j, k) sits at (i dx, j dy, k dz) for periodic problems and
at ((i + 1/2) dx, (j + 1/2) dy, (k + 1/2) dz) for walled channels, so that
halfway bounce-back puts the walls at 0 and n dx.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "grid_coords", "taylor_green_2d", "taylor_green_3d", "gaussian_hill_field",
    "channel_batch", "obstacle_channel", "obstacle_channels", "conv_problem",
    "random_state",
]


def grid_coords(n, dx, centered=False):
    """Physical coordinates of every node, x-fastest, each of shape (N,)."""
    nx, ny, nz = n
    off = 0.5 if centered else 0.0
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = (i.reshape(-1) + off) * dx[0]
    Y = (j.reshape(-1) + off) * dx[1]
    Z = (k.reshape(-1) + off) * dx[2]
    return X, Y, Z


def taylor_green_2d(nx, ny, dx, dy, U0, cs2, noise=0.0, seed=1):
    """Decaying 2D Taylor-Green vortex on a periodic nx x ny box.

    u = -U0 cos(kx x) sin(ky y), v = U0 (kx/ky) sin(kx x) cos(ky y),
    rho = 1 + p / cs2 + xi with p = -(U0^2/4)[cos 2kx x + (kx/ky)^2 cos 2ky y]
    and xi ~ U(-noise, noise)."""
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    kx = 2 * math.pi / (nx * dx)
    ky = 2 * math.pi / (ny * dy)
    u = np.stack([-U0 * np.cos(kx * X) * np.sin(ky * Y),
                  U0 * (kx / ky) * np.sin(kx * X) * np.cos(ky * Y)])
    p = -(U0**2 / 4.0) * (np.cos(2 * kx * X) + (kx / ky) ** 2 * np.cos(2 * ky * Y))
    rho = 1.0 + p / cs2
    if noise > 0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    return rho, u, (kx, ky)


def taylor_green_3d(n, dx, U0, cs2, with_pressure=True):
    """3D Taylor-Green vortex on a periodic box (physical size n_a dx_a).

    u = U0 sin kx cos ky cos kz, v = -U0 cos kx sin ky cos kz, w = 0,
    rho = 1 + (U0^2/16)(cos 2kx + cos 2ky)(cos 2kz + 2) / cs2."""
    X, Y, Z = grid_coords(n, dx)
    kx = 2 * math.pi / (n[0] * dx[0])
    ky = 2 * math.pi / (n[1] * dx[1])
    kz = 2 * math.pi / (n[2] * dx[2])
    u = np.stack([U0 * np.sin(kx * X) * np.cos(ky * Y) * np.cos(kz * Z),
                  -U0 * np.cos(kx * X) * np.sin(ky * Y) * np.cos(kz * Z),
                  np.zeros_like(X)])
    if with_pressure:
        rho = 1.0 + (U0**2 / 16.0) * (np.cos(2 * kx * X) + np.cos(2 * ky * Y)) * (np.cos(2 * kz * Z) + 2.0) / cs2
    else:
        rho = np.ones_like(X)
    return rho, u, (kx, ky, kz)


def gaussian_hill_field(nx, ny, dx, dy, sigma, xc, yc, peak=1.0):
    """phi = peak exp(-|x - xc|^2 / (2 sigma^2)) with physical centre (xc, yc)."""
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    return peak * np.exp(-((X - xc) ** 2 + (Y - yc) ** 2) / (2.0 * sigma**2))


def channel_batch(seed=4, nd=64, nmin=32, nmax=256, Uc=0.02):
    """Force-driven rectangular channels: walls on the y and z faces, periodic x.

    Per domain: n_x, n_y, n_z ~ U{nmin..nmax}; dy, dz ~ U{0.5, 1, 2}; nu ~ U[0.01, 0.1];
    nu_b = 2 nu / 3; body force g = 8 nu Uc / min(H_y, H_z)^2 along x."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(nd):
        n = tuple(int(v) for v in rng.integers(nmin, nmax + 1, size=3))
        dy, dz = (float(v) for v in rng.choice([0.5, 1.0, 2.0], size=2))
        nu = float(rng.uniform(0.01, 0.1))
        H = min(n[1] * dy, n[2] * dz)
        g = 8.0 * nu * Uc / H**2
        out.append(dict(n=n, dx=(1.0, dy, dz), nu=nu, nu_b=2.0 * nu / 3.0, force=(g, 0.0, 0.0)))
    return out


def _shapes_overlap(a, b, gap):
    # conservative: bounding circles plus a gap
    return math.hypot(a["x"] - b["x"], a["y"] - b["y"]) < a["R"] + b["R"] + gap


def obstacle_channel(seed, nx=512, ny=256, dy=0.5, Ut=0.03, kmax=8, rmin=4.0, rmax=12.0,
                     wall_gap=8.0, xmin=64.0, xmax=448.0, Re_range=(10.0, 100.0)):
    """One steady-channel geometry: 1..kmax circles or rectangles, walls at y faces.

    Returns dict(solid (N,) bool, Re, nu, force, shapes).  Sizes are physical (dx = 1)."""
    rng = np.random.default_rng(seed)
    H = ny * dy
    Re = float(rng.uniform(*Re_range))
    nu = Ut * H / Re
    K = int(rng.integers(1, kmax + 1))
    shapes = []
    tries = 0
    while len(shapes) < K and tries < 1000:
        tries += 1
        kind = "circle" if rng.random() < 0.5 else "rect"
        if kind == "circle":
            r = float(rng.uniform(rmin, rmax))
            s = dict(kind=kind, r=r, R=r)
        else:
            hx, hy = (float(v) for v in rng.uniform(rmin, rmax, size=2))
            s = dict(kind=kind, hx=hx, hy=hy, R=math.hypot(hx, hy))
        ext_y = s["r"] if kind == "circle" else s["hy"]
        lo, hi = wall_gap + ext_y, H - wall_gap - ext_y
        if hi <= lo:
            continue
        s["x"] = float(rng.uniform(xmin, xmax))
        s["y"] = float(rng.uniform(lo, hi))
        if any(_shapes_overlap(s, t, 2.0) for t in shapes):
            continue
        shapes.append(s)
    X, Y, _ = grid_coords((nx, ny, 1), (1.0, dy, 1.0), centered=True)
    solid = np.zeros(nx * ny, dtype=bool)
    for s in shapes:
        if s["kind"] == "circle":
            solid |= (X - s["x"]) ** 2 + (Y - s["y"]) ** 2 <= s["r"] ** 2
        else:
            solid |= (np.abs(X - s["x"]) <= s["hx"]) & (np.abs(Y - s["y"]) <= s["hy"])
    g = 8.0 * nu * Ut / H**2
    return dict(solid=solid, Re=Re, nu=nu, force=(g, 0.0, 0.0), shapes=shapes,
                n=(nx, ny, 1), dx=(1.0, dy, 1.0), H=H, Ut=Ut)


def obstacle_channels(seeds, **kw):
    return [obstacle_channel(s, **kw) for s in seeds]


def conv_problem(seed, B=2, H=16, W=24, cin=3, chid=32, cout=3, scale=0.5):
    """Random input batch (B, H, W, cin) and layer weights for the conv surrogate tests."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, H, W, cin))
    chans = [cin, chid, chid, chid, cout]
    Ws, bs = [], []
    for li in range(4):
        fan_in = 9 * chans[li]
        Ws.append(rng.standard_normal((chans[li + 1], 3, 3, chans[li])) * scale / math.sqrt(fan_in))
        bs.append(rng.standard_normal(chans[li + 1]) * 0.1)
    target = rng.standard_normal((B, H, W, cout))
    mask = (rng.random((B, H, W)) > 0.2).astype(np.float64)
    return dict(x=x, W=Ws, b=bs, target=target, mask=mask)


def random_state(q, N, seed, scale=1e-3):
    """Small random deviations, shape (q, N), for collision-only checks."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=(q, N))
