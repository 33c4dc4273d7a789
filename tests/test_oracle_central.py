"""Pins of the oracle's central-moment (cascaded) collision (eq. 5-1-1 and
5-1-2, reading A25): the shift N(u) against the textbook definition of central
moments, the equivalence Lambda = M^-1 N^-1 Sbar N M with the raw-moment model
when Sbar = N S N^-1, the special cases u = 0 and equal rates on the standard
lattice (both reduce to the raw model), the moment and velocity routes, exact
mass and momentum balances with a body force, the Taylor-Green viscous decay
rate on rectangular lattices and a shear wave riding on a uniform flow."""
import math

import numpy as np
import pytest

from gpu_util import random_fields
from inputs import grid_coords, taylor_green_2d
from oracle import rmrt_oracle as O

RECT = {"Q9": dict(lattice="Q9", n=(9, 7, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.09, force=(2e-5, -1e-5, 0.0)),
        "Q27": dict(lattice="Q27", n=(5, 4, 3), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.02, force=(1e-5, 0.0, 3e-6))}


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_shift_gives_textbook_central_moments(lat):
    m = O.Model(dict(RECT[lat], central=True))
    rng = np.random.default_rng(1)
    f = rng.uniform(0.0, 1.0, (m.q, 6))
    u = rng.uniform(-0.3, 0.3, (m.d, 6))
    got = np.einsum("ikn,kn->in", m.shift_matrix(u), m.M @ f)
    brute = np.zeros_like(got)
    for i, ex in enumerate(m.exps):
        w = np.ones((m.q, 6))
        for a, e in enumerate(ex):
            w = w * (m.C[:, a][:, None] - u[a][None, :]) ** e
        brute[i] = (w * f).sum(axis=0)
    np.testing.assert_allclose(got, brute, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_similar_relaxation_matrix_gives_the_raw_model(lat):
    """With Sbar = N S N^-1 per node, eq. 5-1-2 says Lambda is the raw model's."""
    raw = O.Model(RECT[lat])
    cen = O.Model(dict(RECT[lat], central=True))
    rho, u = random_fields(raw, 3)
    f = raw.step(raw.init(rho, u), 3)      # away from equilibrium: S matters
    _, uu = raw.macroscopic(f)
    N = cen.shift_matrix(uu)
    out = np.zeros_like(f)
    for j in range(raw.N):
        cen.S_central = N[:, :, j] @ raw.S @ np.linalg.inv(N[:, :, j])
        sel = np.array([j])
        out[:, j] = cen.collide(f[:, sel], sel=sel)[:, 0]
    np.testing.assert_allclose(out, raw.collide(f), atol=1e-14)


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_at_rest_the_shift_is_the_identity(lat):
    """u = 0 exactly (the half-force correction cancels the first moment):
    N(0) = I, so both models take the same step."""
    raw = O.Model(RECT[lat])
    cen = O.Model(dict(RECT[lat], central=True))
    rng = np.random.default_rng(4)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, raw.N)
    # a non-equilibrium state with zero momentum: equilibrium plus a random part
    # orthogonal to the conserved moments (projected out through M)
    f = raw.init(rho, np.zeros((raw.d, raw.N)))
    noise = 1e-3 * rng.uniform(-1, 1, f.shape)
    mn = raw.M @ noise
    mn[[raw.row0] + raw.rows1] = 0.0
    f = f + np.linalg.solve(raw.M, mn)
    _, u = raw.macroscopic(f)
    assert np.abs(u).max() < 1e-16
    np.testing.assert_allclose(cen.collide(f), raw.collide(f), atol=1e-15)


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_equal_rates_on_the_standard_lattice_give_the_raw_model(lat):
    """c = 1, cs2 = 1/3, nu_b = 2 nu / d and s_hi = s_nu: every rate is s_nu,
    Sbar = s_nu I on the non-conserved moments, and N^-1 Sbar N = Sbar."""
    n = (7, 6, 1) if lat == "Q9" else (4, 4, 3)
    prm = dict(lattice=lat, n=n, dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0, nu=0.03, force=(1e-5, 2e-6, 0.0))
    raw, cen = O.Model(prm), O.Model(dict(prm, central=True))
    rho, u = random_fields(raw, 5)
    f = raw.step(raw.init(rho, u), 3)
    np.testing.assert_allclose(cen.collide(f), raw.collide(f), atol=1e-15)


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_routes_and_balances(lat):
    m = O.Model(dict(RECT[lat], central=True, wall_faces=4 | 8))
    rho, u = random_fields(m, 6)
    f = m.step(m.init(rho, u), 3)          # away from equilibrium: S matters
    np.testing.assert_allclose(m.collide(f), m.collide_velocity_space(f), atol=1e-15)
    # the raw and central steps differ once u != 0 and the rates are not all equal
    raw = O.Model(dict(RECT[lat], wall_faces=4 | 8))
    assert np.abs(m.collide(f) - raw.collide(f)).max() > 1e-9
    g = m.collide(f)
    assert abs(g.sum() - f.sum()) < 1e-13
    np.testing.assert_allclose((m.C.T @ g).sum(axis=1) - (m.C.T @ f).sum(axis=1), m.N * m.force, atol=1e-15)


def _tg_rate(lat, central, U=(0.0, 0.0)):
    """Decay of a 2D shear wave (x-y on rD2Q9 dy = dx/2, x-z on rD3Q27 dz = 2 dx),
    optionally riding on a uniform flow U."""
    nu = 0.02
    if lat == "Q9":
        n, dx = (48, 24, 1), (1.0, 0.5, 1.0)
        ax = 1
    else:
        n, dx = (24, 1, 12), (1.0, 1.0, 2.0)
        ax = 2
    m = O.Model(dict(lattice=lat, n=n, dx=dx, nu=nu, nu_b=0.05, central=central))
    coords = grid_coords(n, dx)
    kx, ky = 2 * math.pi / (n[0] * dx[0]), 2 * math.pi / (n[ax] * dx[ax])
    U0 = 0.01
    u = np.zeros((m.d, m.N))
    u[0] = -U0 * np.cos(kx * coords[0]) * np.sin(ky * coords[ax]) + U[0]
    u[m.d - 1] = U0 * (kx / ky) * np.sin(kx * coords[0]) * np.cos(ky * coords[ax]) + U[1]
    f = m.init(np.ones(m.N), u)
    # |Fourier coefficient| of the wave: unchanged when a uniform flow translates it
    phase = np.exp(-1j * (kx * coords[0] + ky * coords[ax]))
    ts, amps = [], []
    for t in range(100, 801, 100):
        f = m.step(f, 100)
        _, uu = m.macroscopic(f)
        ts.append(t)
        amps.append(abs(((uu[m.d - 1] - U[1]) * phase).sum()))
    rate = -np.polyfit(np.asarray(ts, float), np.log(np.abs(amps)), 1)[0]
    return rate / (nu * (kx**2 + ky**2))


@pytest.mark.parametrize("lat", ["Q9", "Q27"])
def test_taylor_green_decay_rate(lat):
    assert abs(_tg_rate(lat, True) - 1) < 0.01


def test_shear_wave_on_a_uniform_flow_decays_at_nu_k2():
    """Galilean invariance of the recovered viscosity: the wave's decay rate with a
    uniform flow of 0.05 underneath stays within 2% of nu |k|^2."""
    assert abs(_tg_rate("Q9", True, U=(0.05, 0.0)) - 1) < 0.02
