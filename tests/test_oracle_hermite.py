"""Pins of the oracle's Hermite-moment and central-Hermite-moment collisions
(eq. 5-1-1 and 5-1-2, reading A26): H against the textbook tensor-product
Hermite moments (H_0 = 1, H_1 = xi, H_2 = xi^2 - cs2) of c_j and of c_j - u,
the equivalence with the raw-moment model when Sbar = N S N^-1, the special
case of equal rates (every basis gives the raw step), central-Hermite at
rest equal to Hermite, the moment and velocity routes, exact mass and
momentum balances with a body force, a Hermite step that differs from the
raw one once the higher-order rate differs from the second-order ones, and
the Taylor-Green viscous decay rate on rectangular lattices."""
import math

import numpy as np
import pytest

from gpu_util import random_fields
from inputs import grid_coords
from oracle import rmrt_oracle as O

RECT = {"Q9": dict(lattice="Q9", n=(9, 7, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.09, s_hi=1.3,
                   force=(2e-5, -1e-5, 0.0)),
        "Q19": dict(lattice="Q19", n=(5, 4, 3), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.02, s_hi=1.4,
                    force=(1e-5, 0.0, 3e-6)),
        "Q27": dict(lattice="Q27", n=(5, 4, 3), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.02, s_hi=1.2,
                    force=(1e-5, 0.0, 3e-6))}
CENTRAL_OK = ("Q9", "Q27")


def _brute(m, f, u):
    """sum_j prod_axis H_e(c_ja - u_a) f_j for every moment row (e per axis)."""
    n = f.shape[1]
    out = np.zeros((m.q, n))
    for i, ex in enumerate(m.exps):
        w = np.ones((m.q, n))
        for a, e in enumerate(ex):
            xi = m.C[:, a][:, None] - u[a][None, :]
            w = w * (1.0 if e == 0 else (xi if e == 1 else xi * xi - m.cs2))
        out[i] = (w * f).sum(axis=0)
    return out


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_basis_gives_textbook_hermite_moments(lat):
    m = O.Model(dict(RECT[lat], hermite=True))
    rng = np.random.default_rng(2)
    f = rng.uniform(0.0, 1.0, (m.q, 5))
    got = m.hermite_matrix() @ (m.M @ f)
    np.testing.assert_allclose(got, _brute(m, f, np.zeros((m.d, 5))), rtol=1e-13, atol=1e-15)
    if lat in CENTRAL_OK:
        mc = O.Model(dict(RECT[lat], hermite=True, central=True))
        u = rng.uniform(-0.3, 0.3, (m.d, 5))
        got = np.einsum("ikn,kn->in", mc.basis_matrix(u), mc.M @ f)
        np.testing.assert_allclose(got, _brute(mc, f, u), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_similar_relaxation_matrix_gives_the_raw_model(lat):
    """With Sbar = H S H^-1 (per node with the central shift), eq. 5-1-2 says
    Lambda is the raw model's."""
    raw = O.Model(RECT[lat])
    for central in ((False, True) if lat in CENTRAL_OK else (False,)):
        her = O.Model(dict(RECT[lat], hermite=True, central=central))
        rho, u = random_fields(raw, 3)
        f = raw.step(raw.init(rho, u), 3)      # away from equilibrium: S matters
        _, uu = raw.macroscopic(f)
        N = her.basis_matrix(uu)
        out = np.zeros_like(f)
        for j in range(raw.N):
            her.S_central = N[:, :, j] @ raw.S @ np.linalg.inv(N[:, :, j])
            sel = np.array([j])
            out[:, j] = her.collide(f[:, sel], sel=sel)[:, 0]
        np.testing.assert_allclose(out, raw.collide(f), atol=1e-14)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_equal_rates_give_the_raw_model(lat):
    """c = 1, cs2 = 1/3, nu_b = 2 nu / d and s_hi = s_nu: every non-conserved
    rate is s_nu and the conserved moments are at equilibrium, so the basis
    does not matter."""
    n = (7, 6, 1) if lat == "Q9" else (4, 4, 3)
    prm = dict(lattice=lat, n=n, dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0, nu=0.03, force=(1e-5, 2e-6, 0.0))
    raw = O.Model(prm)
    rho, u = random_fields(raw, 5)
    f = raw.step(raw.init(rho, u), 3)
    for central in ((False, True) if lat in CENTRAL_OK else (False,)):
        her = O.Model(dict(prm, hermite=True, central=central))
        np.testing.assert_allclose(her.collide(f), raw.collide(f), atol=1e-15)


@pytest.mark.parametrize("lat", CENTRAL_OK)
def test_central_hermite_at_rest_is_hermite(lat):
    """u = 0 exactly: N(0) = I, so central-Hermite and Hermite take the same step."""
    her = O.Model(dict(RECT[lat], hermite=True, force=(0.0, 0.0, 0.0)))
    ch = O.Model(dict(RECT[lat], hermite=True, central=True, force=(0.0, 0.0, 0.0)))
    rng = np.random.default_rng(4)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, her.N)
    f = her.init(rho, np.zeros((her.d, her.N)))
    noise = 1e-3 * rng.uniform(-1, 1, f.shape)
    mn = her.M @ noise
    mn[[her.row0] + her.rows1] = 0.0
    f = f + np.linalg.solve(her.M, mn)
    _, u = her.macroscopic(f)
    assert np.abs(u).max() < 1e-16
    np.testing.assert_allclose(ch.collide(f), her.collide(f), atol=1e-15)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_routes_balances_and_difference_from_raw(lat):
    for central in ((False, True) if lat in CENTRAL_OK else (False,)):
        m = O.Model(dict(RECT[lat], hermite=True, central=central, wall_faces=4 | 8))
        rho, u = random_fields(m, 6)
        f = m.step(m.init(rho, u), 3)      # away from equilibrium: S matters
        np.testing.assert_allclose(m.collide(f), m.collide_velocity_space(f), atol=1e-15)
        # s_hi differs from the second-order rates: the Hermite basis couples the
        # fourth-order moments to the second-order non-equilibrium
        raw = O.Model(dict(RECT[lat], central=central, wall_faces=4 | 8))
        assert np.abs(m.collide(f) - raw.collide(f)).max() > 1e-9
        g = m.collide(f)
        assert abs(g.sum() - f.sum()) < 1e-13
        np.testing.assert_allclose((m.C.T @ g).sum(axis=1) - (m.C.T @ f).sum(axis=1), m.N * m.force, atol=1e-15)


def _tg_rate(lat, central):
    nu = 0.02
    if lat == "Q9":
        n, dx, ax = (48, 24, 1), (1.0, 0.5, 1.0), 1
    else:
        n, dx, ax = (24, 1, 12), (1.0, 1.0, 2.0), 2
    m = O.Model(dict(lattice=lat, n=n, dx=dx, nu=nu, nu_b=0.05, s_hi=1.5, hermite=True, central=central))
    coords = grid_coords(n, dx)
    kx, ky = 2 * math.pi / (n[0] * dx[0]), 2 * math.pi / (n[ax] * dx[ax])
    U0 = 0.01
    u = np.zeros((m.d, m.N))
    u[0] = -U0 * np.cos(kx * coords[0]) * np.sin(ky * coords[ax])
    u[m.d - 1] = U0 * (kx / ky) * np.sin(kx * coords[0]) * np.cos(ky * coords[ax])
    f = m.init(np.ones(m.N), u)
    phase = np.exp(-1j * (kx * coords[0] + ky * coords[ax]))
    ts, amps = [], []
    for t in range(100, 801, 100):
        f = m.step(f, 100)
        _, uu = m.macroscopic(f)
        ts.append(t)
        amps.append(abs((uu[m.d - 1] * phase).sum()))
    rate = -np.polyfit(np.asarray(ts, float), np.log(np.abs(amps)), 1)[0]
    return rate / (nu * (kx**2 + ky**2))


@pytest.mark.parametrize("lat,central", [("Q9", False), ("Q9", True), ("Q27", False), ("Q19", False)])
def test_taylor_green_decay_rate(lat, central):
    assert abs(_tg_rate(lat, central) - 1) < 0.01


def test_refused_where_not_built():
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q9", equation="NCDE", n=(4, 4, 1), D0=0.01, hermite=True))
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q19", n=(4, 4, 4), nu=0.02, hermite=True, central=True))
