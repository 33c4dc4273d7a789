"""Pins of the oracle's time stepping against exact solutions of the PDEs that the
scheme recovers (Taylor-Green decay, advected Gaussian hill, plane Poiseuille
flow), against exact invariants (mass and momentum), and a negative control
(a single second-order rate must visibly fail on a rectangular lattice)."""
import math

import numpy as np
import pytest

from inputs import gaussian_hill_field, grid_coords, taylor_green_2d
from oracle import rmrt_oracle as O


def _fit_rate(ts, amps):
    return -np.polyfit(np.asarray(ts, float), np.log(np.abs(amps)), 1)[0]


def _tg2d_rate(m, nx, ny, dx, dy, steps, every):
    rho, u, (kx, ky) = taylor_green_2d(nx, ny, dx, dy, 0.01, m.cs2, noise=0.0)
    f = m.init(rho, u)
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    mode = np.sin(kx * X) * np.cos(ky * Y)
    ts, amps = [], []
    for t in range(0, steps + 1, every):
        if t:
            f = m.step(f, every)
        if t >= every:
            _, uu = m.macroscopic(f)
            ts.append(t)
            amps.append((uu[1] * mode).sum() / (mode * mode).sum())
    return _fit_rate(ts, amps), m.nu * (kx**2 + ky**2)


def test_taylor_green_2d_rate_on_rectangular_q9():
    nx, ny, dx, dy = 64, 32, 1.0, 0.5
    m = O.Model(dict(lattice="Q9", n=(nx, ny, 1), dx=(dx, dy, 1.0), nu=0.02, nu_b=0.05))
    rate, exact = _tg2d_rate(m, nx, ny, dx, dy, 2000, 100)
    assert abs(rate / exact - 1) < 0.01, (rate, exact)


def test_single_second_order_rate_fails_negative_control():
    """Remark II of Sec. IV: one viscosity rate cannot give isotropic viscosity
    on a rectangular lattice.  Planting that mistake in the oracle (all
    second-order rows relaxed with s_nu) must break the decay rate."""
    nx, ny, dx, dy = 64, 32, 1.0, 0.5
    m = O.Model(dict(lattice="Q9", n=(nx, ny, 1), dx=(dx, dy, 1.0), nu=0.02, nu_b=0.05))
    for a in m.rows2d:
        for b in m.rows2d:
            m.S[a, b] = m.s_ab if a == b else 0.0
    rate, exact = _tg2d_rate(m, nx, ny, dx, dy, 1000, 100)
    assert abs(rate / exact - 1) > 0.1, (rate, exact)


@pytest.mark.parametrize("lat", ["Q19", "Q27"])
def test_taylor_green_xz_rate_3d(lat):
    """x-z shear-wave decay with dz = 2 dx exercises the full second-order block."""
    nx, nz, dz, nu = 32, 16, 2.0, 0.02
    m = O.Model(dict(lattice=lat, n=(nx, 1, nz), dx=(1.0, 1.0, dz), nu=nu, nu_b=0.05))
    X, _, Z = grid_coords((nx, 1, nz), (1.0, 1.0, dz))
    kx, kz = 2 * math.pi / nx, 2 * math.pi / (nz * dz)
    U0 = 0.01
    u = np.stack([-U0 * np.cos(kx * X) * np.sin(kz * Z), np.zeros_like(X),
                  U0 * (kx / kz) * np.sin(kx * X) * np.cos(kz * Z)])
    f = m.init(np.ones(m.N), u)
    mode = np.sin(kx * X) * np.cos(kz * Z)
    ts, amps = [], []
    for t in range(100, 1001, 100):
        f = m.step(f, 100)
        _, uu = m.macroscopic(f)
        ts.append(t)
        amps.append((uu[2] * mode).sum() / (mode * mode).sum())
    rate = _fit_rate(ts, amps)
    exact = nu * (kx**2 + kz**2)
    assert abs(rate / exact - 1) < 0.01, (rate, exact)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_mass_and_momentum_conservation(lat):
    d = 2 if lat == "Q9" else 3
    n = (12, 10, 1) if d == 2 else (6, 5, 4)
    dx = (1.0, 0.5, 1.0) if d == 2 else (1.0, 0.5, 2.0)
    F = np.array([2e-5, -1e-5, 3e-5])[:d]
    m = O.Model(dict(lattice=lat, n=n, dx=dx, nu=0.03, nu_b=0.06, force=tuple(F)))
    rng = np.random.default_rng(11)
    f = m.init(1 + 1e-3 * rng.standard_normal(m.N), 0.01 * rng.standard_normal((d, m.N)))
    mass0 = f.sum()
    mom0 = (m.C.T @ f).sum(axis=1)
    for k in range(1, 6):
        f = m.step(f)
        assert abs(f.sum() - mass0) < 1e-12
        np.testing.assert_allclose((m.C.T @ f).sum(axis=1), mom0 + k * m.N * F, rtol=0, atol=1e-12)


def test_gaussian_hill_constant_diffusivity():
    """NCDE with D(phi) = D0 (D2 = 0): advected spreading Gaussian (eq. 4-15)."""
    nx, ny, dx, dy = 128, 128, 1.0, 0.5
    D, adv, sigma = 0.01, (0.05, 0.02), 8.0
    m = O.Model(dict(lattice="Q9", equation="NCDE", n=(nx, ny, 1), dx=(dx, dy, 1.0),
                     D0=D, D2=0.0, adv=adv + (0.0,), rho0=0.0))
    xc, yc = 64.0, 32.0
    phi0 = gaussian_hill_field(nx, ny, dx, dy, sigma, xc, yc)
    f = m.init(phi0, None)
    steps = 400
    f = m.step(f, steps)
    phi, _ = m.macroscopic(f)
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    exact = O.gaussian_hill(X, Y, steps, sigma, D, xc, yc, adv, nx * dx, ny * dy)
    l2 = np.sqrt(((phi - exact) ** 2).sum() / (exact**2).sum())
    assert l2 < 5e-3, l2
    assert abs(phi.sum() - phi0.sum()) < 1e-11


def _poiseuille(lat, ny, dy, nu, g, steps):
    d = 2 if lat == "Q9" else 3
    if d == 2:
        n, dx, walls = (2, ny, 1), (1.0, dy, 1.0), O.WALL_YM | O.WALL_YP
    else:
        n, dx, walls = (2, 2, ny), (1.0, 1.0, dy), O.WALL_ZM | O.WALL_ZP
    m = O.Model(dict(lattice=lat, n=n, dx=dx, nu=nu, force=(g, 0.0, 0.0)[:d], wall_faces=walls))
    f = m.init(np.ones(m.N), np.zeros((d, m.N)))
    f = m.step(f, steps)
    rho, u = m.macroscopic(f)
    X, Y, Z = grid_coords(n, dx, centered=True)
    yc = Y if d == 2 else Z
    H = ny * dy
    return m, f, rho, u, O.poiseuille(yc, H, g, nu)


@pytest.mark.parametrize("lat,dy", [("Q9", 0.5), ("Q27", 0.5), ("Q19", 2.0)])
def test_poiseuille_profile_with_bounce_back(lat, dy):
    """Steady profile error of halfway bounce-back is O(dy^2): 4x smaller
    when the channel has twice the nodes at the same lattice viscosity."""
    nu, g = 0.03 if dy < 1 else 0.3, 1e-5
    errs = []
    for ny in (12, 24):
        H = ny * dy
        steps = int(1.2 * H * H / nu) + 200
        m, f, rho, u, exact = _poiseuille(lat, ny, dy, nu, g, steps)
        errs.append(np.abs(u[0] - exact).max() / exact.max())
        assert np.abs(u[1:]).max() < 1e-10
    assert errs[1] < 0.01, errs
    assert 3.6 < errs[0] / errs[1] < 4.4, errs


def test_nonequilibrium_second_moment_matches_eq_4_34_at_steady_state():
    """At a steady Poiseuille flow the second moment of f - f_eq equals eq. 4-34
    evaluated with the exact velocity gradient (interior nodes)."""
    ny, dy, nu, g = 16, 0.5, 0.1, 1e-5
    H = ny * dy
    m, f, rho, u, exact = _poiseuille("Q9", ny, dy, nu, g, int(2 * H * H / nu))
    feq, F, G, _ = m.distributions(f)
    fne = (f + 0.5 * F) - feq                                  # f = fbar + dt F / 2 (eq. 2-3)
    m2 = np.einsum("ja,jb,jn->abn", m.C, m.C, fne)
    _, Y, _ = grid_coords(m.shape, (1.0, dy, 1.0), centered=True)
    dudy = g * (H - 2 * Y) / (2 * nu)
    uex = np.stack([O.poiseuille(Y, H, g, nu), np.zeros_like(Y)])
    mne = m.m2_ne(rho, uex)
    interior = (Y > 2 * dy) & (Y < H - 2 * dy)
    scale = np.abs(rho * nu * dudy).max()
    assert np.abs(m2[0, 1, interior] - mne[0, 1, interior]).max() < 0.02 * scale
    assert np.abs(m2[0, 0, interior] - mne[0, 0, interior]).max() < 0.02 * scale


def test_q27_with_zero_corner_weight_reduces_to_q19():
    """With omega_19 = 0 the rD3Q27 model never populates its corners and its
    other 19 populations evolve exactly as the rD3Q19 model (Sec. III: rD3Q19
    is rD3Q27 with omega_19 = 0)."""
    prm = dict(n=(6, 5, 4), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.07, force=(1e-5, 2e-5, 0.0))
    m19 = O.Model(dict(prm, lattice="Q19"))
    m27 = O.Model(dict(prm, lattice="Q27", w_corner=0.0))
    rng = np.random.default_rng(13)
    rho = 1 + 1e-3 * rng.standard_normal(m19.N)
    u = 0.02 * rng.standard_normal((3, m19.N))
    f19 = m19.step(m19.init(rho, u), 6)
    f27 = m27.step(m27.init(rho, u), 6)
    np.testing.assert_allclose(f27[:19], f19, rtol=0, atol=1e-13)
    assert np.abs(f27[19:]).max() < 1e-13
