"""Pins of the oracle's local derivative outputs (no finite differences in the
scheme): the stress / strain-rate scheme of eq. 4-32-0 with eq. 4-28 and
eq. 4-31, and the grad phi scheme of eq. 4-13.  They are checked against the
exact strain rate of plane Poiseuille flow and of a decaying Taylor-Green
vortex, against central differences of the scheme's own fields (a compressive
wave that exercises the bulk-viscosity block, the NCDE hill), and the
advection-induced error of the grad phi scheme is shown to be first order in
the advection speed."""
import math

import numpy as np
import pytest

from inputs import gaussian_hill_field, grid_coords, taylor_green_2d
from oracle import rmrt_oracle as O


def _poiseuille_state(lat, ny, dy, nu, nu_b, g):
    d = 2 if lat == "Q9" else 3
    if d == 2:
        n, dx, walls = (2, ny, 1), (1.0, dy, 1.0), O.WALL_YM | O.WALL_YP
    else:
        n, dx, walls = (2, 2, ny), (1.0, 1.0, dy), O.WALL_ZM | O.WALL_ZP
    m = O.Model(dict(lattice=lat, n=n, dx=dx, nu=nu, nu_b=nu_b, force=(g, 0.0, 0.0)[:d], wall_faces=walls))
    H = ny * dy
    f = m.step(m.init(np.ones(m.N), np.zeros((d, m.N))), int(2.5 * H * H / nu))
    X, Y, Z = grid_coords(n, dx, centered=True)
    return m, f, (Y if d == 2 else Z), H


@pytest.mark.parametrize("lat,dy,nu_b", [("Q9", 0.5, -1.0), ("Q9", 0.5, 0.3), ("Q19", 2.0, -1.0), ("Q27", 0.5, 0.1)])
def test_poiseuille_strain_rate_and_stress(lat, dy, nu_b):
    """Steady channel: E_xw = g (H - 2 w) / (4 nu) (w the wall-normal axis),
    tau_xw = 2 rho nu E_xw, and no normal strain."""
    nu, g = (0.1 if dy < 1 else 0.5), 1e-5
    m, f, w, H = _poiseuille_state(lat, 12, dy, nu, nu_b, g)
    tau, E = m.local_gradients(f)
    rho, _ = m.macroscopic(f)
    b = 1 if m.d == 2 else 2
    exact = g * (H - 2 * w) / (4 * nu)
    scale = np.abs(exact).max()
    assert np.abs(E[0, b] - exact).max() < 1e-6 * scale
    assert np.abs(E[b, 0] - exact).max() < 1e-6 * scale
    assert np.abs(tau[0, b] - 2 * rho * nu * exact).max() < 1e-6 * 2 * nu * scale
    for a in range(m.d):
        assert np.abs(E[a, a]).max() < 1e-3 * scale


def test_taylor_green_strain_rate_rectangular_full_block():
    """Decaying 2D Taylor-Green vortex on dy = 0.5 dx with a full second-order
    block (nu_b != nu): local strain rate against the exact decayed field."""
    nx, ny, dx, dy = 64, 32, 1.0, 0.5
    m = O.Model(dict(lattice="Q9", n=(nx, ny, 1), dx=(dx, dy, 1.0), nu=0.02, nu_b=0.05, cs2=1.0 / 12.0))
    rho, u, (kx, ky) = taylor_green_2d(nx, ny, dx, dy, 0.01, m.cs2)
    steps = 200
    f = m.step(m.init(rho, u), steps)
    _, E = m.local_gradients(f)
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    U = 0.01 * math.exp(-m.nu * (kx**2 + ky**2) * steps)
    dudx = U * kx * np.sin(kx * X) * np.sin(ky * Y)
    shear = 0.5 * (-U * ky + U * kx * kx / ky) * np.cos(kx * X) * np.cos(ky * Y)
    exact = np.array([[dudx, shear], [shear, -dudx]])
    scale = np.abs(exact).max()
    assert np.abs(E - exact).max() < 5e-3 * scale


def _compressive(nx, nu_b, steps, U=1e-3):
    m = O.Model(dict(lattice="Q9", n=(nx, 4, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=nu_b))
    X, _, _ = grid_coords((nx, 4, 1), (1.0, 0.5, 1.0))
    k = 2 * math.pi / nx
    u0 = np.stack([U * np.sin(k * X), np.zeros_like(X)])
    f = m.step(m.init(np.ones(m.N), u0), steps)
    _, E = m.local_gradients(f)
    _, u = m.macroscopic(f)
    ux = u[0].reshape(4, nx)
    fd = ((np.roll(ux, -1, axis=1) - np.roll(ux, 1, axis=1)) / 2.0).reshape(-1)
    scale = np.abs(fd).max()
    return np.abs(E[0, 0] - fd).max() / scale, np.abs(E[1, 1]).max() / scale


def test_compressive_wave_exercises_the_bulk_block():
    """A 1D compression wave with nu_b != 2 nu / d: E_xx matches the central
    difference of the scheme's own u_x, and the spurious E_yy (zero in the
    flow) decreases linearly with the wavenumber."""
    exx, eyy64 = _compressive(64, 0.15, 30)
    assert exx < 1e-2, exx
    _, eyy128 = _compressive(128, 0.15, 60)
    assert eyy64 < 4e-2
    assert 1.7 < eyy64 / eyy128 < 2.3, (eyy64, eyy128)


def _hill_grad(lat, ux, D=0.01, steps=100, dy=0.5):
    nx, ny = 128, 128
    m = O.Model(dict(lattice=lat, equation="NCDE", n=(nx, ny, 1), dx=(1.0, dy, 1.0), D0=D, D2=0.0,
                     adv=(ux, 0.0, 0.0), rho0=0.0))
    phi0 = gaussian_hill_field(nx, ny, 1.0, dy, 8.0, 64.0, 32.0)
    f = m.init(phi0, None)
    if m.linear:
        f, h = m.step(f, steps, m.init_history(phi0))
        gr = m.local_gradients(f, h)
    else:
        f = m.step(f, steps)
        gr = m.local_gradients(f)
    phi, _ = m.macroscopic(f)
    P = phi.reshape(ny, nx)
    fdx = ((np.roll(P, -1, 1) - np.roll(P, 1, 1)) / 2.0).reshape(-1)
    fdy = ((np.roll(P, -1, 0) - np.roll(P, 1, 0)) / (2.0 * dy)).reshape(-1)
    scale = max(np.abs(fdx).max(), np.abs(fdy).max())
    return np.abs(gr[0] - fdx).max() / scale, np.abs(gr[1] - fdy).max() / scale


@pytest.mark.parametrize("lat", ["Q9", "Q5"])
def test_grad_phi_without_advection(lat):
    """Pure diffusion (D = 0.05): the local grad phi of eq. 4-13 equals the
    central difference of the scheme's own phi to the differencing error."""
    ex, ey = _hill_grad(lat, 0.0, D=0.05)
    assert ex < 1e-2 and ey < 1e-2, (ex, ey)


@pytest.mark.parametrize("lat", ["Q9", "Q5"])
def test_grad_phi_advection_error_is_first_order_in_u(lat):
    """With advection the local scheme carries an error proportional to u_adv
    (a term of order u phi in the first non-equilibrium moment): halving u
    halves it, and the cross-stream component is unaffected."""
    e1, c1 = _hill_grad(lat, 0.05)
    e2, c2 = _hill_grad(lat, 0.025)
    assert 1.6 < e1 / e2 < 2.2, (e1, e2)
    assert e1 < 8e-2
    assert c1 < 1e-2 and c2 < 1e-2
