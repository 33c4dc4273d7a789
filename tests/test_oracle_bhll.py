"""Pins of the oracle's BHLL-moment collision (the orthogonal rD2Q9 basis of
Sec. V, eq. Md2q9-2 / Md2q9-3, with eq. 5-1-2; reading A27): the basis
against the printed N_BHLL and the orthogonality of its rows, the textbook
square-lattice MRT collision (Lallemand-Luo moments written from their
definitions, diagonal rates) at a = 1, the raw model under Sbar = N S N^-1,
the raw model at equal rates, the moment and velocity routes, exact mass and
momentum balances with a body force, a step that differs from the raw one
once s_hi differs from the second-order block, and the Taylor-Green viscous
decay rate on a rectangular lattice."""
import math

import numpy as np
import pytest

from golden_util import read_matrix
from gpu_util import random_fields
from inputs import grid_coords
from oracle import rmrt_oracle as O

RECT = dict(lattice="Q9", n=(9, 7, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.09, s_hi=1.3,
            force=(2e-5, -1e-5, 0.0))


@pytest.mark.parametrize("a", [0.5, 0.8, 2.0])
def test_basis_is_the_printed_matrix(a):
    m = O.Model(dict(RECT, dx=(1.0, a, 1.0), bhll=True))
    np.testing.assert_allclose(m.bhll_matrix(), read_matrix("bhll_N.txt", dict(a=a)), rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("dx", [(1.0, 0.5), (2.0, 1.0), (0.5, 0.8), (1.0, 1.0)])
def test_basis_rows_are_orthogonal(dx):
    """The BHLL moments are an orthogonal basis of velocity space: the rows of
    N M are mutually orthogonal for any spacing, c_x included."""
    m = O.Model(dict(RECT, dx=(dx[0], dx[1], 1.0), bhll=True))
    B = m.bhll_matrix() @ m.M
    G = B @ B.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-12 * np.abs(np.diag(G)).max()


def _lallemand_luo(C):
    """Textbook square-lattice MRT moments (rho, e, eps, jx, qx, jy, qy, pxx,
    pxy) as polynomials of the velocities c_j (rows) -- not built from N_BHLL."""
    cx, cy = C[:, 0], C[:, 1]
    c2 = cx * cx + cy * cy
    return np.stack([np.ones_like(cx), -4 + 3 * c2, 4 - 10.5 * c2 + 4.5 * c2 * c2,
                     cx, (-5 + 3 * c2) * cx, cy, (-5 + 3 * c2) * cy, cx * cx - cy * cy, cx * cy])


def test_square_lattice_is_the_textbook_mrt():
    """At a = 1, cs2 = 1/3 the BHLL relaxation matrix is diagonal, with the
    shear rate 1 / (1/2 + nu / cs2) on p_xx and p_xy, the bulk rate of eq.
    4-31 on e and s_hi on q and epsilon; the step equals the textbook MRT
    collision f - M^-1 S (M f - M f_eq) with those rates."""
    nu, nu_b, s_hi = 0.04, 0.11, 1.3
    m = O.Model(dict(lattice="Q9", n=(7, 6, 1), nu=nu, nu_b=nu_b, s_hi=s_hi, cs2=1.0 / 3.0, bhll=True))
    Sb = m.S_bhll
    noncons = [3, 4, 5, 6, 7, 8]
    sub = Sb[np.ix_(noncons, noncons)]
    assert np.abs(sub - np.diag(np.diag(sub))).max() < 1e-14
    s_nu = 1.0 / (0.5 + nu / m.cs2)
    s_e = 1.0 / (0.5 + 2 * nu_b / (1.0 - m.cs2))
    np.testing.assert_allclose(np.diag(Sb)[[3, 4, 5, 6, 7, 8]], [s_e, s_nu, s_nu, s_hi, s_hi, s_hi], rtol=1e-13)
    rho, u = random_fields(m, 2)
    f = m.step(m.init(rho, u), 3)          # away from equilibrium
    feq, _, _, _ = m.distributions(f)
    ML = _lallemand_luo(m.C)
    SL = np.diag([0.0, s_e, s_hi, 0.0, s_hi, 0.0, s_hi, s_nu, s_nu])
    want = f - np.linalg.solve(ML, SL @ (ML @ (f - feq)))
    np.testing.assert_allclose(m.collide(f), want, atol=1e-15)


def test_similar_relaxation_matrix_gives_the_raw_model():
    """Sbar = N S N^-1 with every coupling between orders kept: eq. 5-1-2 says
    Lambda is the raw model's."""
    raw = O.Model(RECT)
    bh = O.Model(dict(RECT, bhll=True))
    N = bh.bhll_matrix()
    bh.S_central = N @ raw.S @ np.linalg.inv(N)
    rho, u = random_fields(raw, 3)
    f = raw.step(raw.init(rho, u), 3)
    np.testing.assert_allclose(bh.collide(f), raw.collide(f), atol=1e-15)


def test_equal_rates_give_the_raw_model():
    """c = 1, cs2 = 1/3, nu_b = 2 nu / d and s_hi = s_nu: every non-conserved
    rate is s_nu and the conserved moments are at equilibrium."""
    prm = dict(lattice="Q9", n=(7, 6, 1), cs2=1.0 / 3.0, nu=0.03, force=(1e-5, 2e-6, 0.0))
    raw = O.Model(prm)
    rho, u = random_fields(raw, 5)
    f = raw.step(raw.init(rho, u), 3)
    np.testing.assert_allclose(O.Model(dict(prm, bhll=True)).collide(f), raw.collide(f), atol=1e-15)


def test_routes_balances_and_difference_from_raw():
    m = O.Model(dict(RECT, bhll=True, wall_faces=4 | 8))
    rho, u = random_fields(m, 6)
    f = m.step(m.init(rho, u), 3)
    np.testing.assert_allclose(m.collide(f), m.collide_velocity_space(f), atol=1e-15)
    raw = O.Model(dict(RECT, wall_faces=4 | 8))
    assert np.abs(m.collide(f) - raw.collide(f)).max() > 1e-9
    g = m.collide(f)
    assert abs(g.sum() - f.sum()) < 1e-13
    np.testing.assert_allclose((m.C.T @ g).sum(axis=1) - (m.C.T @ f).sum(axis=1), m.N * m.force, atol=1e-15)
    # epsilon holds the second moments: with s_hi equal to a scalar
    # second-order block the BHLL step is the raw one again
    prm = dict(RECT, nu_b=RECT["nu"], s_hi=-1.0, dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0)
    same = O.Model(dict(prm, bhll=True))
    ref = O.Model(prm)
    np.testing.assert_allclose(same.collide(f), ref.collide(f), atol=1e-15)


def test_taylor_green_decay_rate():
    nu = 0.02
    n, dx = (48, 24, 1), (1.0, 0.5, 1.0)
    m = O.Model(dict(lattice="Q9", n=n, dx=dx, nu=nu, nu_b=0.05, s_hi=1.5, bhll=True))
    coords = grid_coords(n, dx)
    kx, ky = 2 * math.pi / (n[0] * dx[0]), 2 * math.pi / (n[1] * dx[1])
    U0 = 0.01
    u = np.zeros((2, m.N))
    u[0] = -U0 * np.cos(kx * coords[0]) * np.sin(ky * coords[1])
    u[1] = U0 * (kx / ky) * np.sin(kx * coords[0]) * np.cos(ky * coords[1])
    f = m.init(np.ones(m.N), u)
    phase = np.exp(-1j * (kx * coords[0] + ky * coords[1]))
    ts, amps = [], []
    for t in range(100, 801, 100):
        f = m.step(f, 100)
        _, uu = m.macroscopic(f)
        ts.append(t)
        amps.append(abs((uu[1] * phase).sum()))
    rate = -np.polyfit(np.asarray(ts, float), np.log(np.abs(amps)), 1)[0]
    assert abs(rate / (nu * (kx**2 + ky**2)) - 1) < 0.01


def test_refused_where_not_built():
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q27", n=(4, 4, 4), nu=0.02, bhll=True))
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q9", equation="NCDE", n=(4, 4, 1), D0=0.01, bhll=True))
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q9", n=(4, 4, 1), nu=0.02, bhll=True, hermite=True))
