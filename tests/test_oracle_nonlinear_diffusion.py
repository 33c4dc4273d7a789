"""Pin of the oracle's nonlinear diffusivity D(phi) = D0 (1 + D2 phi^2) (the NCDE
of Sec. IV with K = D(phi) I set through the local first-order rate of eq. 4-10,
reading A14).

The recovered equation (eq. 4-15 without advection or source) is
    d phi / dt = div(D(phi) grad phi).
On a uniform background phibar with a small perturbation eps cos(k . x) it
linearises to d phi'/dt = D(phibar) lap phi' + O(eps^2): the mode decays at
exactly D0 (1 + D2 phibar^2) |k|^2.  The fitted rate therefore pins the
quadratic dependence on phi (a slip to D2 phi, or phi taken from the wrong
level, moves it by tens of per cent at phibar = 2), the local rate formula and
c_s^2 in it, on the rectangular lattices with dy = dx / 2 and dz = 2 dx.

The scheme's rate carries a lattice error of second order in |k| dx (a few per
cent at 16 nodes per wavelength when s_1 is close to 2), so each case is run at
two wavelengths, L and 2 L, and the two rates are extrapolated to |k| -> 0,
r = (4 r_2L - r_L) / 3, which must match D(phibar) |k|^2 to 2e-3.

A negative control plants the D2 phi slip in the oracle and must fail."""
import math

import numpy as np
import pytest

from inputs import grid_coords
from oracle import rmrt_oracle as O

D0, D2, EPS = 0.01, 1.0, 1e-4


def _decay_rate(lat, phibar, planted=False, scale=1):
    """Fitted decay rate of the mode and D(phibar) |k|^2, on a grid of `scale`
    times the base size (wavelengths grow with it)."""
    d = 2 if lat in ("Q9", "Q5") else 3
    if d == 2:
        n, dx = (32 * scale, 16 * scale, 1), (1.0, 0.5, 1.0)
    else:
        n, dx = (32 * scale, 1, 16 * scale), (1.0, 1.0, 2.0)
    m = O.Model(dict(lattice=lat, equation="NCDE", n=n, dx=dx, D0=D0, D2=D2, rho0=0.0))
    if planted:
        m.s1_ncde = lambda phi: 1.0 / (0.5 + D0 * (1.0 + D2 * phi) / (m.cs2 * m.dt))
    X, Y, Z = grid_coords(n, dx)
    kx = 2 * math.pi / (n[0] * dx[0])
    if d == 2:
        ky, kz = 2 * math.pi / (n[1] * dx[1]), 0.0
        mode = np.cos(kx * X) * np.cos(ky * Y)
    else:
        ky, kz = 0.0, 2 * math.pi / (n[2] * dx[2])
        mode = np.cos(kx * X) * np.cos(kz * Z)
    k2 = kx**2 + ky**2 + kz**2
    phi0 = phibar + EPS * mode
    f = m.init(phi0, None)
    hist = m.init_history(phi0) if m.linear else None
    Dbar = D0 * (1.0 + D2 * phibar**2)
    # run over 0.3 e-foldings of the mode; skip the initial layer
    total = int(round(0.3 / (Dbar * k2)))
    every = max(total // 10, 1)
    ts, amps = [], []
    for t in range(every, 10 * every + 1, every):
        if hist is None:
            f = m.step(f, every)
        else:
            f, hist = m.step(f, every, hist)
        phi, _ = m.macroscopic(f)
        if t >= 2 * every:
            ts.append(t)
            amps.append(((phi - phi.mean()) * mode).sum() / (mode * mode).sum())
    rate = -np.polyfit(np.asarray(ts, float), np.log(np.abs(amps)), 1)[0]
    # the background is conserved exactly (eq. 4-18-1)
    assert abs(phi.mean() - phibar) < 1e-13
    return rate, Dbar * k2


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q5", "Q7"])
@pytest.mark.parametrize("phibar", [0.5, 1.0, 2.0])
def test_linearised_decay_follows_D_of_phibar(lat, phibar):
    r1, e1 = _decay_rate(lat, phibar, scale=1)
    r2, e2 = _decay_rate(lat, phibar, scale=2)
    ratio1, ratio2 = r1 / e1, r2 / e2
    # second-order lattice error: it shrinks with the wavelength
    assert abs(ratio2 - 1) < abs(ratio1 - 1) + 1e-4, (ratio1, ratio2)
    assert abs(ratio2 - 1) < 0.015, (lat, phibar, ratio2)
    extrapolated = (4.0 * ratio2 - ratio1) / 3.0
    assert abs(extrapolated - 1) < 2e-3, (lat, phibar, ratio1, ratio2, extrapolated)


@pytest.mark.parametrize("lat", ["Q9", "Q7"])
def test_planted_linear_phi_dependence_fails(lat):
    """Negative control: D0 (1 + D2 phi) in place of D0 (1 + D2 phi^2)."""
    rate, exact = _decay_rate(lat, 2.0, planted=True)
    assert abs(rate / exact - 1) > 0.2, (lat, rate, exact)
