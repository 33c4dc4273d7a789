"""Pins of the von Neumann reference (tests/vn_reference.py) against the
hydrodynamic limits it must reproduce: mass conservation (eigenvalue 1 at
k = 0), the shear wave of the NSE decaying at exp(-nu k^2 dt) and the
diffusion mode of the NCDE at exp(-D k^2 dt) for the longest wave of a
16-node grid, and the rest state of the default rates being neutrally
stable; the unstable s_hi = 1 of reading A5 shows a growing mode."""
import numpy as np

from oracle import rmrt_oracle as O
from vn_reference import amplification, jacobian, max_amplification


def _eigs(prm, rho0, u0, k):
    m = O.Model(dict(prm, n=(1, 1, 1)))
    return np.linalg.eigvals(amplification(m, jacobian(m, rho0, u0), k))


def test_mass_is_conserved_at_k0():
    prm = dict(lattice="Q19", dx=(1.0, 1.0, 2.0), nu=0.02)
    lam = _eigs(prm, 1.0, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    # rho and the three momenta are collision invariants: four eigenvalues 1
    assert np.sum(np.abs(lam - 1.0) < 1e-8) == 4


def test_shear_wave_decay_rate():
    nu = 0.05
    prm = dict(lattice="Q19", dx=(1.0, 1.0, 2.0), nu=nu)
    k = 2 * np.pi / 16
    lam = _eigs(prm, 1.0, (0.0, 0.0, 0.0), (k, 0.0, 0.0))
    want = np.exp(-nu * k * k)   # dx = dt = 1 along x
    # the shear modes (u_y, u_z varying along x) decay at that rate up to the
    # lattice's O(k^2) correction of the rate (k = 0.39 rad per node: ~1%)
    close = np.sort(np.abs(np.abs(lam) - want))[:2]
    assert close.max() < 2e-2 * (1 - want), (close, want)


def test_diffusion_mode_decay_rate():
    D0 = 0.02
    prm = dict(lattice="Q9", equation="NCDE", dx=(1.0, 0.5, 1.0), D0=D0, D2=0.0, adv=(0.0, 0.0, 0.0))
    k = 2 * np.pi / 16
    lam = _eigs(prm, 1.0, None, (k, 0.0))
    want = np.exp(-D0 * k * k)
    assert np.min(np.abs(np.abs(lam) - want)) < 2e-2 * (1 - want)


def test_default_rates_neutral_and_s_hi_one_unstable():
    base = dict(lattice="Q19", dx=(1.0, 1.0, 2.0), nu=0.005)
    assert max_amplification(base, 1.0, (0.0, 0.0, 0.0), (8, 8, 8)) < 1 + 1e-9
    assert max_amplification(dict(base, s_hi=1.0), 1.0, (0.0, 0.0, 0.0), (8, 8, 8)) > 1.01


def test_c_zero_form_diffusion_mode():
    """The C = 0 NCDE form carries phi of the previous step: its state is (f,
    phi_prev), and its diffusion mode still decays at exp(-D k^2)."""
    D0 = 0.02
    for prm in (dict(lattice="Q7", equation="NCDE", dx=(1.0, 1.0, 2.0), D0=D0, D2=0.0, adv=(0.0, 0.0, 0.0)),
                dict(lattice="Q9", equation="NCDE", dx=(1.0, 0.5, 1.0), D0=D0, D2=0.0, adv=(0.0, 0.0, 0.0),
                     c_zero=True)):
        m = O.Model(dict(prm, n=(1, 1, 1)))
        J = jacobian(m, 1.0, None)
        assert J.shape == (m.q + 1, m.q + 1)
        k = [2 * np.pi / 16] + [0.0] * (m.d - 1)
        lam = np.linalg.eigvals(amplification(m, J, k))
        want = np.exp(-D0 * k[0] ** 2)
        assert np.min(np.abs(np.abs(lam) - want)) < 2e-2 * (1 - want), prm["lattice"]
