"""Pins of the oracle's reduced NCDE lattices rD2Q5 and rD3Q7 (linear
equilibrium, C = 0 form of eq. 4-16): weights against Remark I of Sec. III,
the moments of the linear equilibrium against eq. 3-5, the textbook BGK
diffusion scheme as the equal-rate special case, the advected Gaussian hill in
2D and 3D (constant diffusivity, eq. 4-15), mass conservation, and a negative
control: dropping the dB/dt auxiliary term G leaves the anisotropic u u
diffusion error it exists to cancel."""
import numpy as np
import pytest

from inputs import grid_coords
from oracle import rmrt_oracle as O


def _model(lat, **kw):
    d = 2 if lat == "Q5" else 3
    prm = dict(lattice=lat, equation="NCDE", rho0=0.0)
    prm.setdefault("n", (6, 5, 1) if d == 2 else (4, 5, 3))
    prm.update(kw)
    return O.Model(prm)


@pytest.mark.parametrize("lat,dx", [("Q5", (1.0, 0.5, 1.0)), ("Q5", (1.0, 2.0, 1.0)), ("Q7", (1.0, 0.5, 2.0))])
def test_weights_remark_one(lat, dx):
    m = _model(lat, dx=dx)
    d = m.d
    r = m.cs2 / m.c**2
    for a in range(d):
        assert m.w[1 + a] == pytest.approx(r[a] / 2.0, rel=1e-15)
        assert m.w[1 + d + a] == pytest.approx(r[a] / 2.0, rel=1e-15)
    assert m.w.sum() == pytest.approx(1.0, abs=1e-15)
    assert (m.w >= 0).all()
    # Delta^(2) = c_s^2 I and vanishing odd moments
    np.testing.assert_allclose(np.einsum("j,ja,jb->ab", m.w, m.C, m.C), m.cs2 * np.eye(d), atol=1e-15)
    np.testing.assert_allclose(m.w @ m.C, 0.0, atol=1e-16)


def test_standard_lattice_weights():
    """c = 1: rD2Q5 with c_s^2 = 1/3 is the textbook D2Q5 (1/3, 1/6 x 4); rD3Q7
    with c_s^2 = 1/4 is the textbook D3Q7 (1/4, 1/8 x 6)."""
    m = _model("Q5", dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0)
    np.testing.assert_allclose(m.w, [1 / 3] + [1 / 6] * 4, rtol=1e-15)
    m = _model("Q7", dx=(1.0, 1.0, 1.0), cs2=0.25)
    np.testing.assert_allclose(m.w, [1 / 4] + [1 / 8] * 6, rtol=1e-15)


@pytest.mark.parametrize("lat", ["Q5", "Q7"])
def test_linear_equilibrium_moments_eq_3_5(lat):
    """sum g = A, sum c g = B, sum c c g = A Delta^(2) for M = 0."""
    m = _model(lat, dx=(1.0, 0.5, 2.0))
    rng = np.random.default_rng(3)
    n, d = 7, m.d
    A = rng.normal(size=n)
    B = rng.normal(size=(d, n))
    g = O.g_eq(m.C, m.w, m.c, m.cs2, A, B, np.zeros((d, d, n)))
    np.testing.assert_allclose(g.sum(axis=0), A, atol=1e-14)
    np.testing.assert_allclose(m.C.T @ g, B, atol=1e-14)
    np.testing.assert_allclose(np.einsum("ja,jb,jn->abn", m.C, m.C, g),
                               m.cs2 * np.eye(d)[:, :, None] * A[None, None], atol=1e-14)


def _bgk_textbook(E, w, phi, omega, steps, shape):
    """Textbook lattice-BGK diffusion: f_j(x + e_j) = f_j - omega (f_j - w_j phi)."""
    q = len(w)
    f = w[:, None] * phi[None]
    for _ in range(steps):
        rho = f.sum(axis=0)
        post = f - omega * (f - w[:, None] * rho[None])
        out = np.empty_like(f)
        for j in range(q):
            g = post[j].reshape(shape[::-1])
            for a, e in enumerate(E[j]):
                g = np.roll(g, e, axis=len(shape) - 1 - a)
            out[j] = g.reshape(-1)
        f = out
    return f


@pytest.mark.parametrize("lat,n,dx,cs2", [("Q5", (9, 7, 1), (1.0, 0.5, 1.0), -1.0),
                                          ("Q7", (5, 6, 4), (1.0, 2.0, 0.5), 0.05)])
def test_equal_rates_reduce_to_textbook_bgk(lat, n, dx, cs2):
    """u = 0, S = 0, constant D and s_hi = s_1: every non-conserved rate equals
    s_1, so the moment-space scheme is the BGK scheme written directly in
    populations."""
    D = 0.03
    m = _model(lat, n=n, dx=dx, cs2=cs2, D0=D, D2=0.0)
    s1 = float(m.s1_ncde(np.array([0.0]))[0])
    m = _model(lat, n=n, dx=dx, cs2=cs2, D0=D, D2=0.0, s_hi=s1)
    phi = 1.0 + 0.2 * np.random.default_rng(5).random(m.N)
    f, h = m.step(m.init(phi, None), 6, m.init_history(phi))
    ref = _bgk_textbook(m.E, m.w, phi, s1, 6, n[: m.d])
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-14)


def _hill(lat, n, dx, D, adv, sigma, steps, drop_g=False):
    m = _model(lat, n=n, dx=dx, D0=D, D2=0.0, adv=adv)
    if drop_g:
        # planted omission: the dB/dt auxiliary distribution G set to zero
        full = m.distributions

        def without_g(fbar, phi_prev=None, sel=None):
            feq, F, G, s1 = full(fbar, phi_prev, sel)
            return feq, F, np.zeros_like(G), s1
        m.distributions = without_g
    d = m.d
    X, Y, Z = grid_coords(n, dx)
    coords = [X, Y, Z][:d]
    L = [n[a] * dx[a] for a in range(d)]
    centre = [0.5 * v for v in L]
    phi0 = O.gaussian_hill_nd(coords, 0.0, sigma, D, centre, adv[:d], L)
    f, h = m.step(m.init(phi0, None), steps, m.init_history(phi0))
    phi, _ = m.macroscopic(f)
    exact = O.gaussian_hill_nd(coords, steps, sigma, D, centre, adv[:d], L)
    l2 = np.sqrt(((phi - exact) ** 2).sum() / (exact**2).sum())
    return l2, abs(phi.sum() - phi0.sum())


def test_gaussian_hill_q5_rectangular():
    l2, dm = _hill("Q5", (128, 128, 1), (1.0, 0.5, 1.0), 0.01, (0.05, 0.02, 0.0), 8.0, 400)
    assert l2 < 2e-3, l2
    assert dm < 1e-10


def test_gaussian_hill_q7_rectangular():
    # sigma / dz = 3 nodes: 6.1e-3 here, 3.1e-3 at sigma = 8 on 64 x 64 x 32 (second order)
    l2, dm = _hill("Q7", (48, 48, 24), (1.0, 1.0, 2.0), 0.02, (0.04, -0.02, 0.03), 6.0, 150)
    assert l2 < 8e-3, l2
    assert dm < 1e-10


def test_dropping_g_leaves_the_uu_diffusion_error():
    """Negative control: with G removed the linear equilibrium diffuses with
    K - (K / c_s^2) u u; the hill's error grows several-fold."""
    args = ("Q5", (128, 128, 1), (1.0, 1.0, 1.0), 0.05, (0.15, 0.06, 0.0), 12.0, 800)
    with_g, _ = _hill(*args)
    without_g, _ = _hill(*args, drop_g=True)
    assert with_g < 4e-3, with_g
    assert without_g > 3.0 * with_g, (with_g, without_g)


def test_nonlinear_diffusivity_conserves_mass():
    """D(phi) = D0 (1 + D2 phi^2) (its phi dependence is pinned by the linearised
    decay in test_oracle_nonlinear_diffusion.py): the total phi is conserved
    without a source and grows by N dt S with one."""
    for S in (0.0, 1e-4):
        m = _model("Q5", n=(20, 16, 1), dx=(1.0, 0.5, 1.0), D0=0.02, D2=2.0, adv=(0.03, -0.02, 0.0), source=S)
        phi = 0.5 + 0.3 * np.random.default_rng(9).random(m.N)
        f, h = m.step(m.init(phi, None), 1, m.init_history(phi))
        p1, _ = m.macroscopic(f)
        f, h = m.step(f, 10, h)
        p2, _ = m.macroscopic(f)
        assert abs(p2.sum() - p1.sum() - 10 * m.N * S) < 1e-11


def test_history_is_required_and_updated():
    m = _model("Q5", D0=0.02, adv=(0.05, 0.0, 0.0))
    phi = 1.0 + 0.1 * np.random.default_rng(1).random(m.N)
    f = m.init(phi, None)
    with pytest.raises(ValueError):
        m.step(f, 1)
    f1, h1 = m.step(f, 1, m.init_history(phi))
    np.testing.assert_allclose(h1, m.macroscopic(f)[0], atol=1e-15)   # phi of the step just taken
    with pytest.raises(ValueError):
        O.Model(dict(lattice="Q5", equation="NSE"))
