"""Pins of the oracle's equilibrium, relaxation matrix and collision routes (CPU only)."""
import itertools

import numpy as np
import pytest
import sympy as sp

from golden_util import read_matrix, read_vector
from oracle import rmrt_oracle as O


def _model(lat, c, **kw):
    d = 2 if lat == "Q9" else 3
    n = (3, 3, 1) if d == 2 else (3, 3, 3)
    dx = tuple(c) + ((1.0,) if d == 2 else ())
    return O.Model(dict(lattice=lat, n=n, dx=dx, **kw))


def _rand_state(m, seed, N=5):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal(N)
    u = 0.05 * rng.standard_normal((m.d, N))
    return rho, u


def _feq(m, rho, u):
    return O.g_eq(m.C, m.w, m.c, m.cs2, rho, rho[None] * u, rho[None, None] * np.einsum("an,bn->abn", u, u))


# --------------------------------------------------------- printed equilibria
@pytest.mark.parametrize("c", [(1.0, 0.5), (1.0, 1.0), (0.8, 1.6)])
def test_q9_equilibrium_moments_match_printed(c):
    m = _model("Q9", c, nu=0.05)
    rho, u = _rand_state(m, 1)
    got = m.M @ _feq(m, rho, u)
    for n in range(rho.size):
        env = dict(rho=rho[n], u=u[0, n], v=u[1, n], cs2=m.cs2)
        np.testing.assert_allclose(got[:, n], read_vector("meq_d2q9.txt", env), rtol=0, atol=1e-15)


def _t2_moment(ex, rho, u, cs2):
    """rho * (prod_a h_a) truncated to second order in u, h = 1, u_a, cs2 + u_a^2 (sympy)."""
    eps = sp.Symbol("eps")
    U = sp.symbols("u0:3")
    prod = sp.Integer(1)
    for a, k in enumerate(ex):
        prod *= [sp.Integer(1), eps * U[a], cs2 + eps**2 * U[a] ** 2][k]
    poly = sp.expand(prod)
    trunc = sum(poly.coeff(eps, k) for k in range(3))
    return float(rho * trunc.subs({U[i]: float(u[i]) for i in range(len(u))}))


@pytest.mark.parametrize("lat", ["Q19", "Q27"])
@pytest.mark.parametrize("c", [(1.0, 0.5, 2.0), (1.0, 1.0, 2.0)])
def test_3d_equilibrium_moments_closed_form(lat, c):
    """Q27 (tensor weights): every raw moment equals rho T2[prod h_a].
    Q19: the same, except the three (2,2,0)-type moments, which lose the corner
    contribution: - rho cs^4 u_g^2 / (c_g^2 - cs^2), g the axis with exponent 0."""
    m = _model(lat, c, nu=0.05)
    rho, u = _rand_state(m, 2, N=3)
    got = m.M @ _feq(m, rho, u)
    cs2 = m.cs2
    for n in range(rho.size):
        for i, ex in enumerate(m.exps):
            exp = _t2_moment(ex, rho[n], u[:, n], cs2)
            if lat == "Q19" and sorted(ex) == [0, 2, 2]:
                g = ex.index(0)
                exp -= rho[n] * cs2**2 * u[g, n] ** 2 / (m.c[g] ** 2 - cs2)
            assert abs(got[i, n] - exp) < 1e-15, (lat, ex, got[i, n], exp)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_redf_moments_eq_3_5_and_3_9(lat):
    """sum g = A, sum c g = B, sum cc g = A Delta2 + M, third moment from eq. 3-9."""
    c = (1.0, 0.5) if lat == "Q9" else (1.0, 0.5, 2.0)
    m = _model(lat, c, nu=0.05)
    d, cs2 = m.d, m.cs2
    rng = np.random.default_rng(3)
    N = 4
    A = rng.standard_normal(N)
    B = rng.standard_normal((d, N))
    Mt = rng.standard_normal((d, d, N))
    Mt = Mt + Mt.transpose(1, 0, 2)
    g = O.g_eq(m.C, m.w, m.c, cs2, A, B, Mt)
    np.testing.assert_allclose(g.sum(0), A, atol=1e-14)
    np.testing.assert_allclose(m.C.T @ g, B, atol=1e-14)
    np.testing.assert_allclose(np.einsum("ja,jb,jn->abn", m.C, m.C, g),
                               A[None, None] * cs2 * np.eye(d)[:, :, None] + Mt, atol=1e-14)
    third = np.einsum("ja,jb,jc,jn->abcn", m.C, m.C, m.C, g)
    for a, b, cc in itertools.product(range(d), repeat=3):
        exp = cs2 * ((a == b) * B[cc] + (a == cc) * B[b] + (b == cc) * B[a])
        if a == b == cc:
            exp = exp + cs2 * (m.c[a] ** 2 - 3 * cs2) * B[a] / cs2     # delta^(4) term, eq. 3-8
        np.testing.assert_allclose(third[a, b, cc], exp, atol=1e-14)


# ------------------------------------------------------------------ BHLL basis
@pytest.mark.parametrize("a", [0.5, 1.0, 2.0, 0.8])
def test_bhll_matrices_consistent(a):
    env = dict(a=a)
    N = read_matrix("bhll_N.txt", env)
    Ma = read_matrix("bhll_Ma.txt", env)
    Mb = read_matrix("bhll_M.txt", env)
    np.testing.assert_allclose(N @ Ma, Mb, atol=1e-13)
    # M_a is the oracle's raw-moment matrix with c1 = 1, c2 = a
    m = _model("Q9", (1.0, a), nu=0.05)
    np.testing.assert_allclose(m.M, Ma, atol=1e-15)


@pytest.mark.parametrize("a", [0.5, 0.8])
def test_bhll_equilibrium_moments(a):
    """N_BHLL m_eq reproduces the printed BHLL equilibrium (eq. meqd2q9-1, eq. 5-9)."""
    env = dict(a=a)
    N = read_matrix("bhll_N.txt", env)
    m = _model("Q9", (1.0, a), nu=0.05, cs2=0.2 * a * a)
    rho, u = _rand_state(m, 4, N=3)
    got = N @ (m.M @ _feq(m, rho, u))
    for n in range(rho.size):
        env2 = dict(a=a, rho=rho[n], u=u[0, n], v=u[1, n], cs2=m.cs2)
        np.testing.assert_allclose(got[:, n], read_vector("bhll_meq.txt", env2), atol=1e-14)


def test_collision_matrix_invariant_under_lower_triangular_basis_change():
    """Lambda = M^-1 S M equals (N M)^-1 (N S N^-1) (N M) for N = N_BHLL (eq. 5-1-2)."""
    a = 0.5
    N = read_matrix("bhll_N.txt", dict(a=a))
    m = _model("Q9", (1.0, a), nu=0.03, nu_b=0.07)
    # lower triangular in the block (moment-order) sense
    for i in range(9):
        for j in range(9):
            if m.order[j] > m.order[i]:
                assert N[i, j] == 0
    Lam = m.Minv @ m.S @ m.M
    Mb = N @ m.M
    Sb = N @ m.S @ np.linalg.inv(N)
    np.testing.assert_allclose(np.linalg.inv(Mb) @ Sb @ Mb, Lam, atol=1e-12)


# ---------------------------------------------------------- relaxation matrix
@pytest.mark.parametrize("d,c", [(2, (1.0, 0.5)), (3, (1.0, 0.5, 2.0)), (3, (1.0, 1.0, 1.0))])
@pytest.mark.parametrize("nu,nu_b", [(0.02, 0.05), (0.1, 0.01), (0.005, 0.2)])
def test_sherman_morrison_block(d, c, nu, nu_b):
    c = np.array(c)
    cs2 = min(c**2) / 3
    s_ab, s_s, s_b = O.nse_rates(c, cs2, nu, nu_b, d)
    direct = np.linalg.inv(O.S2_inverse_block(c, cs2, s_s, s_b, d))
    np.testing.assert_allclose(O.S2_sherman_morrison(c, cs2, s_s, s_b, d), direct, rtol=1e-13, atol=1e-14)
    # all rates lie in (0, 2)
    assert 0 < s_ab < 2 and np.all((s_s > 0) & (s_s < 2)) and np.all((s_b > 0) & (s_b < 2))


def test_diagonal_block_when_bulk_matches_remark_v():
    m = _model("Q19", (1.0, 0.5, 2.0), nu=0.03)          # nu_b defaults to 2 nu / d
    off = m.Sbar21 - np.diag(np.diag(m.Sbar21))
    assert np.abs(off).max() < 1e-15


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
def test_moment_route_equals_velocity_route(lat):
    c = (1.0, 0.5) if lat == "Q9" else (1.0, 0.5, 2.0)
    m = _model(lat, c, nu=0.03, nu_b=0.08, force=(1e-3, -2e-3, 5e-4)[: 2 if lat == "Q9" else 3],
               source=2e-4)
    rho, u = _rand_state(m, 5, N=m.N)
    f = m.init(rho, u) + 1e-3 * np.random.default_rng(6).standard_normal((m.q, m.N))
    np.testing.assert_allclose(m.collide(f), m.collide_velocity_space(f), atol=1e-14)


def test_ncde_moment_route_equals_velocity_route():
    m = _model("Q9", (1.0, 0.5), equation="NCDE", D0=0.01, D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0,
               source=1e-3)
    rng = np.random.default_rng(7)
    phi = rng.uniform(0, 1, m.N)
    f = m.init(phi, None) + 1e-3 * rng.standard_normal((m.q, m.N))
    np.testing.assert_allclose(m.collide(f), m.collide_velocity_space(f), atol=1e-14)


def test_lower_blocks_cancel_for_nse():
    """Reading A6: S_10, S_20, S_21 (below the diagonal) do not change the result
    of eq. 2-2-3, because the order-0/1 non-equilibrium moments are -dt m_F/2."""
    m = _model("Q27", (1.0, 0.5, 2.0), nu=0.03, nu_b=0.08, force=(1e-3, -2e-3, 5e-4), source=3e-4)
    rho, u = _rand_state(m, 8, N=m.N)
    f = m.init(rho, u) + 1e-3 * np.random.default_rng(9).standard_normal((m.q, m.N))
    base = m.collide(f)
    rng = np.random.default_rng(10)
    S = m.S.copy()
    low = [i for i in range(m.q) if m.order[i] <= 1]
    for i in range(m.q):
        for j in low:
            if m.order[i] > m.order[j]:
                S[i, j] = rng.uniform(-1, 1)
    for i in low:
        S[i, i] = rng.uniform(0.5, 1.5)
    m.S = S
    np.testing.assert_allclose(m.collide(f), base, atol=1e-14)
