"""Pins of the oracle's lattice tables, weights and moment matrices (CPU only).

Each check compares against something the paper prints (tests/golden) or a
fact of the mathematics (tensor products, standard lattices, brute-force
lattice sums), never against the oracle's own formula retyped."""
import itertools

import numpy as np
import pytest

from golden_util import read_matrix
from oracle import rmrt_oracle as O

C_CASES = [(1.0, 0.5, 2.0), (1.0, 1.0, 1.0), (0.7, 1.3, 0.9)]


def lattice_sum(w, C, powers):
    out = w.copy()
    for a, k in enumerate(powers):
        out = out * C[:, a] ** k
    return out.sum()


# ------------------------------------------------------------------ velocities
def test_q9_velocities_match_printed_table():
    env = dict(c1=1.0, c2=0.5)
    printed = read_matrix("rd2q9_velocities.txt", env).T
    C = O.unit_offsets("Q9") * np.array([1.0, 0.5])
    np.testing.assert_array_equal(C, printed)


def test_q27_printed_table_is_garbled_and_reading_a1_repairs_it():
    env = dict(c1=1.0, c2=2.0, c3=3.0)
    printed = read_matrix("rd3q27_velocities_printed.txt", env).T
    # the printed x-z edge block repeats two vectors
    assert len({tuple(v) for v in printed}) == 25
    C = O.unit_offsets("Q27") * np.array([1.0, 2.0, 3.0])
    differs = [j for j in range(27) if not np.array_equal(C[j], printed[j])]
    assert differs == [12, 14]
    # the repaired set is every vector of {-1,0,1}^3 scaled by c, exactly once
    full = {tuple(np.array(e) * np.array([1.0, 2.0, 3.0])) for e in itertools.product((-1, 0, 1), repeat=3)}
    assert {tuple(v) for v in C} == full
    # the two vectors the print lost are the ones the repair inserts
    missing = full - {tuple(v) for v in printed}
    assert missing == {tuple(C[12]), tuple(C[14])}


def test_q19_is_q27_without_corners_and_opposites():
    E19 = O.unit_offsets("Q19")
    assert E19.shape == (19, 3)
    assert all(np.count_nonzero(e) <= 2 for e in E19)
    for lat in ("Q9", "Q19", "Q27"):
        E = O.unit_offsets(lat)
        opp = O.opposite(E)
        np.testing.assert_array_equal(E[opp], -E)
        assert np.all(opp[opp] == np.arange(len(E)))


# --------------------------------------------------------------------- weights
@pytest.mark.parametrize("c", C_CASES)
def test_q9_weights_are_tensor_product_of_1d(c):
    c = np.array(c[:2])
    cs2 = min(c**2) / 3
    w = O.weights("Q9", c, cs2)
    r = cs2 / c**2
    w1d = [np.array([r[a] / 2, 1 - r[a], r[a] / 2]) for a in range(2)]  # offsets -1, 0, +1
    E = O.unit_offsets("Q9")
    expect = np.array([w1d[0][e[0] + 1] * w1d[1][e[1] + 1] for e in E])
    np.testing.assert_allclose(w, expect, rtol=0, atol=1e-15)


@pytest.mark.parametrize("c", C_CASES)
def test_q27_default_weights_are_tensor_product(c):
    c = np.array(c)
    cs2 = min(c**2) / 3
    w = O.weights("Q27", c, cs2)
    r = cs2 / c**2
    w1d = [np.array([r[a] / 2, 1 - r[a], r[a] / 2]) for a in range(3)]
    E = O.unit_offsets("Q27")
    expect = np.array([np.prod([w1d[a][e[a] + 1] for a in range(3)]) for e in E])
    np.testing.assert_allclose(w, expect, rtol=0, atol=1e-15)


def test_standard_lattice_weights():
    # c = 1, cs^2 = 1/3 gives the textbook D2Q9, D3Q19 and D3Q27 sets (Sec. III, last remark)
    w = O.weights("Q9", np.ones(2), 1 / 3)
    np.testing.assert_allclose(sorted(set(np.round(w, 12))), sorted({4 / 9, 1 / 9, 1 / 36}), atol=1e-12)
    w = O.weights("Q19", np.ones(3), 1 / 3)
    np.testing.assert_allclose(sorted(set(np.round(w, 12))), sorted({1 / 3, 1 / 18, 1 / 36}), atol=1e-12)
    w = O.weights("Q27", np.ones(3), 1 / 3)
    np.testing.assert_allclose(sorted(set(np.round(w, 12))), sorted({8 / 27, 2 / 27, 1 / 54, 1 / 216}), atol=1e-12)


@pytest.mark.parametrize("lat", ["Q9", "Q19", "Q27"])
@pytest.mark.parametrize("c", C_CASES)
def test_velocity_moments_delta2_delta4(lat, c):
    """Delta^(2) = cs^2 I (eq. 3-3-2) and the fourth-order constraints (eq. 3-3-11),
    by brute-force lattice sums; odd moments vanish."""
    d = 2 if lat == "Q9" else 3
    c = np.array(c[:d])
    cs2 = min(c**2) / 3
    wc = None
    if lat == "Q27":
        wc = 0.6 * min(cs2 / c**2) ** 3 / 8  # any admissible omega_19 must satisfy them too
    w = O.weights(lat, c, cs2, wc)
    assert np.all(w >= 0) and abs(w.sum() - 1) < 1e-15
    C = O.unit_offsets(lat) * c
    for powers in itertools.product(range(5), repeat=d):
        s = lattice_sum(w, C, powers)
        deg = sum(powers)
        if deg > 4:
            continue
        if any(k % 2 for k in powers):
            assert abs(s) < 1e-15, powers
            continue
        nz = [a for a in range(d) if powers[a] > 0]
        if deg == 0:
            expect = 1.0
        elif deg == 2:
            expect = cs2
        elif deg == 4 and len(nz) == 1:
            expect = c[nz[0]] ** 2 * cs2
        elif deg == 4:
            expect = cs2 * cs2
        assert abs(s - expect) < 1e-14, (powers, s, expect)


def test_weight_bounds_q19_requires_pairwise_sum():
    # rD3Q19: omega_1 = r1/2 - r1 r2/2 - r1 r3/2 >= 0 needs r2 + r3 <= 1 (from eq. 3-3-8 with omega_19 = 0)
    c = np.array([1.0, 0.5, 0.5])
    cs2 = 0.2
    w = O.weights("Q19", c, cs2)
    assert w[1] < 0  # r2 + r3 = 1.6 > 1
    assert np.all(O.weights("Q19", c, min(c**2) / 3) >= 0)


# ------------------------------------------------------------- moment matrices
@pytest.mark.parametrize("c", [(1.0, 0.5), (1.0, 2.0), (0.3, 0.7)])
def test_q9_moment_matrix_is_printed_factorisation(c):
    env = dict(c1=c[0], c2=c[1])
    Mt = read_matrix("md2q9_Mtilde.txt", env)
    D = np.diag(read_matrix("md2q9_D.txt", env)[0])
    C = O.unit_offsets("Q9") * np.array(c)
    M = O.moment_matrix(C, O.moment_exponents("Q9"))
    np.testing.assert_allclose(M, D @ Mt, rtol=1e-15, atol=1e-15)


@pytest.mark.parametrize("lat", ["Q19", "Q27"])
def test_3d_moment_matrices_invertible(lat):
    for c in C_CASES:
        C = O.unit_offsets(lat) * np.array(c)
        M = O.moment_matrix(C, O.moment_exponents(lat))
        assert M.shape[0] == M.shape[1]
        assert np.linalg.cond(M) < 1e4


def test_q19_dropped_moments_vanish_on_q19():
    """The 8 monomials with three non-zero exponents are identically zero on rD3Q19."""
    C = O.unit_offsets("Q19") * np.array([1.0, 0.5, 2.0])
    rows27 = O.moment_exponents("Q27")
    rows19 = set(O.moment_exponents("Q19"))
    extra = [r for r in rows27 if r not in rows19]
    assert len(extra) == 8
    assert np.all(O.moment_matrix(C, extra) == 0)
