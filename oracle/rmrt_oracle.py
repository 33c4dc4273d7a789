"""Plain FP64 CPU oracle of the RMRT-LB scheme (arXiv:2206.00366).

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Everything is dense and literal: the transformation matrix M is built from its
definition (raw moments, Sec. V eq. 5-2), inverted numerically, the relaxation
matrix S is assembled as a full q x q matrix (eq. 5-1, 5-8), and the
equilibrium, source and auxiliary distributions are evaluated in velocity space
from the general rectangular equilibrium g_eq(A, B, M) (eq. 3-3, 3-4).  One
time step is eq. 2-2-3 followed by propagation (eq. 2-2, second line).

Arrays: populations have shape (q, N) with N = nx*ny*nz nodes in x-fastest
order (node index = x + nx*(y + ny*z)); all arithmetic is float64.

Every part is pinned by tests that check it against something other than
this file (closed forms, printed values, invariants, limits), listed in the
design notes.  The nonlinear diffusivity D(phi) = D0 (1 + D2 phi^2) of the
NCDE (eq. 4-10 with reading A14) is pinned by the linearised decay of a small
mode on uniform backgrounds, whose rate is D(phibar) |k|^2 (eq. 4-15).

Readings of the paper where it is silent or garbled (kept in one place so the
GPU side can take the same ones; numbering as in the design notes):
  A1  the printed rD3Q27 x-z edge velocities (eq. 3-2b, j = 11..14) repeat two
      vectors; they are read as (c1,0,c3), (-c1,0,c3), (-c1,0,-c3), (c1,0,-c3),
      the pattern of the x-y and y-z edges.
  A2  c_s^2 <= 0 selects min_a c_a^2 / 3.
  A3  rD3Q27 omega_19 defaults to r1 r2 r3 / 8 with r_a = c_s^2 / c_a^2.
  A4  3D raw-moment rows: all monomials with exponents in {0,1,2} (rD3Q27), or
      those with at most two non-zero exponents (rD3Q19).
  A5  rates of order >= 3 default to s_nu (NSE) and 1 (NCDE).
  A6  s_0, S_1 and the blocks below the diagonal are 1, 1 and 0 for the NSE.
  A7  dt = 1 unless given.
  A8  the e_alpha of the source distribution (eq. NSEFeq) is 1.
  A9  M_2G uses form (a) of eq. M2GComput with the full S_2 block.
  A10 boundaries: halfway bounce-back at wall faces and solid nodes.
  A11 nu_b < 0 selects 2 nu / d (eq. 4-27-1 with a = 0, Remark V of Sec. IV).
  A14 NCDE: D = phi I, beta = 1, K = D(phi) I with D(phi) = D0 (1 + D2 phi^2),
      B = phi u_adv with constant u_adv, C = phi u_adv u_adv.
  A19 He-Luo option: f_eq = g_eq(rho, rho0 u, rho0 u u) with rho0 u = sum c f
      (eq. meqd2q9-HL); every place that uses u (the forcing moments, the
      stress relation K_mu = rho0 nu, the f_ne initialisation) takes this u
      and rho0 in place of rho.
  A20 viscosity tensor of eq. 4-29: per-entry viscosities (xx, yy, zz, xy,
      xz, yz) set s_s,a (diagonal entries), s_ab (off-diagonal entries) by
      eq. 4-31 entry by entry, and per-axis bulk viscosities set s_b,a;
      unset entries take nu and nu_b.
  A21 gamma = 0 option of eq. 2-1 (NCDE): the dt^2/2 dF/dt term is the
      explicit difference of F, zero for the constant source; populations are
      f (no fbar transform), phi = sum f, and the collision adds dt (G + F).
  A22 diffusive-scaling option (eq. 4-17, NCDE): the dt^2/2 D F term is
      removed (populations f, phi = sum f, as A21), f_eq = g_eq(phi, phi u, 0)
      (C = 0) and G = 0; the grad phi output then drops its dt X / 2 term.
  A18 the reduced lattices rD2Q5 (the rD2Q5I subset of rD2Q9) and rD3Q7 carry
      the NCDE only, in the C = 0 form of eq. 4-16: linear equilibrium
      g_eq(phi, phi u_adv, 0), F_j = w_j S and
      G_j = g_eq(0, (1 - s_1/2) dB/dt, 0) with the first-order difference
      dB/dt = u_adv (phi(t) - phi(t - dt)) / dt.  phi(t - dt) is model state
      (the history field); at t = 0 it is the initial phi, so the first step
      sees dB/dt = 0.  Moment rows are the monomials with at most one non-zero
      exponent; rates of order 2 default to 1 as in A5.
  A23 the same C = 0 form of eq. 4-16 as an option (c_zero) on rD2Q9, rD3Q19
      and rD3Q27: f_eq = g_eq(phi, phi u_adv, 0), G from the first-order
      difference of B = phi u_adv with the history field, rates of order >= 2
      as in A5.
  A24 source fields: the mass source, the NCDE source and the body force may
      vary from node to node and from step to step (set_sources /
      update_sources); every formula takes the node's value at the current
      step.  In the gamma = 0 form the dt^2/2 dF/dt term is the explicit
      difference dt (F(t) - F(t - dt)) / 2 with F(t - dt) the source the
      previous step used; at the first step after the fields are set it is
      taken equal to F(t).
  A25 central-moment (cascaded) collision (option central, NSE on rD2Q9 and
      rD3Q27, whose moment sets are closed under the shift): the moments are
      kappa = N(u) M fbar with N(u) the binomial shift of eq. 5-1-1 at the
      node's u, and the relaxation matrix in that basis has the blocks of the
      raw-moment model (the full second-order block from nu and nu_b, s_ab on
      the off-diagonal second moments, s_hi above); equilibrium, auxiliary and
      source moments are N(u) times the raw ones, so the step is eq. 2-2-3 with
      Lambda = M^-1 N^-1 S N M (eq. 5-1-2).
  A26 Hermite-moment and central-Hermite-moment collisions (option hermite,
      NSE on rD2Q9, rD3Q19 and rD3Q27; with central on rD2Q9 / rD3Q27): the
      moment of exponents (a, b, p) is the tensor-product Hermite polynomial
      H_a(xi_x) H_b(xi_y) H_p(xi_z) with H_0 = 1, H_1 = xi, H_2 = xi^2 - cs2 of
      the velocity xi = c_j (or c_j - u with central), i.e. the basis H M (or
      H N(u) M) of eq. 5-1-1 with H the constant lower-triangular matrix that
      subtracts cs2 times the moment two orders lower per axis; the relaxation
      matrix in that basis has the raw model's blocks as in A25, and every
      moment vector is transformed alike (eq. 5-1-2).  The 19 moments of
      rD3Q19 are closed under H (it lowers exponents of 2 to 0 only).
  A27 BHLL-moment collision (option bhll, NSE on rD2Q9): the moments are
      N_BHLL M_a fbar with N_BHLL the printed matrix of Sec. V at a = c_y / c_x
      and M_a the raw moments of the velocities measured in units of c_x (so
      c_x = 1 gives the printed M_a); the BHLL moments of each order relax on
      their own, with the block of that order of N S N^-1 (S the raw model's
      relaxation matrix): the second-order block of eq. 5-8 carried into the
      BHLL basis by similarity, s_ab on p_xy and s_hi on q_x, q_y and epsilon.
      The couplings between orders that N S N^-1 would have are dropped, so the
      step differs from the raw one once s_hi differs from the second-order
      rates (through epsilon, whose definition holds second-order moments).
"""
from __future__ import annotations

import math

import numpy as np

# --------------------------------------------------------------------------
# Lattices: integer unit offsets e_j; c_j = e_j (.) (dx_a / dt)  (Sec. III)
# --------------------------------------------------------------------------

# rD2Q9, eq. 3-1 (column order as printed)
_E_Q9 = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]

# rD3Q27, eq. 3-2a/b/c; j = 11..14 follow reading A1
_E_Q27 = [
    (0, 0, 0),
    (1, 0, 0), (0, 1, 0), (0, 0, 1), (-1, 0, 0), (0, -1, 0), (0, 0, -1),
    (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0),
    (1, 0, 1), (-1, 0, 1), (-1, 0, -1), (1, 0, -1),
    (0, 1, 1), (0, -1, 1), (0, -1, -1), (0, 1, -1),
    (1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1),
    (-1, -1, -1), (-1, -1, 1), (-1, 1, -1), (1, -1, -1),
]

WALL_XM, WALL_XP, WALL_YM, WALL_YP, WALL_ZM, WALL_ZP = 1, 2, 4, 8, 16, 32


LINEAR_LATTICES = ("Q5", "Q7")


def unit_offsets(lattice: str) -> np.ndarray:
    """Integer offsets e_j, shape (q, d). rD3Q19 = first 19 of rD3Q27, rD2Q5 =
    first 5 of rD2Q9 (the rD2Q5I subset), rD3Q7 = first 7 of rD3Q27 (Sec. III)."""
    if lattice == "Q9":
        return np.array(_E_Q9, dtype=np.int64)
    if lattice == "Q5":
        return np.array(_E_Q9[:5], dtype=np.int64)
    if lattice == "Q7":
        return np.array(_E_Q27[:7], dtype=np.int64)
    if lattice == "Q27":
        return np.array(_E_Q27, dtype=np.int64)
    if lattice == "Q19":
        return np.array(_E_Q27[:19], dtype=np.int64)
    raise ValueError(lattice)


def opposite(E: np.ndarray) -> np.ndarray:
    """opp[j] = index k with e_k = -e_j (brute force search)."""
    q = E.shape[0]
    opp = np.empty(q, dtype=np.int64)
    for j in range(q):
        hits = [k for k in range(q) if np.all(E[k] == -E[j])]
        assert len(hits) == 1
        opp[j] = hits[0]
    return opp


def weights(lattice: str, c: np.ndarray, cs2: float, w_corner: float | None = None) -> np.ndarray:
    """Weights of eq. 3-3-5 (rD2Q9), eq. 3-3-8 (rD3Q27; rD3Q19 has omega_19 = 0)
    and Remark I of Sec. III (rD2Q5I, rD3Q7: omega_a = c_s^2 / (2 c_a^2))."""
    c = np.asarray(c, dtype=np.float64)
    r = cs2 / c**2
    if lattice in LINEAR_LATTICES:
        w = np.concatenate([[0.0], r / 2.0, r / 2.0])
    elif lattice == "Q9":
        w5 = r[0] * r[1] / 4.0
        w1 = r[0] / 2.0 - 2.0 * w5
        w2 = r[1] / 2.0 - 2.0 * w5
        w = np.array([0.0, w1, w2, w1, w2, w5, w5, w5, w5])
    else:
        if lattice == "Q19":
            w19 = 0.0
        else:
            w19 = r[0] * r[1] * r[2] / 8.0 if (w_corner is None or w_corner < 0) else float(w_corner)
        w7 = r[0] * r[1] / 4.0 - 2.0 * w19
        w11 = r[0] * r[2] / 4.0 - 2.0 * w19
        w15 = r[1] * r[2] / 4.0 - 2.0 * w19
        w1 = r[0] / 2.0 - 2.0 * (w7 + w11) - 4.0 * w19
        w2 = r[1] / 2.0 - 2.0 * (w7 + w15) - 4.0 * w19
        w3 = r[2] / 2.0 - 2.0 * (w11 + w15) - 4.0 * w19
        w = [0.0, w1, w2, w3, w1, w2, w3] + [w7] * 4 + [w11] * 4 + [w15] * 4
        if lattice == "Q27":
            w += [w19] * 8
        w = np.array(w)
    w[0] = 1.0 - w[1:].sum()
    return w


def moment_exponents(lattice: str) -> list[tuple[int, ...]]:
    """Raw-moment rows c_x^a c_y^b (c_z^p), exponents in {0,1,2} (eq. 5-2).

    rD2Q9 rows follow the printed factorisation M = D M~ (eq. Md2q9); 3D rows
    follow reading A4 (by total degree, diagonal second moments first)."""
    if lattice == "Q9":
        return [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (1, 2), (2, 1), (2, 2)]
    if lattice == "Q5":
        return [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2)]
    if lattice == "Q7":
        return [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2)]
    rows = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
            (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1), (0, 1, 1),
            (2, 1, 0), (2, 0, 1), (1, 2, 0), (0, 2, 1), (1, 0, 2), (0, 1, 2), (1, 1, 1),
            (2, 2, 0), (2, 0, 2), (0, 2, 2), (2, 1, 1), (1, 2, 1), (1, 1, 2),
            (2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)]
    if lattice == "Q19":
        rows = [r for r in rows if sum(1 for k in r if k > 0) <= 2]
    return rows


def moment_matrix(C: np.ndarray, exps) -> np.ndarray:
    """M[i, j] = prod_a C[j, a] ** exps[i][a]  (eq. 5-2)."""
    q = C.shape[0]
    M = np.ones((len(exps), q))
    for i, ex in enumerate(exps):
        for a, k in enumerate(ex):
            M[i] *= C[:, a] ** k
    return M


def g_eq(C, w, c, cs2, A, B, Mt):
    """General rectangular equilibrium, eq. 3-3 with eq. 3-4 and c_sa = c_s.

    A: (N,), B: (d, N), Mt: (d, d, N) symmetric.  Returns (q, N).
    g_j = w_j (A + c~_j . B + Q~_j : M),  c~ = c_j / cs2,
    Q~_aa = Q_aa / (cs2 (c_a^2 - cs2)),  Q~_ab = Q_ab / (2 cs2^2) (a != b),
    Q_j = c_j c_j - cs2 I.
    """
    q, d = C.shape
    c = np.asarray(c, dtype=np.float64)
    Q = np.einsum("ja,jb->jab", C, C) - cs2 * np.eye(d)[None]
    Qt = np.empty_like(Q)
    for a in range(d):
        for b in range(d):
            if a == b:
                Qt[:, a, a] = Q[:, a, a] / (cs2 * (c[a] ** 2 - cs2))
            else:
                Qt[:, a, b] = Q[:, a, b] / (2.0 * cs2 * cs2)
    ct = C / cs2
    return w[:, None] * (A[None, :] + ct @ B + np.einsum("jab,abn->jn", Qt, Mt))


# --------------------------------------------------------------------------
# Relaxation rates and the second-order block (Sec. IV eq. 4-27 .. 4-31, Sec. V eq. 5-8)
# --------------------------------------------------------------------------

def nse_rates(c, cs2, nu, nu_b, d, dt=1.0):
    """Solve eq. 4-31 for the rates: s_ab (off-diagonal), s_s,a and s_b,a."""
    c = np.asarray(c, dtype=np.float64)
    s_ab = 1.0 / (0.5 + nu / (cs2 * dt))
    s_s = 1.0 / (0.5 + 2.0 * nu / ((c**2 - cs2) * dt))
    s_b = 1.0 / (0.5 + d * nu_b / ((c**2 - cs2) * dt))
    return s_ab, s_s, s_b


def S2_inverse_block(c, cs2, s_s, s_b, d):
    """S_2^(1) = diag(1/s_s) + a b^T / d of eq. 4-27-1."""
    c = np.asarray(c, dtype=np.float64)
    a = (1.0 / s_b - 1.0 / s_s) * (c**2 - cs2)
    b = 1.0 / (c**2 - cs2)
    return np.diag(1.0 / s_s) + np.outer(a, b) / d


def S2_sherman_morrison(c, cs2, s_s, s_b, d):
    """Closed-form inverse of eq. 5-8-1: A - A a~ b^T A / (1 + b^T A a~)."""
    c = np.asarray(c, dtype=np.float64)
    A = np.diag(s_s)
    a = (1.0 / s_b - 1.0 / s_s) * (c**2 - cs2)
    abar = a / d
    b = 1.0 / (c**2 - cs2)
    return A - (A @ np.outer(abar, b) @ A) / (1.0 + b @ A @ abar)


# --------------------------------------------------------------------------
# Model
# --------------------------------------------------------------------------

DEFAULTS = dict(lattice="Q9", equation="NSE", n=(8, 8, 1), dx=(1.0, 1.0, 1.0), dt=1.0,
                cs2=-1.0, nu=0.1, nu_b=-1.0, s_hi=-1.0, w_corner=-1.0,
                D0=0.0, D2=0.0, adv=(0.0, 0.0, 0.0), force=(0.0, 0.0, 0.0),
                source=0.0, rho0=1.0, wall_faces=0, incompressible=False, nu_tensor=None, nu_b_axis=None,
                gamma0=False, diffusive=False, c_zero=False, central=False, hermite=False,
                bhll=False)


class Model:
    """Dense FP64 RMRT-LB model for one rectangular domain."""

    def __init__(self, params: dict, solid: np.ndarray | None = None):
        p = dict(DEFAULTS)
        p.update(params)
        self.p = p
        self.lattice = p["lattice"]
        self.nse = p["equation"] == "NSE"
        self.linear = self.lattice in LINEAR_LATTICES                          # A18
        if self.linear and self.nse:
            raise ValueError("rD2Q5 / rD3Q7 carry the NCDE only (linear equilibrium)")
        # the C = 0 form of eq. 4-16 (G from dB/dt, history of phi): always on the
        # reduced lattices (A18), an option on the others (A23)
        self.c_zero = bool(p["c_zero"]) and not self.nse
        self.hist_form = self.linear or self.c_zero
        # central-moment (cascaded) collision, eq. 5-1-1 / 5-1-2 (A25)
        self.central = bool(p["central"])
        if self.central and not (self.nse and self.lattice in ("Q9", "Q27")):
            raise ValueError("the central-moment collision is built for the NSE on rD2Q9 and rD3Q27")
        # Hermite-moment collision (central-Hermite with central), eq. 5-1-1 / 5-1-2 (A26)
        self.hermite = bool(p["hermite"])
        if self.hermite and not (self.nse and self.lattice in ("Q9", "Q19", "Q27")):
            raise ValueError("the Hermite-moment collision is built for the NSE on rD2Q9, rD3Q19 and rD3Q27")
        # BHLL-moment collision, eq. Md2q9-3 with eq. 5-1-2 (A27)
        self.bhll = bool(p["bhll"])
        if self.bhll and not (self.nse and self.lattice == "Q9"):
            raise ValueError("the BHLL-moment collision is built for the NSE on rD2Q9")
        if self.bhll and (self.central or self.hermite):
            raise ValueError("the BHLL basis is not combined with the central or Hermite one")
        E = unit_offsets(self.lattice)
        self.E = E
        self.q, self.d = E.shape
        nx, ny, nz = (int(v) for v in p["n"])
        if self.d == 2:
            assert nz == 1
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.dt = float(p["dt"])
        c = np.array(p["dx"][: self.d], dtype=np.float64) / self.dt          # c_a = dx_a / dt
        self.c = c
        cs2 = float(p["cs2"])
        if cs2 <= 0:
            cs2 = float(np.min(c**2)) / 3.0                                    # A2
        self.cs2 = cs2
        self.C = E * c[None, :]
        self.opp = opposite(E)
        self.w = weights(self.lattice, c, cs2, p["w_corner"])
        self.exps = moment_exponents(self.lattice)
        self.M = moment_matrix(self.C, self.exps)
        self.Minv = np.linalg.inv(self.M)
        self.order = np.array([sum(e) for e in self.exps])
        self.rho0 = float(p["rho0"])
        self.force = np.array(p["force"][: self.d], dtype=np.float64)
        self.source = float(p["source"])
        self.adv = np.array(p["adv"][: self.d], dtype=np.float64)
        d, q = self.d, self.q
        row = {e: i for i, e in enumerate(self.exps)}
        unit = [tuple(1 if k == a else 0 for k in range(d)) for a in range(d)]
        self.row0 = row[tuple([0] * d)]
        self.rows1 = [row[unit[a]] for a in range(d)]
        self.rows2d = [row[tuple(2 * v for v in unit[a])] for a in range(d)]
        self.pairs = [(a, b) for a in range(d) for b in range(a + 1, d)]
        # off-diagonal second moments (absent on the reduced lattices)
        self.rows2o = [row[tuple(unit[a][k] + unit[b][k] for k in range(d))] for a, b in self.pairs
                       if tuple(unit[a][k] + unit[b][k] for k in range(d)) in row]

        S = np.zeros((q, q))
        self.hl = bool(p["incompressible"]) and self.nse                        # A19
        self.gamma0 = bool(p["gamma0"]) and not self.nse                       # A21
        self.diffusive = bool(p["diffusive"]) and not self.nse                 # A22
        self.half_src = 0.0 if (self.gamma0 or self.diffusive) else 0.5        # phi = sum f (+ dt S / 2)
        if self.nse:
            nu = float(p["nu"])
            nu_b = float(p["nu_b"])
            if nu_b < 0:
                nu_b = 2.0 * nu / d                                            # A11
            self.nu, self.nu_b = nu, nu_b
            s_ab, s_s, s_b = nse_rates(c, cs2, nu, nu_b, d, self.dt)
            self.s_ab, self.s_s, self.s_b = s_ab, s_s, s_b
            # viscosity tensor entries (A20): nu_t[a] diagonal, nu_pair[k] for pairs[k]
            nt = p["nu_tensor"] if p["nu_tensor"] is not None else [-1.0] * 6
            nb = p["nu_b_axis"] if p["nu_b_axis"] is not None else [-1.0] * 3
            self.nu_diag = np.array([float(nt[a]) if nt[a] > 0 else nu for a in range(d)])
            pair_slot = {(0, 1): 3, (0, 2): 4, (1, 2): 5}
            self.nu_pair = np.array([float(nt[pair_slot[pr]]) if nt[pair_slot[pr]] > 0 else nu for pr in self.pairs])
            self.nu_b_ax = np.array([float(nb[a]) if nb[a] > 0 else nu_b for a in range(d)])
            g = c**2 - cs2
            self.s_s = 1.0 / (0.5 + 2.0 * self.nu_diag / (g * self.dt))          # eq. 4-31, per entry
            self.s_b = 1.0 / (0.5 + d * self.nu_b_ax / (g * self.dt))
            self.s_pair = 1.0 / (0.5 + self.nu_pair / (cs2 * self.dt))
            s_s, s_b = self.s_s, self.s_b
            self.S2inv1 = S2_inverse_block(c, cs2, s_s, s_b, d)
            self.Sbar21 = np.linalg.inv(self.S2inv1)                           # eq. 5-8-1 (numeric)
            s_hi = float(p["s_hi"])
            if s_hi <= 0:
                s_hi = s_ab                                                    # A5
            self.s_hi = s_hi
            for i in range(q):
                if self.order[i] == 0 or self.order[i] == 1:
                    S[i, i] = 1.0                                              # A6
                elif self.order[i] >= 3:
                    S[i, i] = s_hi
            for a in range(d):
                for b in range(d):
                    S[self.rows2d[a], self.rows2d[b]] = self.Sbar21[a, b]
            for k, r in enumerate(self.rows2o):
                S[r, r] = self.s_pair[k]
        else:
            s_hi = float(p["s_hi"])
            if s_hi <= 0:
                s_hi = 1.0                                                     # A5 / A14
            self.s_hi = s_hi
            for i in range(q):
                if self.order[i] == 0:
                    S[i, i] = 1.0
                elif self.order[i] >= 2:
                    S[i, i] = s_hi
            # order-1 rows carry the local rate s_1(phi), added per node
        self.S = S
        self.P1 = np.zeros((q, q))
        for r in self.rows1:
            self.P1[r, r] = 1.0
        self._build_streaming(solid)
        self.S_node = self.F_node = self.S_prev = None
        self.S_central = None      # a relaxation matrix for the shifted basis other than S (tests only)
        self.S_bhll = self.bhll_relaxation() if self.bhll else None

    # ------------------------------------------------------------------ sources
    def set_sources(self, S=None, F=None):
        """Per-node source fields in place of the parameter set's constant source
        and force (eq. NSE, eq. NCDE): S (N,) the NSE mass source Sbar or the NCDE
        source S, F (d, N) the NSE body-force density Fbar; None for one of them
        means zero, None for both returns to the constants.  The previous-step
        source of the gamma = 0 form starts equal to S, so the first step sees no
        difference (A24)."""
        if S is None and F is None:
            self.S_node = self.F_node = self.S_prev = None
            return
        self.S_node = np.zeros(self.N) if S is None else np.array(S, dtype=np.float64).reshape(self.N)
        self.F_node = (np.zeros((self.d, self.N)) if F is None
                       else np.array(F, dtype=np.float64).reshape(self.d, self.N))
        self.S_prev = self.S_node.copy()

    def update_sources(self, S=None, F=None):
        """New values of the per-node fields for the following steps; the
        previous-step source keeps the values the last step used."""
        if S is not None:
            self.S_node = np.array(S, dtype=np.float64).reshape(self.N)
        if F is not None:
            self.F_node = np.array(F, dtype=np.float64).reshape(self.d, self.N)

    def _sources(self, n, sel):
        """Source, force and previous-step source of n nodes (the nodes `sel` of
        the domain, all when None): (S (n,), F (d, n), S_prev (n,))."""
        if self.S_node is None:
            S = np.full(n, self.source)
            return S, np.repeat(self.force[:, None], n, axis=1), S
        idx = slice(None) if sel is None else sel
        return self.S_node[idx], self.F_node[:, idx], self.S_prev[idx]

    # ---------------------------------------------------------------- geometry
    def _build_streaming(self, solid):
        nx, ny, nz = self.shape
        walls = int(self.p["wall_faces"])
        if solid is None:
            solid = np.zeros(self.N, dtype=bool)
        self.solid = np.asarray(solid, dtype=bool).reshape(self.N)
        self.fluid = ~self.solid
        idx = np.arange(self.N)
        x = idx % nx
        y = (idx // nx) % ny
        z = idx // (nx * ny)
        self.xyz = (x, y, z)
        E3 = np.zeros((self.q, 3), dtype=np.int64)
        E3[:, : self.d] = self.E
        self.target = np.empty((self.q, self.N), dtype=np.int64)
        self.bounce = np.zeros((self.q, self.N), dtype=bool)
        dims = (nx, ny, nz)
        for j in range(self.q):
            t = [x + E3[j, 0], y + E3[j, 1], z + E3[j, 2]]
            out_wall = np.zeros(self.N, dtype=bool)
            for a in range(3):
                lo = t[a] < 0
                hi = t[a] >= dims[a]
                if walls & (1 << (2 * a)):
                    out_wall |= lo
                if walls & (1 << (2 * a + 1)):
                    out_wall |= hi
                t[a] = np.mod(t[a], dims[a])
            lin = t[0] + nx * (t[1] + ny * t[2])
            self.target[j] = lin
            self.bounce[j] = out_wall | self.solid[lin]

    # -------------------------------------------------------------- equilibria
    def macroscopic(self, fbar, sel=None):
        """rho (or phi) and u from fbar, eq. 2-4-1 / eq. 2-4-2 (sel: the nodes of
        fbar when they are not all the domain's)."""
        S, F, _ = self._sources(fbar.shape[1], sel)
        if self.nse:
            rho = fbar.sum(axis=0) + self.dt * S / 2.0
            den = self.rho0 if self.hl else rho[None, :]                         # A19: rho0 u = j
            u = (self.C.T @ fbar + self.dt * F / 2.0) / den
            return rho, u
        phi = fbar.sum(axis=0) + self.half_src * self.dt * S
        return phi, np.repeat(self.adv[:, None], fbar.shape[1], axis=1)

    def s1_ncde(self, phi):
        """Local first-order rate from eq. 4-10 with beta = 1, K = D(phi) I."""
        D = self.p["D0"] * (1.0 + self.p["D2"] * phi**2)
        return 1.0 / (0.5 + D / (self.cs2 * self.dt))

    def distributions(self, fbar, phi_prev=None, sel=None):
        """f_eq, F and G of the node states in fbar (eq. NSEfeq/NSEFeq/NSEGeq,
        eq. 4-14/4-14-1, or eq. 4-16 in the C = 0 form, which needs the previous
        step's phi in phi_prev); sel: the nodes of fbar (all when None)."""
        d, n = self.d, fbar.shape[1]
        I = np.eye(d)[:, :, None]
        Sn, Fn, _ = self._sources(n, sel)
        if self.nse:
            rho, u = self.macroscopic(fbar, sel)
            rr = np.full_like(rho, self.rho0) if self.hl else rho                 # A19
            feq = g_eq(self.C, self.w, self.c, self.cs2, rho, rr[None] * u,
                       rr[None, None] * np.einsum("an,bn->abn", u, u))
            F = g_eq(self.C, self.w, self.c, self.cs2, Sn, Fn, -self.cs2 * Sn[None, None] * I)
            T = (np.einsum("an,bn->abn", u, Fn) + np.einsum("an,bn->abn", Fn, u)
                 + self.cs2 * Sn[None, None] * I)
            M2G = self._apply_I_minus_half_S2(T)
            G = g_eq(self.C, self.w, self.c, self.cs2, np.zeros(n), np.zeros((d, n)), M2G)
            return feq, F, G, None
        phi, u = self.macroscopic(fbar, sel)
        B = phi[None] * u
        F = g_eq(self.C, self.w, self.c, self.cs2, Sn, np.zeros((d, n)), np.zeros((d, d, n)))
        s1 = self.s1_ncde(phi)
        if self.diffusive:
            feq = g_eq(self.C, self.w, self.c, self.cs2, phi, B, np.zeros((d, d, n)))   # eq. 4-17
            M1G = np.zeros((d, n))
        elif self.hist_form:
            feq = g_eq(self.C, self.w, self.c, self.cs2, phi, B, np.zeros((d, d, n)))   # eq. 4-16a
            dBdt = u * (phi - phi_prev)[None] / self.dt                        # first-order difference
            M1G = (1.0 - s1[None] / 2.0) * dBdt                                # eq. 4-16b
        else:
            feq = g_eq(self.C, self.w, self.c, self.cs2, phi, B,
                       phi[None, None] * np.einsum("an,bn->abn", u, u))
            M1G = (1.0 - s1[None] / 2.0) * u * Sn[None]                        # eq. 4-11, B' = u_adv
        G = g_eq(self.C, self.w, self.c, self.cs2, np.zeros(n), M1G, np.zeros((d, d, n)))
        return feq, F, G, s1

    def source_difference(self, n, sel=None):
        """dt/2 times the explicit difference F(t) - F(t - dt) of the NCDE source
        distribution F_j = w_j S (eq. 4-14-1): the dt^2/2 dF/dt term of eq. 2-1
        with gamma = 0 (A21, A24); zero in the gamma = 1 form."""
        if not self.gamma0:
            return np.zeros((self.q, n))
        S, _, Sp = self._sources(n, sel)
        d = self.d
        return 0.5 * g_eq(self.C, self.w, self.c, self.cs2, S - Sp, np.zeros((d, n)), np.zeros((d, d, n)))

    def _second_order_vec(self, T):
        """Symmetric tensor -> vector over the second-order rows (diagonal then off-diagonal)."""
        return [T[a, a] for a in range(self.d)] + [T[a, b] for a, b in self.pairs]

    def _apply_I_minus_half_S2(self, T):
        """(I - S_2/2) acting on the second-order moment rows (eq. M2GComput a)."""
        rows = self.rows2d + self.rows2o
        S22 = self.S[np.ix_(rows, rows)]
        v = np.array(self._second_order_vec(T))
        v2 = v - 0.5 * np.einsum("ij,jn->in", S22, v)
        out = np.zeros_like(T)
        for a in range(self.d):
            out[a, a] = v2[a]
        for k, (a, b) in enumerate(self.pairs):
            out[a, b] = v2[self.d + k]
            out[b, a] = v2[self.d + k]
        return out

    def shift_matrix(self, u):
        """N(u) of eq. 5-1-1 for the central moments: row i (exponents a) holds
        prod_axis binom(a, b) (-u)^(a - b) at column k (exponents b <= a), so that
        N(u) M f = sum_j prod_axis (c_j - u)^a f_j.  u: (d, n); returns (q, q, n)."""
        q, n = self.q, u.shape[1]
        N = np.zeros((q, q, n))
        for i, ea in enumerate(self.exps):
            for k, eb in enumerate(self.exps):
                if all(b <= a for a, b in zip(ea, eb)):
                    v = np.ones(n)
                    for ax, (a, b) in enumerate(zip(ea, eb)):
                        v = v * math.comb(a, b) * (-u[ax]) ** (a - b)
                    N[i, k] = v
        return N

    def hermite_matrix(self):
        """H of A26: row i (exponents a) holds prod_axis h(a, b) at column k
        (exponents b), with h(a, a) = 1, h(2, 0) = -cs2 and 0 otherwise, so that
        H M f = sum_j prod_axis H_a(c_j) f_j (H_0 = 1, H_1 = xi, H_2 = xi^2 - cs2)."""
        q = self.q
        H = np.zeros((q, q))
        for i, ea in enumerate(self.exps):
            for k, eb in enumerate(self.exps):
                v = 1.0
                for a, b in zip(ea, eb):
                    if a == b:
                        continue
                    if a == 2 and b == 0:
                        v *= -self.cs2
                    else:
                        v = 0.0
                        break
                H[i, k] = v
        return H

    def bhll_matrix(self):
        """N of A27: the printed N_BHLL (eq. Md2q9-3) at a = c_y / c_x, times
        diag(c_x^-order) that turns the raw moments M into M_a."""
        a = self.c[1] / self.c[0]
        a2 = a * a
        Nb = np.array([
            [1, 0, 0, 0, 0, 0, 0, 0, 0],
            [0, 1, 0, 0, 0, 0, 0, 0, 0],
            [0, 0, 1, 0, 0, 0, 0, 0, 0],
            [-2 * a2 - 2, 0, 0, 3, 3, 0, 0, 0, 0],
            [-2 * a2 + 2, 0, 0, 3 * a2, -3 / a2, 0, 0, 0, 0],
            [0, 0, 0, 0, 0, 1, 0, 0, 0],
            [0, -2, 0, 0, 0, 0, 3 / a2, 0, 0],
            [0, 0, -2, 0, 0, 0, 0, 3, 0],
            [4, 0, 0, -6, -6 / a2, 0, 0, 0, 9 / a2]], dtype=np.float64)
        # the printed matrix acts on the rows (1, x, y, x^2, y^2, xy, xy^2, x^2y, x^2y^2)
        assert [tuple(e) for e in self.exps] == [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1),
                                                 (1, 2), (2, 1), (2, 2)]
        return Nb @ np.diag(self.c[0] ** (-self.order.astype(np.float64)))

    def bhll_relaxation(self):
        """Sbar of A27 in the BHLL basis: the blocks of N S N^-1 between moments
        of one order, nothing between orders."""
        N = self.bhll_matrix()
        full = N @ self.S @ np.linalg.inv(N)
        same_order = self.order[:, None] == self.order[None, :]
        return np.where(same_order, full, 0.0)

    def basis_matrix(self, u):
        """The basis change N of eq. 5-1-1 per node: N(u) (central), H
        (hermite), H N(u) (both), N_BHLL M_a M^-1 (bhll).  u: (d, n); returns
        (q, q, n)."""
        n = u.shape[1]
        if self.bhll:
            return np.repeat(self.bhll_matrix()[:, :, None], n, axis=2)
        N = self.shift_matrix(u) if self.central else np.repeat(np.eye(self.q)[:, :, None], n, axis=2)
        if self.hermite:
            N = np.einsum("ik,kjn->ijn", self.hermite_matrix(), N)
        return N

    def _basis_relaxation(self):
        """Sbar of the basis collisions: a test's override, the BHLL blocks
        (A27), or the raw model's blocks (A25, A26)."""
        if self.S_central is not None:
            return self.S_central
        return self.S_bhll if self.bhll else self.S

    def apply_S(self, x, s1=None):
        """S x with S the block relaxation matrix; NCDE adds s_1(phi) on the first-order rows."""
        y = self.S @ x
        if s1 is not None:
            y = y + s1[None, :] * (self.P1 @ x)
        return y

    # --------------------------------------------------------------- collision
    def collide(self, fbar, phi_prev=None, sel=None):
        """Post-collision fbar* in moment space, eq. 2-2-3 (before propagation)."""
        feq, F, G, s1 = self.distributions(fbar, phi_prev, sel)
        m = self.M @ fbar
        meq = self.M @ feq
        mF = self.M @ F
        mG = self.M @ G
        if self.central or self.hermite or self.bhll:
            # the same step in the moments kappa = N m of the central (A25),
            # Hermite or central-Hermite (A26) or BHLL (A27) basis of eq. 5-1-1,
            # whose relaxation matrix Sbar has this model's blocks (eq. 5-1-2)
            _, u = self.macroscopic(fbar, sel)
            N = self.basis_matrix(u)
            k, keq, kF, kG = (np.einsum("ikn,kn->in", N, v) for v in (m, meq, mF, mG))
            Sb = self._basis_relaxation()
            kstar = k - Sb @ (k - keq) + self.dt * (kG + kF - 0.5 * (Sb @ kF))
            mstar = np.stack([np.linalg.solve(N[:, :, j], kstar[:, j]) for j in range(kstar.shape[1])], axis=1)
            return np.linalg.solve(self.M, mstar)
        mD = self.M @ self.source_difference(fbar.shape[1], sel)
        # gamma = 1 (eq. 2-3): dt (G + (I - Lambda/2) F); gamma = 0 (eq. 2-1, A21):
        # dt (G + F + (F(t) - F(t - dt)) / 2)
        mstar = (m - self.apply_S(m - meq, s1) + self.dt * (mG + mF - self.half_src * self.apply_S(mF, s1))
                 + self.dt * mD)
        return np.linalg.solve(self.M, mstar)

    def collide_velocity_space(self, fbar, phi_prev=None, sel=None):
        """Same collision written in velocity space with Lambda = M^-1 S M (eq. 2-3, eq. 5-1)."""
        feq, F, G, s1 = self.distributions(fbar, phi_prev, sel)
        if self.central or self.hermite or self.bhll:
            _, u = self.macroscopic(fbar, sel)
            N = self.basis_matrix(u)
            Sb = self._basis_relaxation()
            # per node: Lambda = M^-1 N^-1 Sbar N M (eq. 5-1-2)
            Lam_n = np.stack([self.Minv @ np.linalg.solve(N[:, :, j], Sb @ N[:, :, j]) @ self.M
                              for j in range(fbar.shape[1])], axis=2)

            def Lam(x):
                return np.einsum("jkn,kn->jn", Lam_n, x)
        else:
            def Lam(x):
                return self.Minv @ self.apply_S(self.M @ x, s1)

        return (fbar - Lam(fbar - feq) + self.dt * (G + F - self.half_src * Lam(F))
                + self.dt * self.source_difference(fbar.shape[1], sel))

    # ------------------------------------------------------------- propagation
    def stream(self, fstar, fprev):
        """Propagation (eq. 2-2) with halfway bounce-back (reading A10).

        Fluid nodes push fstar_j to x + e_j; a population whose target is a
        wall or a solid node returns to its own node in direction opp(j).
        Solid nodes keep their previous content."""
        out = fprev.copy()
        fl = self.fluid
        for j in range(self.q):
            go = fl & ~self.bounce[j]
            out[j, self.target[j, go]] = fstar[j, go]
            back = fl & self.bounce[j]
            out[self.opp[j], back] = fstar[j, back]
        return out

    def step(self, fbar, nsteps=1, hist=None):
        """nsteps collide-and-stream steps.  In the C = 0 form (the reduced
        lattices, A18, or the c_zero option, A23) hist is the previous step's
        phi per node (init_history gives it at t = 0) and the call returns
        (fbar, hist); otherwise it returns fbar."""
        if self.hist_form != (hist is not None):
            raise ValueError("hist is required in the C = 0 form and meaningless elsewhere")
        fl = self.fluid
        sel = np.flatnonzero(fl)
        if hist is not None:
            hist = np.array(hist, dtype=np.float64).reshape(self.N)
        for _ in range(nsteps):
            fstar = fbar.copy()
            if self.hist_form:
                phi, _ = self.macroscopic(fbar[:, fl], sel)
                fstar[:, fl] = self.collide(fbar[:, fl], hist[fl], sel)
                hist[fl] = phi
            else:
                fstar[:, fl] = self.collide(fbar[:, fl], sel=sel)
            fbar = self.stream(fstar, fbar)
            if self.S_node is not None:
                self.S_prev = self.S_node.copy()                               # F(t - dt) of the next step
        return fbar if hist is None else (fbar, hist)

    def init_history(self, phi):
        """phi(t - dt) at t = 0 in the C = 0 form: the initial phi (A18, A23)."""
        return np.array(phi, dtype=np.float64).reshape(self.N)

    # ------------------------------------------------------- local gradients
    def local_gradients(self, fbar, hist=None):
        """Local (no finite differences) derivative outputs of a state.

        NSE: the generalized shear stress of eq. 4-32-0 (first line),
            tau = -(I - S_2/2) [m_2^ne + dt/2 (u F + F u + (cs2 I - u u) S)],
        with m_2^ne = sum_k c_k c_k f_k^ne, f = fbar + dt F / 2 (eq. 2-3), and the
        strain rate E = (grad u + grad u^T) / 2 from eq. 4-28 with the isotropic
        tensors K_mu = rho nu I, K_mu_b = rho nu_b I of eq. 4-31:
            tr E = tr tau / (d rho nu_b),  E = (tau - (rho nu_b - 2 rho nu / d) tr E I) / (2 rho nu).
        Returns (tau, E), each (d, d, N).

        NCDE: grad phi from eq. 4-13 with D = phi I and K = D(phi) I:
            -D(phi) grad phi = (1 - s_1/2) (m_1^ne + dt/2 X),
        X = u_adv S for C = phi u u (first branch) or the dB/dt of eq. 4-16
        (second branch, reduced lattices; hist = phi of the previous step).
        Returns grad phi, (d, N)."""
        d = self.d
        n = fbar.shape[1]
        feq, F, G, s1 = self.distributions(fbar, hist)
        fne = fbar + self.half_src * self.dt * F - feq
        Sn, Fn, _ = self._sources(n, None)
        if self.nse:
            rho, u = self.macroscopic(fbar)
            I = np.eye(d)[:, :, None]
            m2ne = np.einsum("ja,jb,jn->abn", self.C, self.C, fne)
            T = (np.einsum("an,bn->abn", u, Fn) + np.einsum("an,bn->abn", Fn, u)
                 + (self.cs2 * I - np.einsum("an,bn->abn", u, u)) * Sn[None, None])
            tau = -self._apply_I_minus_half_S2(m2ne + 0.5 * self.dt * T)
            rr = np.full_like(rho, self.rho0) if self.hl else rho
            # invert eq. 4-28 with the tensors of eq. 4-29:
            #   tau_ab = K_ab 2 E_ab (a != b),
            #   tau_aa = K_aa (2 E_aa - (2/d) tr E) + Kb_a tr E
            E = np.zeros_like(tau)
            Kd = rr[None] * self.nu_diag[:, None]
            Kb = rr[None] * self.nu_b_ax[:, None]
            num = sum(tau[a, a] / (2.0 * Kd[a]) for a in range(d))
            den = 1.0 + sum((Kb[a] - 2.0 * Kd[a] / d) / (2.0 * Kd[a]) for a in range(d))
            trE = num / den
            for a in range(d):
                E[a, a] = (tau[a, a] - (Kb[a] - 2.0 * Kd[a] / d) * trE) / (2.0 * Kd[a])
            for k, (a, b) in enumerate(self.pairs):
                E[a, b] = E[b, a] = tau[a, b] / (2.0 * rr * self.nu_pair[k])
            return tau, E
        phi, u = self.macroscopic(fbar)
        m1ne = self.C.T @ fne
        if self.diffusive:
            X = np.zeros_like(u)
        elif self.hist_form:
            X = u * (phi - hist)[None] / self.dt
        else:
            X = u * Sn[None]
        D = self.p["D0"] * (1.0 + self.p["D2"] * phi**2)
        return -(1.0 - 0.5 * s1)[None] * (m1ne + 0.5 * self.dt * X) / D[None]

    # ---------------------------------------------------------- initialisation
    def init(self, rho, u, with_fne=False):
        """fbar(t=0) = f_eq(rho, u) - dt F / 2 [+ f_ne from eq. fne].

        rho (or phi): (N,); u: (d, N) (ignored for the NCDE, which uses u_adv)."""
        n = self.N
        d = self.d
        rho = np.asarray(rho, dtype=np.float64).reshape(n)
        I = np.eye(d)[:, :, None]
        Sn, Fn, _ = self._sources(n, None)
        if self.nse:
            u = np.asarray(u, dtype=np.float64).reshape(d, n)
            rr = np.full_like(rho, self.rho0) if self.hl else rho                 # A19
            Mt = rr[None, None] * np.einsum("an,bn->abn", u, u)
            if with_fne:
                Mt = Mt + self.m2_ne(rr, u)
            feq = g_eq(self.C, self.w, self.c, self.cs2, rho, rr[None] * u, Mt)
            F = g_eq(self.C, self.w, self.c, self.cs2, Sn, Fn, -self.cs2 * Sn[None, None] * I)
        else:
            u = np.repeat(self.adv[:, None], n, axis=1)
            Mt = (np.zeros((d, d, n)) if (self.hist_form or self.diffusive)
                  else rho[None, None] * np.einsum("an,bn->abn", u, u))
            feq = g_eq(self.C, self.w, self.c, self.cs2, rho, rho[None] * u, Mt)
            F = g_eq(self.C, self.w, self.c, self.cs2, Sn, np.zeros((d, n)), np.zeros((d, d, n)))
        return feq - self.half_src * self.dt * F

    def velocity_gradient(self, u):
        """grad[a, b] = d u_a / d x_b; central differences, one-sided next to walls/solids."""
        d, n = self.d, self.N
        nx, ny, nz = self.shape
        walls = int(self.p["wall_faces"])
        x, y, z = self.xyz
        coords = [x, y, z]
        dims = (nx, ny, nz)
        g = np.zeros((d, d, n))
        for b in range(d):
            nbr = []
            for s in (+1, -1):
                t = [x.copy(), y.copy(), z.copy()]
                t[b] = coords[b] + s
                ok = np.ones(n, dtype=bool)
                if s < 0 and (walls & (1 << (2 * b))):
                    ok &= t[b] >= 0
                if s > 0 and (walls & (1 << (2 * b + 1))):
                    ok &= t[b] < dims[b]
                t[b] = np.mod(t[b], dims[b])
                lin = t[0] + nx * (t[1] + ny * t[2])
                ok &= self.fluid[lin]
                nbr.append((lin, ok))
            (lp, okp), (lm, okm) = nbr
            h = self.c[b] * self.dt
            for a in range(d):
                both = okp & okm
                g[a, b, both] = (u[a, lp[both]] - u[a, lm[both]]) / (2 * h)
                po = okp & ~okm
                g[a, b, po] = (u[a, lp[po]] - u[a, po]) / h
                mo = okm & ~okp
                g[a, b, mo] = (u[a, mo] - u[a, lm[mo]]) / h
        return g

    def m2_ne(self, rho, u):
        """m_2^ne = -(I - S_2/2)^-1 tau - dt/2 (u F + F u + cs2 S I)  (eq. 4-34, eq. 4-28)."""
        d, n = self.d, self.N
        g = self.velocity_gradient(u)
        div = np.einsum("aan->n", g)
        I = np.eye(d)[:, :, None]
        # eq. 4-28 with the tensors of eq. 4-29 (A20)
        tau = np.zeros((d, d, n))
        for a in range(d):
            tau[a, a] = rho * (self.nu_diag[a] * (2.0 * g[a, a] - (2.0 / d) * div) + self.nu_b_ax[a] * div)
        for k, (a, b) in enumerate(self.pairs):
            tau[a, b] = tau[b, a] = rho * self.nu_pair[k] * (g[a, b] + g[b, a])
        rows = self.rows2d + self.rows2o
        S22 = self.S[np.ix_(rows, rows)]
        K = np.linalg.inv(np.eye(len(rows)) - 0.5 * S22)
        v = np.einsum("ij,jn->in", K, np.array(self._second_order_vec(tau)))
        out = np.zeros((d, d, n))
        for a in range(d):
            out[a, a] = -v[a]
        for k, (a, b) in enumerate(self.pairs):
            out[a, b] = -v[d + k]
            out[b, a] = -v[d + k]
        Sn, Fn, _ = self._sources(n, None)
        out -= 0.5 * self.dt * (np.einsum("an,bn->abn", u, Fn) + np.einsum("an,bn->abn", Fn, u)
                                + self.cs2 * Sn[None, None] * I)
        return out


# --------------------------------------------------------------------------
# Closed-form solutions used to pin the oracle (exact solutions of the PDEs the
# scheme recovers: eq. NSE, eq. 4-15)
# --------------------------------------------------------------------------

def gaussian_hill(xp, yp, t, sigma0, D, xc, yc, adv, Lx, Ly, images=2):
    """2D advected Gaussian with constant diffusivity on a periodic box (peak 1 at t = 0)."""
    s2 = sigma0**2 + 2.0 * D * t
    amp = sigma0**2 / s2
    out = np.zeros_like(xp, dtype=np.float64)
    for i in range(-images, images + 1):
        for k in range(-images, images + 1):
            dx = xp - (xc + adv[0] * t) - i * Lx
            dy = yp - (yc + adv[1] * t) - k * Ly
            out += amp * np.exp(-(dx**2 + dy**2) / (2.0 * s2))
    return out


def gaussian_hill_nd(coords, t, sigma0, D, centre, adv, L, images=2):
    """d-dimensional advected Gaussian with constant diffusivity on a periodic
    box (peak 1 at t = 0); the advected centre is wrapped into the box before
    the periodic images are summed."""
    d = len(coords)
    s2 = sigma0**2 + 2.0 * D * t
    out = np.full(np.shape(coords[0]), (sigma0**2 / s2) ** (d / 2.0))
    for a in range(d):
        xc = np.mod(centre[a] + adv[a] * t, L[a])
        acc = np.zeros(np.shape(coords[a]))
        for i in range(-images, images + 1):
            acc += np.exp(-((coords[a] - xc - i * L[a]) ** 2) / (2.0 * s2))
        out = out * acc
    return out


def poiseuille(yc, H, g, nu):
    """Plane channel profile u(y) = g y (H - y) / (2 nu)."""
    return g * yc * (H - yc) / (2.0 * nu)
