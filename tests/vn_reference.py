"""Von Neumann analysis of the oracle's collide-and-stream step (test
infrastructure for rmrt_preflight): the Jacobian J of the oracle's collision
(eq. 2-2-3) at a uniform state, by central differences on one node, and the
amplification matrices A(k) = diag(exp(-i k . e_j)) J of the linearised step
for a Fourier mode exp(i k . x) (streaming moves population j by e_j nodes,
eq. 2-2).  The largest |eigenvalue| over the wave vectors of a periodic grid
is what a growing perturbation on that grid measures."""
import itertools

import numpy as np

from oracle import rmrt_oracle as O


def jacobian(m, rho0, u0, eps=1e-6):
    """Jacobian of one node's update at the uniform state.  Without a history
    it is d f* / d f (q x q).  In the C = 0 form (eq. 4-16) the state is (f,
    phi_prev): the collision reads phi_prev and the step stores the new
    phi_prev = phi(f) (eq. 2-4-1) before colliding, so the matrix is
    (q + 1) x (q + 1) with last row d phi / d f and a zero corner."""
    u = np.zeros((m.d, 1)) if u0 is None else np.array(u0[: m.d], dtype=np.float64).reshape(m.d, 1)
    f0 = m.init(np.array([rho0], dtype=np.float64), u)
    hist = m.hist_form
    h0 = np.array([rho0], dtype=np.float64)
    n = m.q + (1 if hist else 0)
    J = np.zeros((n, n))

    def post(f, h):
        fs = m.collide(f, h) if hist else m.collide(f)
        if not hist:
            return fs[:, 0]
        phi, _ = m.macroscopic(f)
        return np.concatenate([fs[:, 0], phi])

    for j in range(n):
        fp, fm, hp, hm = f0.copy(), f0.copy(), h0.copy(), h0.copy()
        if j < m.q:
            fp[j] += eps
            fm[j] -= eps
        else:
            hp += eps
            hm -= eps
        J[:, j] = (post(fp, hp) - post(fm, hm)) / (2.0 * eps)
    return J


def amplification(m, J, k):
    """A(k) for a wave vector k in radians per node along each axis: the
    populations stream, the history (when present) stays at its node."""
    phase = np.exp(-1j * (m.E @ np.asarray(k, dtype=np.float64)))
    if J.shape[0] > m.q:
        phase = np.concatenate([phase, [1.0]])
    return phase[:, None] * J


def max_amplification(prm, rho0, u0, grid):
    """max over the nonzero wave vectors 2 pi m / grid of max |eig A(k)|."""
    m = O.Model(dict(prm, n=(1, 1, 1)))
    J = jacobian(m, rho0, u0)
    best = 0.0
    for mm in itertools.product(*(range(g) for g in grid[: m.d])):
        if not any(mm):
            continue
        k = 2.0 * np.pi * np.array(mm) / np.array(grid[: m.d])
        best = max(best, np.abs(np.linalg.eigvals(amplification(m, J, k))).max())
    return best
