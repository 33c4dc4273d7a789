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
    u = np.zeros((m.d, 1)) if u0 is None else np.array(u0[: m.d], dtype=np.float64).reshape(m.d, 1)
    f0 = m.init(np.array([rho0], dtype=np.float64), u)
    J = np.zeros((m.q, m.q))
    for j in range(m.q):
        fp, fm = f0.copy(), f0.copy()
        fp[j] += eps
        fm[j] -= eps
        J[:, j] = (m.collide(fp) - m.collide(fm))[:, 0] / (2.0 * eps)
    return J


def amplification(m, J, k):
    """A(k) for a wave vector k in radians per node along each axis."""
    phase = np.exp(-1j * (m.E @ np.asarray(k, dtype=np.float64)))
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
