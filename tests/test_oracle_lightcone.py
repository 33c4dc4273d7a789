"""The light-cone evolution used by the full-size multi-step GPU checks
(tests/gpu_util.lightcone_oracle) against the oracle stepping the whole domain:
after k steps a node's populations depend only on the initial state within k
nodes per axis, so the staged sub-box evolution must reproduce the whole-domain
result at that node, at corners, next to walls and across periodic faces."""
import numpy as np
import pytest

from gpu_util import lightcone_oracle, random_fields
from oracle import rmrt_oracle as O

CASES = [
    dict(lattice="Q9", equation="NCDE", n=(40, 30, 1), dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0, adv=(0.05, 0.02, 0.0),
         rho0=0.0),
    dict(lattice="Q9", n=(25, 14, 1), dx=(1.0, 0.5, 1.0), nu=0.05, force=(1e-5, 0.0, 0.0), wall_faces=4 | 8),
    dict(lattice="Q19", n=(20, 18, 16), dx=(1.0, 1.0, 2.0), nu=0.01, cs2=1.0 / 3.0),
    dict(lattice="Q27", n=(21, 9, 30), dx=(1.0, 0.5, 2.0), nu=0.05, force=(1e-5, 0.0, 0.0), wall_faces=4 | 8 | 16 | 32),
    dict(lattice="Q27", n=(21, 9, 30), dx=(1.0, 0.5, 2.0), nu=0.05, force=(1e-5, 0.0, 0.0), wall_faces=4 | 8),
]


@pytest.mark.parametrize("k", [1, 2, 5])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_lightcone_equals_whole_domain(case, k):
    prm = CASES[case]
    m = O.Model(prm)
    rho, u = random_fields(m, seed=3)
    if not m.nse:
        u = None
    full = m.step(m.init(rho, u), k)
    nx, ny, nz = m.shape
    rng = np.random.default_rng(case)
    nodes = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, 1, nz - 2), (3, ny - 2, 0)]
    nodes += [tuple(int(rng.integers(0, s)) for s in m.shape) for _ in range(3)]
    for node in nodes:
        got, _ = lightcone_oracle(prm, rho, u, node, k)
        i = node[0] + nx * (node[1] + ny * node[2])
        assert np.abs(got - full[:, i]).max() <= 1e-14 * np.abs(full).max(), (node, k)
