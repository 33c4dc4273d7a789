"""FP16 deviation storage under the alternative moment bases (eq. 5-1-1 /
5-1-2, readings A25-A27): central, Hermite, central-Hermite and BHLL steps
on rD2Q9 / rD3Q19 / rD3Q27 against the FP64 oracle, with the bar of the
raw-moment FP16 parity (rho within 3e-3 of rho0, u within 3e-3 of its
scale)."""
import sys

import numpy as np
import pytest

from gpu_util import WALLS, random_fields
from oracle import rmrt_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_00366_amd import rmrt
    return rmrt


CASES = {
    "q9_bhll": dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, nu_b=0.08, s_hi=1.3,
                    force=(2e-5, 0.0, 0.0), wall_faces=WALLS["y"], bhll=True),
    "q9_central_hermite": dict(lattice="Q9", n=(37, 23, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05, s_hi=1.4,
                               central=True, hermite=True),
    "q19_hermite": dict(lattice="Q19", n=(14, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05, s_hi=1.3,
                        force=(1e-5, 0.0, 2e-6), wall_faces=WALLS["yz"], hermite=True),
    "q27_central": dict(lattice="Q27", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.01, s_hi=1.3,
                        central=True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_basis_collision_fp16_storage(R, case):
    print(f"[basis f16] {case}", flush=True)
    sys.stdout.flush()
    prm = CASES[case]
    m = O.Model(prm)
    rho, u = random_fields(m, sum(map(ord, case)) % 977)
    f_or = m.step(m.init(rho, u), 20)
    dom = R.Domain(R.make_params(**prm, storage="f16dev", pattern="AA"), rho, u)
    dom.step(20)
    r_g, u_g = (t.cpu().numpy() for t in dom.moments())
    dom.close()
    r_o, u_o = m.macroscopic(f_or)
    er = np.abs(r_g - r_o).max() / m.rho0
    eu = np.abs(u_g - u_o).max() / np.abs(u_o).max()
    print(f"   rho err {er:.2e}, u err {eu:.2e}", flush=True)
    assert er < 3e-3 and eu < 3e-3
