"""GPU parity of the Hermite-moment and central-Hermite-moment collisions
(hermite = 1, with or without central = 1; eq. 5-1-1 / 5-1-2, reading A26)
against the FP64 oracle on rD2Q9, rD3Q19 and rD3Q27: periodic and walled
domains, solids, body force and source, both memory patterns, FP64 (1e-12
of max |f|) and FP32 deviation storage (rho within 1e-5 of rho0, u within
1e-5 of its scale), a batch; central-Hermite is refused on rD3Q19, local
outputs with either."""
import sys

import numpy as np
import pytest

from gpu_util import WALLS, circle_mask, random_fields, rel_err
from oracle import rmrt_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_00366_amd import rmrt
    return rmrt


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "q9_periodic": (dict(lattice="Q9", n=(37, 23, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05, s_hi=1.4), None, 25),
    "q9_channel_solid_force": (dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, s_hi=1.2,
                                    force=(2e-5, 1e-6, 0.0), source=1e-6, wall_faces=WALLS["y"]),
                               lambda n: circle_mask(n, (12, 10), 4), 25),
    "q19_periodic": (dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.05, s_hi=1.5), None, 15),
    "q19_walls_force": (dict(lattice="Q19", n=(14, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05, s_hi=1.3,
                             force=(1e-5, 0.0, 2e-6), wall_faces=WALLS["yz"]), None, 15),
    "q27_periodic": (dict(lattice="Q27", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.01, s_hi=1.3), None, 15),
    "q27_walls_force_solid": (dict(lattice="Q27", n=(14, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05, s_hi=1.2,
                                   force=(1e-5, 0.0, 2e-6), wall_faces=WALLS["yz"]),
                              lambda n: circle_mask(n, (6, 4), 2), 15),
}
VARIANTS = [(c, False) for c in CASES] + [(c, True) for c in CASES if not c.startswith("q19")]


def _case(R, case, central, storage, pattern):
    prm, solid_fn, steps = CASES[case]
    prm = dict(prm, hermite=True, central=central)
    solid = None if solid_fn is None else solid_fn(prm["n"])
    m = O.Model(prm, solid=solid)
    rho, u = random_fields(m, sum(map(ord, case)) % 991 + (7 if central else 0))
    dom = R.Domain(R.make_params(**prm, storage=storage, pattern=pattern), rho, u,
                   solid=None if solid is None else solid.astype(np.uint8))
    return m, dom, rho, u, steps


_oracle = {}


def _oracle_run(key, m, rho, u, steps):
    if key not in _oracle:
        _oracle[key] = m.step(m.init(rho, u), steps)
    return _oracle[key]


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case,central", VARIANTS)
def test_hermite_collision_matches_oracle(R, case, central, pattern, storage):
    m, dom, rho, u, steps = _case(R, case, central, storage, pattern)
    f_or = _oracle_run((case, central), m, rho, u, steps)
    dom.step(steps)
    fl = m.fluid
    label = f"{case} {'central-' if central else ''}Hermite {pattern} {storage}"
    if storage == "f64":
        err = rel_err(dom.populations().cpu().numpy()[:, fl], f_or[:, fl])
        say(f"[hermite] {label}: {err:.2e}")
        assert err < 1e-12
    else:
        r_g, u_g = (t.cpu().numpy() for t in dom.moments())
        r_o, u_o = m.macroscopic(f_or)
        er = np.abs(r_g[fl] - r_o[fl]).max()
        eu = np.abs(u_g[:, fl] - u_o[:, fl]).max() / np.abs(u_o).max()
        say(f"[hermite] {label}: rho {er:.2e}, u {eu:.2e}")
        assert er < 1e-5 and eu < 1e-5
    dom.close()


def test_hermite_differs_from_raw_and_central(R):
    """s_hi differs from the second-order rates: the Hermite step is neither the
    raw nor the central one, and both GPU runs match their oracles."""
    prm = dict(CASES["q27_periodic"][0])
    m_r = O.Model(prm)
    rho, u = random_fields(m_r, 8)
    out = {}
    for lab, extra in (("raw", {}), ("hermite", dict(hermite=True)), ("central", dict(central=True)),
                       ("central_hermite", dict(central=True, hermite=True))):
        m = O.Model(dict(prm, **extra))
        f_or = m.step(m.init(rho, u), 9)
        dom = R.Domain(R.make_params(**prm, **extra, storage="f64", pattern="AA"), rho, u)
        dom.step(9)
        fg = dom.populations().cpu().numpy()
        dom.close()
        assert rel_err(fg, f_or) < 1e-12, lab
        out[lab] = fg
    for a in out:
        for b in out:
            if a < b:
                assert rel_err(out[a], out[b]) > 1e-9, (a, b)


def test_hermite_batch_matches_oracle(R):
    prms = [dict(CASES["q19_periodic"][0], hermite=True),
            dict(lattice="Q19", n=(9, 13, 7), dx=(1.0, 2.0, 1.0), nu=0.08, s_hi=1.2, force=(1e-5, 0.0, 0.0),
                 wall_faces=WALLS["yz"], hermite=True)]
    b = R.Batch([R.make_params(**p, storage="f64", pattern="AA") for p in prms])
    refs = []
    for k, p in enumerate(prms):
        m = O.Model(p)
        rho, u = random_fields(m, 30 + k)
        b.domains[k].set_fields(rho, u)
        refs.append(m.step(m.init(rho, u), 12))
    b.step(12)
    for k in range(len(prms)):
        assert rel_err(b.domains[k].populations().cpu().numpy(), refs[k]) < 1e-12
    b.close()


def test_hermite_refused_where_not_built(R):
    with pytest.raises(R.RMRTError) as e:
        R.derive(R.make_params(lattice="Q19", n=(4, 4, 4), nu=0.05, hermite=True, central=True))
    assert e.value.code == R.EUNSUPPORTED
    with pytest.raises(R.RMRTError) as e:
        R.derive(R.make_params(lattice="Q9", equation="NCDE", n=(4, 4, 1), D0=0.05, hermite=True))
    assert e.value.code == R.EINVAL
    prm = dict(CASES["q19_periodic"][0], hermite=True)
    m = O.Model(prm)
    rho, u = random_fields(m, 1)
    dom = R.Domain(R.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    with pytest.raises(R.RMRTError) as e:
        dom.local_gradients(R.GRAD_STRAIN)
    assert e.value.code == R.EUNSUPPORTED
    dom.close()
    # a batch mixing the raw and the Hermite collision is refused
    with pytest.raises(R.RMRTError) as e:
        R.Batch([R.make_params(**CASES["q19_periodic"][0], storage="f64", pattern="AA"),
                 R.make_params(**prm, storage="f64", pattern="AA")])
    assert e.value.code == R.EINVAL
