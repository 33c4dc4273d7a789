"""GPU parity of the BHLL-moment collision (bhll = 1: the orthogonal rD2Q9
basis of Sec. V, eq. Md2q9-3, with eq. 5-1-2; reading A27) against the FP64
oracle: periodic and walled domains, solids, body force and source, c_x other
than 1, both memory patterns, FP64 (1e-12 of max |f|) and FP32 deviation
storage (rho within 1e-5 of rho0, u within 1e-5 of its scale), a batch; the
step differs from the raw one; other lattices, the NCDE and mixed bases are
refused, and so are local outputs."""
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
    "periodic": (dict(lattice="Q9", n=(37, 23, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05, s_hi=1.4), None, 25),
    "channel_solid_force": (dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05, s_hi=1.2,
                                 force=(2e-5, 1e-6, 0.0), source=1e-6, wall_faces=WALLS["y"]),
                            lambda n: circle_mask(n, (12, 10), 4), 25),
    "cx2_walls": (dict(lattice="Q9", n=(29, 18, 1), dx=(2.0, 1.0, 1.0), nu=0.1, nu_b=0.3, s_hi=1.1,
                       force=(1e-5, 0.0, 0.0), wall_faces=WALLS["y"]), None, 20),
    "square": (dict(lattice="Q9", n=(24, 20, 1), dx=(1.0, 1.0, 1.0), nu=0.03, nu_b=0.08, s_hi=1.6), None, 20),
}


def _case(R, case, storage, pattern):
    prm, solid_fn, steps = CASES[case]
    prm = dict(prm, bhll=True)
    solid = None if solid_fn is None else solid_fn(prm["n"])
    m = O.Model(prm, solid=solid)
    rho, u = random_fields(m, sum(map(ord, case)) % 991)
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
@pytest.mark.parametrize("case", list(CASES))
def test_bhll_collision_matches_oracle(R, case, pattern, storage):
    m, dom, rho, u, steps = _case(R, case, storage, pattern)
    f_or = _oracle_run(case, m, rho, u, steps)
    dom.step(steps)
    fl = m.fluid
    label = f"{case} BHLL {pattern} {storage}"
    if storage == "f64":
        err = rel_err(dom.populations().cpu().numpy()[:, fl], f_or[:, fl])
        say(f"[bhll] {label}: {err:.2e}")
        assert err < 1e-12
    else:
        r_g, u_g = (t.cpu().numpy() for t in dom.moments())
        r_o, u_o = m.macroscopic(f_or)
        er = np.abs(r_g[fl] - r_o[fl]).max()
        eu = np.abs(u_g[:, fl] - u_o[:, fl]).max() / np.abs(u_o).max()
        say(f"[bhll] {label}: rho {er:.2e}, u {eu:.2e}")
        assert er < 1e-5 and eu < 1e-5
    dom.close()


def test_bhll_differs_from_raw_and_hermite(R):
    """s_hi differs from the second-order block: the BHLL step is neither the
    raw nor the Hermite one, and each GPU run matches its oracle."""
    prm = dict(CASES["periodic"][0])
    m_r = O.Model(prm)
    rho, u = random_fields(m_r, 8)
    out = {}
    for lab, extra in (("raw", {}), ("bhll", dict(bhll=True)), ("hermite", dict(hermite=True))):
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


def test_bhll_batch_matches_oracle(R):
    prms = [dict(CASES["periodic"][0], bhll=True),
            dict(lattice="Q9", n=(19, 31, 1), dx=(1.0, 2.0, 1.0), nu=0.08, s_hi=1.2, force=(1e-5, 0.0, 0.0),
                 wall_faces=WALLS["y"], bhll=True)]
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


def test_basis_batches_every_tile_shape_match_oracle(R):
    """Batches under the BHLL and the central-Hermite collision, in every tile
    shape the autotuner chooses from (512-node tiles, which the basis kernels
    walk in two passes, and persistent grids included) and in the autotuned
    one, against the oracle."""
    for extra, lat, dims in ((dict(bhll=True), "Q9", [(37, 23, 1), (19, 31, 1), (64, 9, 1)]),
                             (dict(central=True, hermite=True), "Q27", [(11, 9, 7), (13, 6, 9)])):
        prms = [dict(lattice=lat, n=n, dx=(1.0, 0.5, 1.0) if lat == "Q9" else (1.0, 0.5, 2.0), nu=0.04,
                     s_hi=1.3, force=(1e-5, 0.0, 0.0), wall_faces=WALLS["y"], **extra) for n in dims]
        fields, refs = [], []
        for k, p in enumerate(prms):
            m = O.Model(p)
            rho, u = random_fields(m, 50 + k)
            fields.append((rho, u))
            refs.append(m.step(m.init(rho, u), 10))
        b = R.Batch([R.make_params(**p, storage="f64", pattern="AA") for p in prms])
        best = b.autotune(steps=2)
        for cfg in list(range(len(R.Batch.configs()))) + [best]:
            b.set_config(cfg)
            for k, (rho, u) in enumerate(fields):
                b.domains[k].set_fields(rho, u)
            b.step(10)
            err = max(rel_err(b.domains[k].populations().cpu().numpy(), refs[k]) for k in range(len(prms)))
            say(f"[bhll] {lat} {extra} config {R.Batch.configs()[cfg]}{' (autotuned)' if cfg == best else ''}: "
                f"{err:.2e}")
            assert err < 1e-12, (lat, cfg)
        b.close()


def test_bhll_refused_where_not_built(R):
    with pytest.raises(R.RMRTError) as e:
        R.derive(R.make_params(lattice="Q27", n=(4, 4, 4), nu=0.05, bhll=True))
    assert e.value.code == R.EUNSUPPORTED
    with pytest.raises(R.RMRTError) as e:
        R.derive(R.make_params(lattice="Q9", equation="NCDE", n=(4, 4, 1), D0=0.05, bhll=True))
    assert e.value.code == R.EINVAL
    for other in (dict(hermite=True), dict(central=True)):
        with pytest.raises(R.RMRTError) as e:
            R.derive(R.make_params(lattice="Q9", n=(4, 4, 1), nu=0.05, bhll=True, **other))
        assert e.value.code == R.EINVAL
    prm = dict(CASES["periodic"][0], bhll=True)
    m = O.Model(prm)
    rho, u = random_fields(m, 1)
    dom = R.Domain(R.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    with pytest.raises(R.RMRTError) as e:
        dom.local_gradients(R.GRAD_STRAIN)
    assert e.value.code == R.EUNSUPPORTED
    dom.close()
    with pytest.raises(R.RMRTError) as e:
        R.Batch([R.make_params(**CASES["periodic"][0], storage="f64", pattern="AA"),
                 R.make_params(**prm, storage="f64", pattern="AA")])
    assert e.value.code == R.EINVAL
