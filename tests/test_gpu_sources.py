"""GPU parity of the source and force fields (rmrt_set_source_fields; eq. NSE
and eq. NCDE with S, Sbar, Fbar varying by node and step), of the gamma = 0
explicit difference of dF/dt with the library-held previous-step source
(eq. 2-1), and of the C = 0 NCDE form of eq. 4-16 on rD2Q9 / rD3Q19 / rD3Q27
(c_zero), also under the central, Hermite, central-Hermite and BHLL
collisions, against the FP64 oracle.  Bars: FP64 populations within 1e-12 of
max |f|; FP32 rho within 1e-5 of rho0, u within 1e-5 of its scale, phi within
1e-5 of its peak."""
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
    "q9_channel_fields": dict(lattice="Q9", n=(37, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.07,
                              wall_faces=WALLS["y"]),
    "q19_periodic_fields": dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03),
    "q27_walls_fields": dict(lattice="Q27", n=(11, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05, wall_faces=WALLS["yz"]),
    "q9_heluo_fields": dict(lattice="Q9", n=(29, 17, 1), dx=(1.0, 0.5, 1.0), nu=0.04, incompressible=True,
                            rho0=1.05, wall_faces=WALLS["y"]),
    "q27_central_fields": dict(lattice="Q27", n=(11, 9, 8), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.02, s_hi=1.3,
                               central=True, wall_faces=WALLS["z"]),
    "q19_hermite_fields": dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03, s_hi=1.4, hermite=True),
    "q9_central_hermite_fields": dict(lattice="Q9", n=(37, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.07,
                                      s_hi=1.2, central=True, hermite=True, wall_faces=WALLS["y"]),
    "q9_bhll_fields": dict(lattice="Q9", n=(37, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.07, s_hi=1.2,
                           bhll=True, wall_faces=WALLS["y"]),
    "q9_ncde_fields": dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0,
                           adv=(0.05, 0.02, 0.0), rho0=0.0),
    "q9_ncde_gamma0_fields": dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01,
                                  D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0, gamma0=True),
    "q19_ncde_fields": dict(lattice="Q19", equation="NCDE", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), D0=0.02, D2=0.5,
                            adv=(0.03, -0.01, 0.02), rho0=0.0),
    "q5_fields": dict(lattice="Q5", equation="NCDE", n=(31, 19, 1), dx=(1.0, 0.5, 1.0), D0=0.02, D2=0.5,
                      adv=(0.04, -0.02, 0.0), rho0=0.0),
    "q7_gamma0_fields": dict(lattice="Q7", equation="NCDE", n=(11, 9, 7), dx=(1.0, 1.0, 2.0), D0=0.02, D2=0.5,
                             adv=(0.03, 0.01, -0.02), rho0=0.0, gamma0=True),
    "q9_czero": dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0,
                     adv=(0.05, 0.02, 0.0), rho0=0.0, c_zero=True, source=1e-3),
    "q19_czero_fields": dict(lattice="Q19", equation="NCDE", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), D0=0.02, D2=0.5,
                             adv=(0.03, -0.01, 0.02), rho0=0.0, c_zero=True),
    "q27_czero_solid": dict(lattice="Q27", equation="NCDE", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), D0=0.02, D2=0.3,
                            adv=(0.02, 0.01, -0.01), rho0=0.0, c_zero=True, wall_faces=WALLS["z"]),
}
FIELDS = {k for k in CASES if "fields" in k}
STEPS = 12


def _fields(m, seed, dtype):
    """Seeded source / force fields (values representable in the storage's field type)."""
    rng = np.random.default_rng(seed)
    S = 1e-4 * rng.uniform(-1, 1, m.N)
    F = 2e-5 * rng.uniform(-1, 1, (m.d, m.N)) if m.nse else None
    cast = (lambda a: a) if dtype == "f64" else (lambda a: a.astype(np.float32).astype(np.float64))
    return cast(S), None if F is None else cast(F)


def _run(R, case, storage, pattern, time_varying=False):
    prm = CASES[case]
    solid = circle_mask(prm["n"], (5, 4), 2) if "solid" in case else None
    m = O.Model(prm, solid=solid)
    seed = sum(map(ord, case)) % 997
    rho, u = random_fields(m, seed, du=0.02 if m.nse else 0.0)
    uu = u if m.nse else None
    dom = R.Domain(R.make_params(**prm, storage=storage, pattern=pattern), rho, uu,
                   solid=None if solid is None else solid.astype(np.uint8))
    dt = dom.source_dtype()
    S = F = None
    if case in FIELDS:
        S, F = _fields(m, seed + 1, storage)
        m.set_sources(S, F)
        S_dev = torch.tensor(S, dtype=dt, device="cuda")
        F_dev = None if F is None else torch.tensor(F, dtype=dt, device="cuda")
        dom.set_source_fields(S_dev, F_dev)
        dom.set_fields(rho, uu)                       # the initial state takes the fields
    f = m.init(rho, uu)
    hist = m.init_history(rho) if m.hist_form else None
    if time_varying:
        rng = np.random.default_rng(seed + 2)
        for k in range(STEPS):
            f = m.step(f, 1) if hist is None else m.step(f, 1, hist)
            if hist is not None:
                f, hist = f
            dom.step(1)
            # new values for the next step, written in place on the GPU
            S2 = S * np.cos(0.3 * (k + 1)) + 2e-5 * rng.uniform(-1, 1, m.N)
            F2 = None if F is None else F * np.sin(0.2 * (k + 2))
            if storage != "f64":
                S2 = S2.astype(np.float32).astype(np.float64)
                F2 = None if F2 is None else F2.astype(np.float32).astype(np.float64)
            m.update_sources(S2, F2)
            dom._src[0].copy_(torch.tensor(S2, dtype=dt, device="cuda"))
            if F2 is not None:
                dom._src[1].copy_(torch.tensor(F2, dtype=dt, device="cuda"))
    else:
        if hist is None:
            f = m.step(f, STEPS)
        else:
            f, hist = m.step(f, STEPS, hist)
        dom.step(STEPS)
    return m, dom, f


def _check(m, dom, f, storage, label):
    fg = dom.populations().cpu().numpy()
    fl = m.fluid
    r_g, u_g = dom.moments()
    r_g, u_g = r_g.cpu().numpy(), u_g.cpu().numpy()
    r_o, u_o = m.macroscopic(f)
    if storage == "f64":
        err = rel_err(fg[:, fl], f[:, fl])
        say(f"[sources] {label}: max|f - f_oracle| / max|f| {err:.2e}")
        assert err < 1e-12
        assert np.abs(r_g[fl] - r_o[fl]).max() < 1e-12 * max(1.0, np.abs(r_o).max())
    else:
        if m.nse:
            er = np.abs(r_g[fl] - r_o[fl]).max() / m.rho0
            eu = np.abs(u_g[:, fl] - u_o[:, fl]).max() / max(np.abs(u_o).max(), 1e-3)
            say(f"[sources] {label}: rho {er:.2e}, u {eu:.2e}")
            assert er < 1e-5 and eu < 1e-5
        else:
            ep = np.abs(r_g[fl] - r_o[fl]).max() / np.abs(r_o).max()
            say(f"[sources] {label}: phi {ep:.2e}")
            assert ep < 1e-5


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", list(CASES))
def test_source_fields_and_c_zero_match_oracle(R, case, pattern, storage):
    m, dom, f = _run(R, case, storage, pattern)
    _check(m, dom, f, storage, f"{case} {pattern} {storage}")
    dom.close()


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("case", ["q9_channel_fields", "q27_walls_fields", "q9_ncde_fields",
                                  "q9_ncde_gamma0_fields", "q7_gamma0_fields", "q19_czero_fields",
                                  "q27_central_fields", "q9_bhll_fields"])
def test_time_varying_fields_match_oracle(R, case, storage):
    """Fields rewritten in place between single steps: each step reads the
    values of its own time, and the gamma = 0 form differences them against the
    previous step's."""
    m, dom, f = _run(R, case, storage, "AA", time_varying=True)
    _check(m, dom, f, storage, f"{case} time-varying {storage}")
    dom.close()


def test_fields_enter_reductions_and_detach(R):
    """rmrt_reduce takes the fields' half-step corrections (sum rho = sum fbar +
    dt sum Sbar / 2, sum rho u with dt sum Fbar / 2); detaching returns to the
    parameter set's constants; local outputs are refused while fields are
    attached."""
    prm = dict(CASES["q27_walls_fields"], force=(1e-5, 0.0, 0.0))
    m = O.Model(prm)
    rho, u = random_fields(m, 5)
    dom = R.Domain(R.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    S, F = _fields(m, 6, "f64")
    dom.set_source_fields(torch.tensor(S, device="cuda"), torch.tensor(F, device="cuda"))
    dom.step(3)
    red = dom.reduce()
    fg = dom.populations().cpu().numpy()
    mass = fg.sum() + 0.5 * S.sum()
    mom = (m.C.T @ fg).sum(axis=1) + 0.5 * F.sum(axis=1)
    assert abs(red[0] - mass) < 1e-12 * mass
    assert np.abs(np.array(red[1:]) - mom).max() < 1e-12
    with pytest.raises(R.RMRTError) as e:
        dom.local_gradients(R.GRAD_STRAIN)
    assert e.value.code == R.EUNSUPPORTED
    # detached: the next steps are the constant-force model's
    dom.set_source_fields(None, None)
    m.set_sources(None, None)
    f_or = m.step(fg, 4)
    dom.step(4)
    assert rel_err(dom.populations().cpu().numpy(), f_or) < 1e-12
    assert R.lib().rmrt_set_source_fields(None, None, None, None) == R.EINVAL
    dom.close()
    # a body-force field is an NSE input
    prm = CASES["q9_ncde_fields"]
    m = O.Model(prm)
    nc = R.Domain(R.make_params(**prm, storage="f64", pattern="AA"), np.ones(m.N))
    with pytest.raises(R.RMRTError) as e:
        nc.set_source_fields(None, torch.zeros((2, m.N), dtype=torch.float64, device="cuda"))
    assert e.value.code == R.EINVAL
    nc.close()
