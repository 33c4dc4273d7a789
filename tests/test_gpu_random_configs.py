"""Seeded sweep of random parameter sets through the C ABI against the FP64
oracle: lattice (rD2Q9 / rD3Q19 / rD3Q27), equation (NSE / NCDE), ragged grid
sizes, grid spacings, c_s^2, viscosities, higher-order rate, wall pairs, random
solid nodes, body force and mass source, He-Luo equilibrium, viscosity tensors,
the central, Hermite, central-Hermite and BHLL moment bases, the NCDE
variants, AA or AB pattern, odd and even step counts.  FP64 storage:
every fluid population within 1e-12 of max |f|.  Draws that the library rejects
as invalid (rmrt_derive) are redrawn."""
import sys

import numpy as np
import pytest

from gpu_util import WALLS, random_fields, rel_err
from oracle import rmrt_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

NCASES = 48


@pytest.fixture(scope="module")
def rmrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_00366_amd import rmrt as R
    return R


def _draw(rng):
    lat = str(rng.choice(["Q9", "Q19", "Q27"]))
    d = 2 if lat == "Q9" else 3
    nse = rng.random() < 0.7
    n = [int(rng.integers(3, 14)) for _ in range(d)] + ([1] if d == 2 else [])
    dx = [1.0] + [float(rng.choice([0.5, 1.0, 2.0])) for _ in range(d - 1)] + ([1.0] if d == 2 else [])
    prm = dict(lattice=lat, equation="NSE" if nse else "NCDE", n=tuple(n), dx=tuple(dx))
    if rng.random() < 0.3:
        prm["cs2"] = float(rng.uniform(0.15, 0.33)) * min(v * v for v in dx[:d])
    if rng.random() < 0.4:
        prm["s_hi"] = float(rng.uniform(0.8, 1.7))
    axes = [a for a in range(d) if rng.random() < 0.35]
    prm["wall_faces"] = sum((3 << (2 * a)) for a in axes)
    if nse:
        prm["nu"] = float(rng.uniform(0.01, 0.1))
        if rng.random() < 0.5:
            prm["nu_b"] = float(rng.uniform(0.01, 0.2))
        if rng.random() < 0.5:
            prm["force"] = tuple(float(v) for v in rng.uniform(-2e-5, 2e-5, 3) * ([1, 1, 1] if d == 3 else [1, 1, 0]))
        if rng.random() < 0.25:
            prm["source"] = float(rng.choice([-1.0, 1.0]) * 1e-6)
        if rng.random() < 0.2:
            prm["incompressible"] = True
        if rng.random() < 0.2:
            prm["nu_tensor"] = tuple(float(v) for v in rng.uniform(0.01, 0.1, 6))
        # the alternative moment bases (combinations a lattice lacks are redrawn)
        basis = rng.random()
        if basis < 0.1:
            prm["central"] = True
        elif basis < 0.2:
            prm["hermite"] = True
        elif basis < 0.25:
            prm["central"] = prm["hermite"] = True
        elif basis < 0.3:
            prm["bhll"] = True
    else:
        prm["D0"] = float(rng.uniform(0.01, 0.1))
        prm["D2"] = float(rng.choice([0.0, rng.uniform(0.0, 1.0)]))
        prm["adv"] = tuple(float(v) for v in rng.uniform(-0.05, 0.05, 3) * ([1, 1, 1] if d == 3 else [1, 1, 0]))
        prm["rho0"] = 0.0
        if rng.random() < 0.4:
            prm["source"] = float(rng.uniform(-1e-3, 1e-3))
        variant = rng.random()
        if variant < 0.2:
            prm["gamma0"] = True
        elif variant < 0.35:
            prm["diffusive"] = True
    N = int(np.prod(n))
    solid = (rng.random(N) < 0.08) if rng.random() < 0.3 else None
    pattern = str(rng.choice(["AA", "AB"]))
    steps = int(rng.integers(5, 16))
    return prm, solid, pattern, steps


def _valid(R, prm):
    try:
        R.derive(R.make_params(**prm))
        return True
    except R.RMRTError:
        return False


@pytest.mark.parametrize("k", range(NCASES))
def test_random_configuration_matches_oracle(rmrt, k):
    rng = np.random.default_rng(1000 + k)
    while True:
        prm, solid, pattern, steps = _draw(rng)
        if _valid(rmrt, prm):
            break
    print(f"[random {k}] {prm} solid={solid is not None} {pattern} {steps} steps", flush=True)
    sys.stdout.flush()
    m = O.Model(prm, solid=solid)
    rho, u = random_fields(m, seed=k, du=0.02 if m.nse else 0.0)
    if not m.nse:
        u = None
    f_or = m.step(m.init(rho, u), steps)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern=pattern), rho, u,
                      solid=None if solid is None else solid.astype(np.uint8))
    dom.step(steps)
    g = dom.populations().cpu().numpy()
    dom.close()
    fl = m.fluid
    err = rel_err(g[:, fl], f_or[:, fl])
    print(f"   max rel |f - f_oracle| = {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("k", range(0, NCASES, 2))
def test_random_configuration_fp32_storage(rmrt, k):
    """The same draws in FP32 deviation storage: rho (or phi) within 1e-5 of rho0
    (of the peak phi) and u within 1e-5 of its maximum, at every fluid node."""
    rng = np.random.default_rng(1000 + k)
    while True:
        prm, solid, pattern, steps = _draw(rng)
        if _valid(rmrt, prm):
            break
    print(f"[random fp32 {k}] {prm['lattice']} {prm['equation']} {pattern} {steps} steps", flush=True)
    m = O.Model(prm, solid=solid)
    rho, u = random_fields(m, seed=k, du=0.02 if m.nse else 0.0)
    if not m.nse:
        u = None
    f_or = m.step(m.init(rho, u), steps)
    r_o, u_o = m.macroscopic(f_or)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f32dev", pattern=pattern), rho, u,
                      solid=None if solid is None else solid.astype(np.uint8))
    dom.step(steps)
    r_g, u_g = dom.moments()
    dom.close()
    fl = m.fluid
    scale = m.rho0 if m.nse else np.abs(r_o[fl]).max()
    err_r = np.abs(r_g.cpu().numpy()[fl] - r_o[fl]).max() / scale
    print(f"   rho/phi err {err_r:.2e}", flush=True)
    assert err_r < 1e-5
    if m.nse:
        err_u = rel_err(u_g.cpu().numpy()[:, fl], u_o[:, fl])
        print(f"   u err {err_u:.2e}", flush=True)
        assert err_u < 1e-5


def _draw_batch(rng):
    """3..7 random domains sharing lattice, equation, moment basis and pattern
    (what a batch requires); everything else per domain."""
    lat = str(rng.choice(["Q9", "Q19", "Q27"]))
    nse = rng.random() < 0.75
    pattern = str(rng.choice(["AA", "AB"]))
    doms = []
    basis = None
    while len(doms) < int(rng.integers(3, 8)):
        prm, solid, _, _ = _draw(rng)
        if prm["lattice"] != lat or (prm["equation"] == "NSE") != nse:
            continue
        b = tuple(bool(prm.get(k)) for k in ("central", "hermite", "bhll"))
        if basis is not None and b != basis:
            continue
        basis = b
        doms.append((prm, solid))
    return doms, pattern


@pytest.mark.parametrize("k", range(12))
def test_random_batch_matches_oracle(rmrt, k):
    """Random batches in FP64: every domain within 1e-12 of the oracle after an odd
    number of steps split over a graph chunk and a single step, in a random tile
    shape, with or without domain groups."""
    rng = np.random.default_rng(5000 + k)
    while True:
        doms, pattern = _draw_batch(rng)
        if all(_valid(rmrt, p) for p, _ in doms):
            break
    shape = int(rng.integers(0, len(rmrt.Batch.configs())))
    groups = int(rng.choice([0, 1, 20000]))
    print(f"[random batch {k}] {len(doms)} x {doms[0][0]['lattice']} {doms[0][0]['equation']} {pattern} "
          f"tile shape {shape} group bytes {groups}", flush=True)
    models, fields, refs = [], [], []
    for j, (prm, solid) in enumerate(doms):
        m = O.Model(prm, solid=solid)
        rho, u = random_fields(m, seed=100 * k + j, du=0.02 if m.nse else 0.0)
        if not m.nse:
            u = None
        models.append(m)
        fields.append((rho, u))
        refs.append(m.step(m.init(rho, u), 13))
    b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern=pattern) for p, _ in doms],
                   solids=[None if s is None else s.astype(np.uint8) for _, s in doms])
    b.set_config(shape)
    b.set_group_bytes(groups)
    for d, (rho, u) in zip(b.domains, fields):
        d.set_fields(rho, u)
    b.step(12)
    b.step(1)
    for j, (d, m, f_or) in enumerate(zip(b.domains, models, refs)):
        g = d.populations().cpu().numpy()
        err = rel_err(g[:, m.fluid], f_or[:, m.fluid])
        assert err < 1e-12, (j, err)
    b.close()


def _draw_reduced(rng):
    lat = str(rng.choice(["Q5", "Q7"]))
    d = 2 if lat == "Q5" else 3
    n = [int(rng.integers(3, 16)) for _ in range(d)] + ([1] if d == 2 else [])
    dx = [1.0] + [float(rng.choice([0.5, 1.0, 2.0])) for _ in range(d - 1)] + ([1.0] if d == 2 else [])
    prm = dict(lattice=lat, equation="NCDE", n=tuple(n), dx=tuple(dx), rho0=0.0,
               D0=float(rng.uniform(0.01, 0.1)), D2=float(rng.choice([0.0, rng.uniform(0.0, 1.0)])),
               adv=tuple(float(v) for v in rng.uniform(-0.05, 0.05, 3) * ([1, 1, 1] if d == 3 else [1, 1, 0])))
    if rng.random() < 0.3:
        prm["cs2"] = float(rng.uniform(0.15, 0.33)) * min(v * v for v in dx[:d])
    if rng.random() < 0.3:
        prm["s_hi"] = float(rng.uniform(0.8, 1.7))
    if rng.random() < 0.5:
        prm["source"] = float(rng.uniform(-1e-3, 1e-3))
    variant = rng.random()
    if variant < 0.2:
        prm["gamma0"] = True
    elif variant < 0.35:
        prm["diffusive"] = True
    prm["wall_faces"] = sum((3 << (2 * a)) for a in range(d) if rng.random() < 0.35)
    N = int(np.prod(n))
    solid = (rng.random(N) < 0.08) if rng.random() < 0.3 else None
    return prm, solid, str(rng.choice(["AA", "AB"])), int(rng.integers(5, 16))


@pytest.mark.parametrize("k", range(16))
def test_random_reduced_lattice_matches_oracle(rmrt, k):
    """Random rD2Q5 / rD3Q7 NCDE parameter sets (with the previous-step phi that
    the library keeps): FP64 populations within 1e-12 of max |f|."""
    rng = np.random.default_rng(7000 + k)
    while True:
        prm, solid, pattern, steps = _draw_reduced(rng)
        if _valid(rmrt, prm):
            break
    print(f"[random reduced {k}] {prm} solid={solid is not None} {pattern} {steps} steps", flush=True)
    m = O.Model(prm, solid=solid)
    phi, _ = random_fields(m, seed=k, du=0.0)
    f_or, _ = m.step(m.init(phi, None), steps, m.init_history(phi))
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern=pattern), phi, None,
                      solid=None if solid is None else solid.astype(np.uint8))
    dom.step(steps)
    g = dom.populations().cpu().numpy()
    dom.close()
    err = rel_err(g[:, m.fluid], f_or[:, m.fluid])
    print(f"   max rel |f - f_oracle| = {err:.2e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("k", range(0, NCASES, 3))
def test_random_configuration_local_outputs(rmrt, k):
    """Local outputs (strain rate and stress for the NSE, grad phi for the NCDE) of
    the random draws after their steps, FP64 storage, against the oracle's formulas
    on its own state: within 1e-11 of the output's magnitude; zero at solid nodes.
    Local outputs belong to the raw-moment collision: the basis draws are dropped."""
    rng = np.random.default_rng(1000 + k)
    while True:
        prm, solid, pattern, steps = _draw(rng)
        for key in ("central", "hermite", "bhll"):
            prm.pop(key, None)
        if _valid(rmrt, prm):
            break
    print(f"[random local {k}] {prm['lattice']} {prm['equation']} {pattern} {steps} steps", flush=True)
    m = O.Model(prm, solid=solid)
    rho, u = random_fields(m, seed=k, du=0.02 if m.nse else 0.0)
    if not m.nse:
        u = None
    f_or = m.step(m.init(rho, u), steps)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern=pattern), rho, u,
                      solid=None if solid is None else solid.astype(np.uint8))
    dom.step(steps)
    fl = m.fluid
    if m.nse:
        tau, E = m.local_gradients(f_or[:, fl])
        pairs = [(a, a) for a in range(m.d)] + [(a, b) for a in range(m.d) for b in range(a + 1, m.d)]
        refs = {rmrt.GRAD_STRAIN: np.stack([E[a, b] for a, b in pairs]),
                rmrt.GRAD_STRESS: np.stack([tau[a, b] for a, b in pairs])}
    else:
        refs = {rmrt.GRAD_PHI: m.local_gradients(f_or[:, fl])}
    for kind, ref in refs.items():
        got = dom.local_gradients(kind).cpu().numpy()
        err = np.abs(got[:, fl] - ref).max() / np.abs(ref).max()
        print(f"   kind {kind}: max rel err {err:.2e}", flush=True)
        assert err < 1e-11
        assert np.all(got[:, ~fl] == 0.0)
    dom.close()


@pytest.mark.parametrize("k", range(1, NCASES, 3))
def test_random_configuration_fp16_storage(rmrt, k):
    """The draws in FP16 deviation storage (held to the loose bound of the other
    FP16 parity cases, 3e-3 in rho or phi and u).  FP16 storage needs every weight
    positive; draws the library refuses for it are redrawn."""
    rng = np.random.default_rng(1000 + k)
    while True:
        prm, solid, pattern, steps = _draw(rng)
        if not _valid(rmrt, prm):
            continue
        m = O.Model(prm, solid=solid)
        rho, u = random_fields(m, seed=k, du=0.02 if m.nse else 0.0)
        if not m.nse:
            u = None
        try:
            dom = rmrt.Domain(rmrt.make_params(**prm, storage="f16dev", pattern=pattern), rho, u,
                              solid=None if solid is None else solid.astype(np.uint8))
            break
        except rmrt.RMRTError:
            continue
    print(f"[random fp16 {k}] {prm['lattice']} {prm['equation']} {pattern} {steps} steps", flush=True)
    f_or = m.step(m.init(rho, u), steps)
    r_o, u_o = m.macroscopic(f_or)
    dom.step(steps)
    r_g, u_g = dom.moments()
    dom.close()
    fl = m.fluid
    scale = m.rho0 if m.nse else np.abs(r_o[fl]).max()
    err_r = np.abs(r_g.cpu().numpy()[fl] - r_o[fl]).max() / scale
    err_u = rel_err(u_g.cpu().numpy()[:, fl], u_o[:, fl]) if m.nse else 0.0
    print(f"   rho/phi err {err_r:.2e}, u err {err_u:.2e}", flush=True)
    assert err_r < 3e-3 and err_u < 3e-3
