"""Multi-step parity at the benchmark configurations' full sizes, in the launch
configuration the benchmark times (default launch shapes, graph-replayed
steps; the autotuned tile configuration for the 64-channel batch), against the
FP64 oracle evolving each sampled node's light cone (tests/gpu_util.py):
after k steps a node depends only on the initial state within k nodes per
axis, so the oracle steps a (2k+1)-wide sub-box around it.

  rD3Q19 Taylor-Green 256 x 256 x 128 (dz = 2 dx), 16 steps, FP64 / FP32 / FP16
  rD2Q9 NCDE Gaussian hill 2048 x 1024 (dy = dx / 2), nonlinear D, 128 steps,
      FP64 / FP32
  rD3Q27 batch of 64 force-driven walled channels (32..256 nodes per axis), 16
      steps, on its 4 smallest domains and its largest, FP32 (autotuned) / FP64
  the benchmark's basis-collision sizes: rD3Q27 central-Hermite 256 x 256 x 128,
      8 steps, and rD2Q9 BHLL 4096 x 2048 (dy = dx / 2), 16 steps, FP64 / FP32

The initial fields carry seeded noise so that every sampled node sees a
non-trivial state.  Samples include domain corners (periodic wrap, wall
corners) and seeded interior nodes.  Bars: FP64 populations within 1e-12 of
max |f|; FP32 rho within 1e-5 of rho0 and u within 1e-5 of the reference
velocity (phi within 1e-5 of its peak); FP16 within 3e-3.

Also: the 2048 x 1024 hill through all 5000 of its steps in FP32 deviation
storage against the same run in FP64 storage (whose multi-step parity with the
oracle is checked above at 1e-12), phi within 1e-5 of the peak."""
import sys

import numpy as np
import pytest

from gpu_util import lightcone_oracle
from inputs import channel_batch, gaussian_hill_field, taylor_green_3d
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


def _lin(n, node):
    return node[0] + n[0] * (node[1] + n[1] * node[2])


def _gpu_samples(dom, n, nodes):
    f = dom.populations()
    idx = torch.tensor([_lin(n, p) for p in nodes], device=f.device)
    return f[:, idx].cpu().numpy().T        # (samples, q)


def _macro(m, f):
    """rho (or phi) and u of the populations f (samples, q)."""
    r, u = m.macroscopic(np.asarray(f).T)
    return r, u


# --------------------------------------------------------------------------
# rD3Q19 Taylor-Green 256 x 256 x 128
# --------------------------------------------------------------------------
TG = dict(lattice="Q19", n=(256, 256, 128), dx=(1.0, 1.0, 2.0), nu=0.005, cs2=1.0 / 3.0, rho0=1.0)
TG_K = 16


@pytest.fixture(scope="module")
def tg_case():
    rho, u, _ = taylor_green_3d(TG["n"], TG["dx"], 0.02, TG["cs2"])
    rng = np.random.default_rng(31)
    rho = rho + rng.uniform(-1e-4, 1e-4, rho.shape)
    u = u + rng.uniform(-2e-3, 2e-3, u.shape)
    n = TG["n"]
    nodes = [(0, 0, 0), (255, 255, 127), (0, 255, 64), (128, 0, 127)]
    nodes += [tuple(int(rng.integers(0, s)) for s in n) for _ in range(4)]
    ref = np.stack([lightcone_oracle(TG, rho, u, p, TG_K)[0] for p in nodes])
    return rho, u, nodes, ref


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32dev", 1e-5), ("f16dev", 3e-3)])
def test_q19_taylor_green_full_size_16_steps(R, tg_case, storage, tol):
    rho, u, nodes, ref = tg_case
    say(f"[full-size multistep] rD3Q19 256x256x128 {storage}, {TG_K} steps, {len(nodes)} light cones")
    dom = R.Domain(R.make_params(**TG, storage=storage, pattern="AA"), rho, u)
    dom.step(TG_K)
    got = _gpu_samples(dom, TG["n"], nodes)
    dom.close()
    del dom
    torch.cuda.empty_cache()
    m = O.Model(dict(TG, n=(1, 1, 1)))
    ef = np.abs(got - ref).max() / np.abs(ref).max()
    r_g, u_g = _macro(m, got)
    r_o, u_o = _macro(m, ref)
    er, eu = np.abs(r_g - r_o).max() / 1.0, np.abs(u_g - u_o).max() / 0.02
    say(f"   max|df|/max|f| {ef:.2e}, max|drho|/rho0 {er:.2e}, max|du|/U0 {eu:.2e}")
    if storage == "f64":
        assert ef <= tol
    else:
        assert er <= tol and eu <= tol


# --------------------------------------------------------------------------
# rD2Q9 NCDE Gaussian hill 2048 x 1024
# --------------------------------------------------------------------------
HILL = dict(lattice="Q9", equation="NCDE", n=(2048, 1024, 1), dx=(1.0, 0.5, 1.0), D0=0.01, D2=1.0,
            adv=(0.05, 0.02, 0.0), rho0=0.0)
HILL_K = 128


def _hill_phi(noise=True):
    phi = gaussian_hill_field(2048, 1024, 1.0, 0.5, 40.0, 1024.0, 256.0)
    if noise:
        phi = phi + np.random.default_rng(32).uniform(0.0, 0.01, phi.shape)
    return phi


@pytest.fixture(scope="module")
def hill_case():
    phi = _hill_phi()
    nodes = [(1024, 512, 0), (1060, 470, 0), (990, 560, 0), (0, 1023, 0)]
    ref = np.stack([lightcone_oracle(HILL, phi, None, p, HILL_K)[0] for p in nodes])
    return phi, nodes, ref


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_q9_ncde_hill_full_size_128_steps(R, hill_case, storage):
    phi, nodes, ref = hill_case
    say(f"[full-size multistep] rD2Q9 NCDE 2048x1024 {storage}, {HILL_K} steps, {len(nodes)} light cones")
    dom = R.Domain(R.make_params(**HILL, storage=storage, pattern="AA"), phi)
    dom.step(HILL_K)
    got = _gpu_samples(dom, HILL["n"], nodes)
    dom.close()
    m = O.Model(dict(HILL, n=(1, 1, 1)))
    ef = np.abs(got - ref).max() / np.abs(ref).max()
    ep = np.abs(_macro(m, got)[0] - _macro(m, ref)[0]).max() / 1.01
    say(f"   max|df|/max|f| {ef:.2e}, max|dphi|/peak {ep:.2e}")
    if storage == "f64":
        assert ef <= 1e-12
    else:
        assert ep <= 1e-5


def test_q9_ncde_hill_5000_steps_f32_against_f64(R):
    """The configuration's full run: FP32 deviation storage against FP64
    storage, both on the GPU, through all 5000 steps."""
    phi = _hill_phi(noise=False)
    out = {}
    for storage in ("f64", "f32dev"):
        dom = R.Domain(R.make_params(**HILL, storage=storage, pattern="AA"), phi)
        dom.step(5000)
        p, _ = dom.moments()
        out[storage] = p.cpu().numpy()
        dom.close()
    err = np.abs(out["f32dev"] - out["f64"]).max() / 1.0
    mass = abs(out["f32dev"].sum() - out["f64"].sum()) / out["f64"].sum()
    say(f"[full-size multistep] rD2Q9 NCDE 2048x1024, 5000 steps: max|phi32 - phi64| / peak {err:.2e}, "
        f"relative mass difference {mass:.2e}, peak now {out['f64'].max():.4f}")
    assert err <= 1e-5
    assert np.isfinite(out["f32dev"]).all()


# --------------------------------------------------------------------------
# rD3Q27 batch of 64 walled, force-driven channels
# --------------------------------------------------------------------------
WALLS_YZ = O.WALL_YM | O.WALL_YP | O.WALL_ZM | O.WALL_ZP
BATCH_K = 16


def _channel_params(d):
    return dict(lattice="Q27", n=d["n"], dx=d["dx"], nu=d["nu"], nu_b=d["nu_b"], force=d["force"],
                wall_faces=WALLS_YZ, rho0=1.0)


@pytest.fixture(scope="module")
def batch_case():
    doms = channel_batch(seed=4, nd=64, nmin=32, nmax=256)
    sizes = [int(np.prod(d["n"])) for d in doms]
    order = np.argsort(sizes)
    picked = [int(i) for i in order[:4]] + [int(order[-1])]
    rng = np.random.default_rng(33)
    cases = {}
    for k in picked:
        prm = _channel_params(doms[k])
        n = prm["n"]
        N = int(np.prod(n))
        rho = 1.0 + rng.uniform(-1e-3, 1e-3, N)
        u = rng.uniform(-0.01, 0.01, (3, N))
        nodes = [(0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (n[0] // 2, 0, n[2] - 1),
                 tuple(int(rng.integers(0, s)) for s in n)]
        ref = np.stack([lightcone_oracle(prm, rho, u, p, BATCH_K)[0] for p in nodes])
        cases[k] = (prm, rho, u, nodes, ref)
    return doms, cases


@pytest.mark.parametrize("storage", ["f32dev", "f64"])
def test_q27_64_channel_batch_full_size_16_steps(R, batch_case, storage):
    doms, cases = batch_case
    say(f"[full-size multistep] rD3Q27 64-channel batch {storage}, domains {sorted(cases)}, {BATCH_K} steps")
    params = [R.make_params(**_channel_params(d), storage=storage, pattern="AA") for d in doms]
    b = R.Batch(params)
    if storage == "f32dev":
        cfg = b.autotune(steps=2)
        say(f"   autotuned config {R.Batch.configs()[cfg]}, groups {b.group_bytes()}")
    for k, (prm, rho, u, nodes, ref) in cases.items():
        b.domains[k].set_fields(rho, u)
    b.step(BATCH_K)
    worst = {}
    for k, (prm, rho, u, nodes, ref) in cases.items():
        got = _gpu_samples(b.domains[k], prm["n"], nodes)
        m = O.Model(dict(prm, n=(1, 1, 1)))
        ef = np.abs(got - ref).max() / np.abs(ref).max()
        r_g, u_g = _macro(m, got)
        r_o, u_o = _macro(m, ref)
        er, eu = np.abs(r_g - r_o).max(), np.abs(u_g - u_o).max() / 0.01
        worst[k] = (ef, er, eu)
        say(f"   domain {k} {prm['n']}: max|df|/max|f| {ef:.2e}, max|drho|/rho0 {er:.2e}, max|du|/U {eu:.2e}")
    b.close()
    del b
    torch.cuda.empty_cache()
    for k, (ef, er, eu) in worst.items():
        if storage == "f64":
            assert ef <= 1e-12, k
        else:
            assert er <= 1e-5 and eu <= 1e-5, k


# --------------------------------------------------------------------------
# The alternative moment bases at the sizes of the benchmark's basis leg
# --------------------------------------------------------------------------
BASIS_CASES = {
    "q27_central_hermite": (dict(lattice="Q27", n=(256, 256, 128), dx=(1.0, 1.0, 2.0), nu=0.005, cs2=1.0 / 3.0,
                                 rho0=1.0, central=True, hermite=True), 8),
    "q9_bhll": (dict(lattice="Q9", n=(4096, 2048, 1), dx=(1.0, 0.5, 1.0), nu=0.01, nu_b=0.03, s_hi=1.2,
                     rho0=1.0, bhll=True), 16),
}


def _basis_fields(prm, seed):
    rng = np.random.default_rng(seed)
    if prm["lattice"] == "Q27":
        rho, u, _ = taylor_green_3d(prm["n"], prm["dx"], 0.02, prm["cs2"])
    else:
        from inputs import taylor_green_2d
        nx, ny = prm["n"][:2]
        rho, u, _ = taylor_green_2d(nx, ny, prm["dx"][0], prm["dx"][1], 0.02, 0.25 / 3.0)
    return rho + rng.uniform(-1e-4, 1e-4, rho.shape), u + rng.uniform(-2e-3, 2e-3, u.shape)


@pytest.fixture(scope="module")
def basis_cases():
    out = {}
    for name, (prm, k) in BASIS_CASES.items():
        rho, u = _basis_fields(prm, 41)
        n = prm["n"]
        rng = np.random.default_rng(42)
        nodes = [(0, 0, 0), tuple(s - 1 for s in n)]
        nodes += [tuple(int(rng.integers(0, s)) for s in n) for _ in range(2)]
        ref = np.stack([lightcone_oracle(prm, rho, u, p, k)[0] for p in nodes])
        out[name] = (rho, u, nodes, ref)
    return out


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", list(BASIS_CASES))
def test_basis_collision_full_size(R, basis_cases, name, storage):
    prm, k = BASIS_CASES[name]
    rho, u, nodes, ref = basis_cases[name]
    say(f"[full-size multistep] {name} {prm['n']} {storage}, {k} steps, {len(nodes)} light cones")
    dom = R.Domain(R.make_params(**prm, storage=storage, pattern="AA"), rho, u)
    dom.step(k)
    got = _gpu_samples(dom, prm["n"], nodes)
    dom.close()
    del dom
    torch.cuda.empty_cache()
    m = O.Model(dict(prm, n=(1, 1, 1)))
    ef = np.abs(got - ref).max() / np.abs(ref).max()
    r_g, u_g = _macro(m, got)
    r_o, u_o = _macro(m, ref)
    er, eu = np.abs(r_g - r_o).max(), np.abs(u_g - u_o).max() / 0.02
    say(f"   max|df|/max|f| {ef:.2e}, max|drho|/rho0 {er:.2e}, max|du|/U0 {eu:.2e}")
    if storage == "f64":
        assert ef <= 1e-12
    else:
        assert er <= 1e-5 and eu <= 1e-5
