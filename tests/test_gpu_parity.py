"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP64 storage max|f - f_oracle| / max|f_oracle| <= 1e-12 on every fluid
population; FP32 deviation storage max|rho - rho_oracle| / rho0 and
max|u - u_oracle| / U_ref <= 1e-5 (phi: relative to its peak); FP16 deviation
storage is reported and held to a loose bound only."""
import sys
import zlib

import numpy as np
import pytest

from gpu_util import WALLS, circle_mask, random_fields, rel_err
from inputs import gaussian_hill_field, grid_coords, taylor_green_2d, taylor_green_3d
from oracle import rmrt_oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmrt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_00366_amd import rmrt as R
    return R


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    # name: (oracle/GPU parameters, solid-mask builder or None, steps)
    "q9_periodic": (dict(lattice="Q9", n=(37, 23, 1), dx=(1.0, 0.5, 1.0), nu=0.02, nu_b=0.05), None, 25),
    "q9_channel_solid_force": (dict(lattice="Q9", n=(40, 21, 1), dx=(1.0, 0.5, 1.0), nu=0.05,
                                    force=(2e-5, 1e-6, 0.0), source=1e-6, wall_faces=WALLS["y"]),
                               lambda n: circle_mask(n, (12, 10), 4), 25),
    "q9_ncde_nonlinear": (dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01,
                               D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0, source=1e-3), None, 25),
    "q19_periodic": (dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.08), None, 15),
    "q19_channel_force": (dict(lattice="Q19", n=(12, 10, 8), dx=(1.0, 1.0, 2.0), nu=0.04,
                               force=(1e-5, 0.0, 2e-6), wall_faces=WALLS["yz"]), None, 15),
    "q19_ncde": (dict(lattice="Q19", equation="NCDE", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), D0=0.02, D2=0.5,
                      adv=(0.03, -0.01, 0.02), rho0=0.0), None, 15),
    "q27_periodic": (dict(lattice="Q27", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.01), None, 15),
    "q19_standard_lattice": (dict(lattice="Q19", n=(12, 10, 9), dx=(1.0, 1.0, 1.0), cs2=1.0 / 3.0, nu=0.02), None, 15),
    "q9_heluo_walls_force": (dict(lattice="Q9", n=(29, 17, 1), dx=(1.0, 0.5, 1.0), nu=0.04, nu_b=0.09,
                                  force=(2e-5, -1e-5, 0.0), source=1e-6, wall_faces=WALLS["y"], incompressible=True,
                                  rho0=1.05), None, 21),
    "q27_viscosity_tensor_heluo": (dict(lattice="Q27", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), nu=0.05, nu_b=0.1,
                                        nu_tensor=(0.03, 0.06, 0.04, 0.02, 0.07, 0.05), nu_b_axis=(0.08, 0.05, 0.12),
                                        force=(1e-5, 0.0, 3e-6), wall_faces=WALLS["z"], incompressible=True),
                                   lambda n: circle_mask(n, (5, 4), 2), 15),
    "q9_ncde_gamma0_source": (dict(lattice="Q9", equation="NCDE", n=(33, 17, 1), dx=(1.0, 0.5, 1.0), D0=0.01,
                                   D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0, source=1e-3, gamma0=True), None, 25),
    "q19_ncde_diffusive_source": (dict(lattice="Q19", equation="NCDE", n=(11, 9, 7), dx=(1.0, 0.5, 2.0), D0=0.02,
                                       D2=0.5, adv=(0.01, -0.005, 0.004), source=-1e-3, diffusive=True, rho0=0.0),
                                  None, 15),
    "q19_viscosity_tensor": (dict(lattice="Q19", n=(13, 11, 9), dx=(1.0, 2.0, 1.0), nu=0.04,
                                  nu_tensor=(0.02, 0.05, 0.03, 0.06, 0.025, 0.045), nu_b_axis=(0.1, -1.0, 0.04)),
                             None, 15),
    "q27_channel_solid_force": (dict(lattice="Q27", n=(14, 9, 8), dx=(1.0, 2.0, 1.0), nu=0.05,
                                     force=(1e-5, 0.0, 0.0), source=-1e-6, wall_faces=WALLS["yz"],
                                     w_corner=0.0008), lambda n: circle_mask(n, (6, 4), 2), 15),
}


def _build(case, R, storage="f64", pattern="AB"):
    prm, solid_fn, steps = CASES[case]
    m = O.Model(prm, solid=None if solid_fn is None else solid_fn(prm["n"]))
    rho, u = random_fields(m, seed=zlib.crc32(case.encode()) % 1000, du=0.02 if m.nse else 0.0)
    if not m.nse:
        u = None
    gp = R.make_params(**prm, storage=storage, pattern=pattern)
    solid = None if solid_fn is None else m.solid.astype(np.uint8)
    dom = R.Domain(gp, rho, u, solid=solid)
    return m, dom, rho, u, steps


_oracle_cache = {}


def _oracle_run(case, m, rho, u, steps):
    if case not in _oracle_cache:
        f = m.init(rho, u)
        _oracle_cache[case] = (f, m.step(f, steps))
    return _oracle_cache[case]


@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", list(CASES))
def test_f64_populations_match_oracle(rmrt, case, pattern):
    say(f"[parity f64] {case} {pattern}")
    m, dom, rho, u, steps = _build(case, rmrt, "f64", pattern)
    f0, f_or = _oracle_run(case, m, rho, u, steps)
    fl = m.fluid
    # the initial state first (init kernel vs oracle init)
    g0 = dom.populations().cpu().numpy()
    assert rel_err(g0[:, fl], f0[:, fl]) < 1e-14
    dom.step(steps)                  # odd step counts end AA on the swapped layout
    g = dom.populations().cpu().numpy()
    err = rel_err(g[:, fl], f_or[:, fl])
    say(f"   max rel |f - f_oracle| = {err:.3e}")
    assert err < 1e-12
    rho_g, u_g = dom.moments()
    rho_o, u_o = m.macroscopic(f_or)
    assert np.abs(rho_g.cpu().numpy()[fl] - rho_o[fl]).max() < 1e-12 * max(1.0, np.abs(rho_o).max())
    if m.nse:
        assert rel_err(u_g.cpu().numpy()[:, fl], u_o[:, fl]) < 1e-11
    dom.close()


@pytest.mark.parametrize("case", ["q9_channel_solid_force", "q19_periodic", "q27_channel_solid_force"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_aa_equals_ab_bitwise(rmrt, case, storage):
    say(f"[AA==AB] {case} {storage}")
    out = {}
    for pattern in ("AB", "AA"):
        m, dom, rho, u, steps = _build(case, rmrt, storage, pattern)
        res = []
        for n in (steps, 1):          # an odd total ends AA on the swapped layout
            dom.step(n)
            res.append(dom.populations().cpu().numpy())
        out[pattern] = res
        dom.close()
    for a, b in zip(out["AB"], out["AA"]):
        assert np.array_equal(a[:, m.fluid], b[:, m.fluid])


@pytest.mark.parametrize("storage", ["f64", "f32dev", "f16dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", ["q9_channel_solid_force", "q19_channel_force", "q27_channel_solid_force",
                                  "q9_ncde_nonlinear"])
def test_graph_replays_match_single_steps(rmrt, case, pattern, storage):
    """Multi-step calls replay cached HIP graphs; single steps launch eagerly.
    The same graph is replayed several times, with eager kernels (moments, a
    reduction) and host synchronisations between the replays, and every replay
    must leave the bits the same number of single steps leaves."""
    _, g, _, _, _ = _build(case, rmrt, storage, pattern)
    _, e, _, _, _ = _build(case, rmrt, storage, pattern)
    # six steps keep the parity, so (6, parity) is one graph replayed three
    # times; five steps alternate between the two parities' graphs
    for k, n in enumerate((6, 6, 6, 5, 5, 5, 256 + 3)):
        g.step(n)
        for _ in range(n):
            e.step(1)
        g.moments()
        g.reduce()
        torch.cuda.synchronize()
        fg, fe = g.populations().cpu().numpy(), e.populations().cpu().numpy()
        assert g.steps_taken() == e.steps_taken()
        assert np.array_equal(fg, fe), (k, n, np.abs(fg - fe).max())
    say(f"[graph replay] {case} {pattern} {storage}: {g.steps_taken()} steps bitwise")
    g.close()
    e.close()


@pytest.mark.parametrize("check_every", [0, 7])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_prepared_graphs_take_no_steps_and_replay_bitwise(rmrt, pattern, check_every):
    """rmrt_step_prepare captures the graphs of a later rmrt_step without
    running them: the step count and the state do not move, and the prepared
    call then leaves the bits of eager single steps (chunks of 256 and a
    remainder, both parities, with and without the health-check split)."""
    prm, _, _ = CASES["q19_channel_force"]
    prm = dict(prm, check_every=check_every)
    m = O.Model(prm)
    rho, u = random_fields(m, seed=11)
    g = rmrt.Domain(rmrt.make_params(**prm, storage="f32dev", pattern=pattern), rho, u)
    e = rmrt.Domain(rmrt.make_params(**prm, storage="f32dev", pattern=pattern), rho, u)
    g.step(1)
    e.step(1)
    before = g.populations().cpu().numpy()
    for n in (300, 5, 6):
        g.prepare(n)
        torch.cuda.synchronize()
        assert g.steps_taken() == e.steps_taken()
        assert np.array_equal(g.populations().cpu().numpy(), before)
        g.step(n)
        for _ in range(n):
            e.step(1)
        torch.cuda.synchronize()
        before = g.populations().cpu().numpy()
        assert np.array_equal(before, e.populations().cpu().numpy()), n
    say(f"[prepared graphs] {pattern} check_every={check_every}: {g.steps_taken()} steps bitwise")
    g.close()
    e.close()


@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_graph_cache_eviction_mid_flight(rmrt, pattern):
    """More distinct step counts than the graph cache holds, issued back to back
    with no host synchronisation, so that cached graphs are dropped while earlier
    ones may still run; then a launch-shape change, which drops them again.  The
    result must be the bits of eager single steps."""
    _, g, _, _, _ = _build("q19_channel_force", rmrt, "f32dev", pattern)
    _, e, _, _, _ = _build("q19_channel_force", rmrt, "f32dev", pattern)
    total = 0
    for n in list(range(2, 22)) + [2, 3]:
        g.step(n)
        total += n
    cap, flags = g.get_launch()
    g.set_launch(0 if cap else 3, flags)
    g.step(7)
    total += 7
    for _ in range(total):
        e.step(1)
    torch.cuda.synchronize()
    assert g.steps_taken() == e.steps_taken() == total
    assert np.array_equal(g.populations().cpu().numpy(), e.populations().cpu().numpy())
    say(f"[graph eviction] {pattern}: {total} steps bitwise")
    g.close()
    e.close()


@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", list(CASES))
def test_two_nodes_per_thread_is_bitwise_identical(rmrt, case, pattern):
    """The paired-node launch (both nodes read before either collides, ragged
    last tile, solid nodes skipped per node) writes exactly what the one-node
    launch writes."""
    say(f"[two nodes per thread] {case} {pattern}")
    out = []
    for fl in (0, rmrt.LAUNCH_WIDE_TILES, rmrt.LAUNCH_WIDE_TILES | rmrt.LAUNCH_PERSISTENT):
        m, dom, rho, u, steps = _build(case, rmrt, "f32dev", pattern)
        dom.set_launch(1 if fl & rmrt.LAUNCH_PERSISTENT else 0, fl)
        dom.step(steps)
        out.append(dom.populations().cpu().numpy())
        dom.close()
    for g in out[1:]:
        assert np.array_equal(g[:, m.fluid], out[0][:, m.fluid])


@pytest.mark.parametrize("storage", ["f64", "f32dev", "f16dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", list(CASES))
def test_buffer_offsets_are_bitwise_identical(rmrt, case, pattern, storage):
    """Buffer addressing of the streams (scalar stream offset, per-lane node
    offset) writes exactly what the 64-bit form writes, with one and with two
    nodes per thread, over an odd number of steps so that both AA phases run.
    With walls or a solid mask, waves without a bounced link take the periodic
    addresses and the others select full 32-bit offsets.

    FP16 storage: the compiler may fuse an FP16 decode product (h_j w_j) into
    the first add of the moment transform in one code form and round it
    separately in the other, so the forms can differ by an FP16 rounding of a
    few stored values; they are held to 2e-4 of max |f| (a half rounding of a
    deviation is 4.9e-4 of the deviation, itself at most ~0.1 of f).  (One and
    two nodes per thread are compared with each other for FP32 only, in the
    test above: in FP16 and FP64 the compiler may contract a product into a
    different add when it schedules two nodes together.)"""
    say(f"[buffer offsets] {case} {pattern} {storage}")
    B, W = rmrt.LAUNCH_BUFFER_OFFSETS, rmrt.LAUNCH_WIDE_TILES
    out = {}
    for fl in (0, B, W, B | W):
        m, dom, rho, u, steps = _build(case, rmrt, storage, pattern)
        dom.set_launch(0, fl)
        assert dom.get_launch() == (0, fl)
        dom.step(steps | 1)
        out[fl] = dom.populations().cpu().numpy()[:, m.fluid]
        dom.close()
    for ref, buf in ((0, B), (W, B | W)):
        if storage == "f16dev":
            err = rel_err(out[buf], out[ref])
            say(f"   f16 flags {buf} vs {ref}: max |df| / max |f| = {err:.2e}")
            assert err < 2e-4, (buf, ref)
        else:
            assert np.array_equal(out[buf], out[ref]), (buf, ref)


@pytest.mark.parametrize("storage", ["f64", "f32dev", "f16dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
@pytest.mark.parametrize("case", list(CASES))
def test_alternating_tile_order_is_bitwise_identical(rmrt, case, pattern, storage):
    """Walking the tiles backwards on odd steps (RMRT_LAUNCH_ALTERNATE_ORDER)
    writes the same bits as the forward order: the nodes of one step are
    independent.  Over an odd number of steps, with one and two nodes per
    thread, buffer or 64-bit addressing, a persistent grid and the XCD order
    (whose ranges, ragged when the tile count is not a multiple of 8, each
    XCD reverses on its own)."""
    say(f"[alternating order] {case} {pattern} {storage}")
    A, B, W, P, X = (rmrt.LAUNCH_ALTERNATE_ORDER, rmrt.LAUNCH_BUFFER_OFFSETS, rmrt.LAUNCH_WIDE_TILES,
                     rmrt.LAUNCH_PERSISTENT, rmrt.LAUNCH_XCD_ORDER)
    out = {}
    for bpc, fl in ((0, B), (0, B | A), (0, A), (0, B | W), (0, B | W | A), (2, B | P), (2, B | P | A),
                    (0, B | X | A), (2, B | P | X | A)):
        m, dom, rho, u, steps = _build(case, rmrt, storage, pattern)
        dom.set_launch(bpc, fl)
        dom.step(steps | 1)
        out[(bpc, fl)] = dom.populations().cpu().numpy()[:, m.fluid]
        dom.close()
    for ref, alt in (((0, B), (0, B | A)), ((0, B), (0, A)), ((0, B | W), (0, B | W | A)), ((2, B | P), (2, B | P | A)),
                     ((0, B), (0, B | X | A)), ((0, B), (2, B | P | X | A))):
        if storage == "f64" or storage == "f32dev" or alt != (0, A):
            assert np.array_equal(out[alt], out[ref]), (ref, alt)
        else:   # FP16, 64-bit against buffer addressing: see the buffer-offsets test
            assert rel_err(out[alt], out[ref]) < 2e-4


@pytest.mark.parametrize("storage,tol", [("f32dev", 1e-5), ("f16dev", 3e-3)])
@pytest.mark.parametrize("case", ["q9_periodic", "q9_channel_solid_force", "q9_ncde_nonlinear", "q19_periodic",
                                  "q19_channel_force", "q27_periodic", "q27_channel_solid_force", "q19_ncde"])
def test_reduced_precision_storage(rmrt, case, storage, tol):
    say(f"[parity {storage}] {case}")
    m, dom, rho, u, steps = _build(case, rmrt, storage, "AA")
    f0, f_or = _oracle_run(case, m, rho, u, steps)
    dom.step(steps)
    rho_g, u_g = dom.moments()
    rho_o, u_o = m.macroscopic(f_or)
    fl = m.fluid
    if m.nse:
        e_rho = np.abs(rho_g.cpu().numpy()[fl] - rho_o[fl]).max() / m.rho0
        e_u = np.abs(u_g.cpu().numpy()[:, fl] - u_o[:, fl]).max() / np.abs(u_o[:, fl]).max()
    else:
        e_rho = np.abs(rho_g.cpu().numpy()[fl] - rho_o[fl]).max() / np.abs(rho_o).max()
        e_u = 0.0
    say(f"   {storage}: rho err {e_rho:.2e}, u err {e_u:.2e}")
    assert e_rho < tol and e_u < tol
    dom.close()


def test_taylor_green_2d_64x32_fp64_2000_steps(rmrt):
    """rD2Q9 NSE Taylor-Green, 64x32, dx = 1, dy = 0.5, U0 = 0.01, nu = 0.02, nu_b = 0.05,
    rho0 = 1 plus seeded 1e-4 noise, FP64, 2000 steps (graph replay)."""
    say("[tg2d] rD2Q9 TG 64x32 2000 steps")
    nx, ny, dx, dy = 64, 32, 1.0, 0.5
    prm = dict(lattice="Q9", n=(nx, ny, 1), dx=(dx, dy, 1.0), nu=0.02, nu_b=0.05)
    m = O.Model(prm)
    rho, u, (kx, ky) = taylor_green_2d(nx, ny, dx, dy, 0.01, m.cs2, noise=1e-4, seed=1)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    f = m.init(rho, u)
    X, Y, _ = grid_coords((nx, ny, 1), (dx, dy, 1.0))
    mode = np.sin(kx * X) * np.cos(ky * Y)
    ts, amps = [], []
    for t in range(100, 2001, 100):
        dom.step(100)
        f = m.step(f, 100)
        if t in (100, 1000, 2000):
            g = dom.populations().cpu().numpy()
            err = rel_err(g, f)
            say(f"   t={t}: max rel |f - f_oracle| = {err:.3e}")
            assert err < 1e-12
        _, ug = dom.moments()
        ts.append(t)
        amps.append((ug[1].cpu().numpy() * mode).sum() / (mode * mode).sum())
    rate = -np.polyfit(ts, np.log(np.abs(amps)), 1)[0]
    exact = 0.02 * (kx**2 + ky**2)
    say(f"   decay rate {rate:.6e} vs nu(kx^2+ky^2) {exact:.6e}")
    assert abs(rate / exact - 1) < 0.01
    dom.close()


@pytest.fixture(scope="module")
def tg3d_q19_32cubed_oracle():
    n, dx = (32, 32, 32), (1.0, 1.0, 2.0)
    prm = dict(lattice="Q19", n=n, dx=dx, nu=0.005, cs2=1.0 / 3.0)
    m = O.Model(prm)
    rho, u, _ = taylor_green_3d(n, dx, 0.02, m.cs2, with_pressure=False)
    steps = 1000
    f = m.step(m.init(rho, u), steps)
    r, uu = m.macroscopic(f)
    return prm, rho, u, steps, r, uu


@pytest.mark.parametrize("storage,tol", [("f32dev", 1e-5), ("f16dev", 3e-3)])
def test_taylor_green_3d_q19_32cubed_reduced_storage(rmrt, tg3d_q19_32cubed_oracle, storage, tol):
    """rD3Q19 3D Taylor-Green with dz = 2 dx on 32^3, FP32/FP16 deviation storage vs FP64 oracle."""
    prm, rho, u, steps, r_o, u_o = tg3d_q19_32cubed_oracle
    say(f"[tg3d 32^3] {storage}")
    dom = rmrt.Domain(rmrt.make_params(**prm, storage=storage, pattern="AA"), rho, u)
    dom.step(steps)
    r_g, u_g = dom.moments()
    e_rho = np.abs(r_g.cpu().numpy() - r_o).max()
    e_u = np.abs(u_g.cpu().numpy() - u_o).max() / 0.02
    say(f"   {storage}: rho err {e_rho:.2e}, u err / U0 {e_u:.2e}")
    assert e_rho < tol and e_u < tol
    dom.close()


def test_ncde_gaussian_hill_256x128_f32dev(rmrt):
    """rD2Q9 NCDE Gaussian hill with D(phi) = 0.01 (1 + phi^2), u = (0.05, 0.02), dy = 0.5,
    FP32 deviation storage, on a 256 x 128 box (oracle-sized), 300 steps."""
    say("[ncde 256x128] f32dev")
    nx, ny, dx, dy = 256, 128, 1.0, 0.5
    prm = dict(lattice="Q9", equation="NCDE", n=(nx, ny, 1), dx=(dx, dy, 1.0), D0=0.01, D2=1.0,
               adv=(0.05, 0.02, 0.0), rho0=0.0)
    m = O.Model(prm)
    phi = gaussian_hill_field(nx, ny, dx, dy, 10.0, 128.0, 32.0)
    f = m.step(m.init(phi, None), 300)
    p_o, _ = m.macroscopic(f)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f32dev", pattern="AA"), phi)
    dom.step(300)
    p_g, _ = dom.moments(with_u=False)
    err = np.abs(p_g.cpu().numpy() - p_o).max() / phi.max()
    say(f"   phi err / peak {err:.2e}")
    assert err < 1e-5
    dom.close()


def _sampled_one_step(rmrt, prm, rho, u, storage, pattern, samples, seed, flags=None):
    """Full-size launch, one step; oracle collision evaluated only at the
    upstream nodes of `samples` sampled outputs (periodic, no walls).  flags:
    launch flags (None = the default launch)."""
    g = rmrt.make_params(**prm, storage=storage, pattern=pattern)
    dom = rmrt.Domain(g, rho, u)
    if flags is not None:
        dom.set_launch(0, flags)
    dom.step(1)
    f_g = dom.populations()
    nx, ny, nz = prm["n"]
    rng = np.random.default_rng(seed)
    idx = np.concatenate([rng.integers(0, nx * ny * nz, size=samples), [0, nx * ny * nz - 1]])
    # oracle: a model of len(idx)*q nodes is only used for its matrices and per-node collision
    lat = prm["lattice"]
    E = O.unit_offsets(lat)
    q = E.shape[0]
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    E3 = np.zeros((q, 3), dtype=np.int64)
    E3[:, : E.shape[1]] = E
    ups = []
    for j in range(q):
        ups.append(((x - E3[j, 0]) % nx) + nx * (((y - E3[j, 1]) % ny) + ny * ((z - E3[j, 2]) % nz)))
    ups = np.stack(ups)                                  # (q, S) upstream node of population j
    flat = ups.reshape(-1)
    sub = dict(prm)
    sub["n"] = (flat.size, 1, 1)
    sub["wall_faces"] = 0
    mo = O.Model(sub)
    rr = rho[flat]
    uu = None if u is None else u[:, flat]
    fstar = mo.collide(mo.init(rr, uu))                  # (q, q*S)
    S = idx.size
    expect = np.stack([fstar[j, j * S:(j + 1) * S] for j in range(q)])
    got = f_g[:, torch.as_tensor(idx, device=f_g.device)].cpu().numpy()
    dom.close()
    return got, expect


@pytest.mark.parametrize("storage,tol", [("f32dev", 2e-6), ("f16dev", 2e-3)])
def test_q19_256x256x128_one_step_sampled(rmrt, storage, tol):
    """rD3Q19 256 x 256 x 128, dz = 2 dx, U0 = 0.02, nu = 0.005: one step at full size in the
    benchmark's launch configuration, 4096 sampled nodes against the oracle."""
    say(f"[q19 256x256x128 sampled] {storage}")
    n, dx = (256, 256, 128), (1.0, 1.0, 2.0)
    prm = dict(lattice="Q19", n=n, dx=dx, nu=0.005, cs2=1.0 / 3.0)
    rho, u, _ = taylor_green_3d(n, dx, 0.02, 1.0 / 3.0)
    got, expect = _sampled_one_step(rmrt, prm, rho, u, storage, "AA", 4096, 3)
    err = np.abs(got - expect).max() / np.abs(expect).max()
    say(f"   sampled max rel err {err:.2e}")
    assert err < tol


@pytest.mark.parametrize("lat,storage,tol", [("Q19", "f32dev", 1e-7), ("Q19", "f16dev", 5e-5), ("Q27", "f32dev", 1e-7),
                                             ("Q9", "f32dev", 1e-7)])
def test_full_size_odd_phase_sampled(rmrt, lat, storage, tol):
    """The second step, the odd AA phase, at full size in the benchmark's default launch
    (alternating tile order, buffer addressing): rD3Q19 / rD3Q27 Taylor-Green at
    256 x 256 x 128 with dz = 2 dx, and the rD2Q9 NCDE Gaussian hill at 2048 x 1024 with
    dy = dx / 2, each with seeded noise so that neighbouring nodes differ.  The GPU's own
    state after the first step is the input: the oracle collides it at the upstream nodes
    of 2048 sampled outputs (plus both ends), and the second step must have pulled exactly
    those values.  With the GPU's own input the only difference is one collision in
    working precision and one store: 3e-9 (FP32) and 4e-6 (FP16) of max |f| observed."""
    rng = np.random.default_rng(11)
    if lat == "Q9":
        n, dx = (2048, 1024, 1), (1.0, 0.5, 1.0)
        prm = dict(lattice="Q9", equation="NCDE", n=n, dx=dx, D0=0.01, D2=1.0, adv=(0.05, 0.02, 0.0), rho0=0.0)
        rho = gaussian_hill_field(n[0], n[1], dx[0], dx[1], 40.0, 1024.0, 256.0)
        rho = rho + 1e-4 * rng.uniform(-1, 1, rho.size)
        u = None
    else:
        n, dx = (256, 256, 128), (1.0, 1.0, 2.0)
        prm = dict(lattice=lat, n=n, dx=dx, nu=0.005, cs2=1.0 / 3.0)
        rho, u, _ = taylor_green_3d(n, dx, 0.02, 1.0 / 3.0)
        rho = rho + 1e-4 * rng.uniform(-1, 1, rho.size)
    say(f"[{lat} {n} odd phase sampled] {storage}")
    dom = rmrt.Domain(rmrt.make_params(**prm, storage=storage, pattern="AA"), rho, u)
    cap, flags = dom.get_launch()
    assert flags & rmrt.LAUNCH_ALTERNATE_ORDER and flags & rmrt.LAUNCH_BUFFER_OFFSETS
    dom.step(1)
    f1 = dom.populations()                                   # (q, N) FP64 on the GPU
    dom.step(1)
    f2 = dom.populations()
    nx, ny, nz = n
    N = nx * ny * nz
    idx = np.concatenate([np.random.default_rng(12).integers(0, N, 2048), [0, N - 1]])
    E = O.unit_offsets(lat)
    q = E.shape[0]
    E3 = np.zeros((q, 3), dtype=np.int64)
    E3[:, : E.shape[1]] = E
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    ups = np.stack([((x - E3[j, 0]) % nx) + nx * (((y - E3[j, 1]) % ny) + ny * ((z - E3[j, 2]) % nz))
                    for j in range(q)])                      # (q, S) upstream node of population j
    flat = ups.reshape(-1)
    fin = f1[:, torch.as_tensor(flat, device=f1.device)].cpu().numpy()
    got = f2[:, torch.as_tensor(idx, device=f2.device)].cpu().numpy()
    dom.close()
    sub = dict(prm, n=(flat.size, 1, 1))
    fstar = O.Model(sub).collide(fin)                        # (q, q S)
    S = idx.size
    expect = np.stack([fstar[j, j * S:(j + 1) * S] for j in range(q)])
    err = np.abs(got - expect).max() / np.abs(expect).max()
    say(f"   launch cap {cap} flags {flags}: sampled max rel err {err:.2e}")
    assert err < tol


def test_ncde_2048x1024_one_step_sampled(rmrt):
    say("[ncde 2048x1024 sampled] f32dev")
    nx, ny, dx, dy = 2048, 1024, 1.0, 0.5
    prm = dict(lattice="Q9", equation="NCDE", n=(nx, ny, 1), dx=(dx, dy, 1.0), D0=0.01, D2=1.0,
               adv=(0.05, 0.02, 0.0), rho0=0.0)
    phi = gaussian_hill_field(nx, ny, dx, dy, 40.0, 1024.0, 256.0)
    got, expect = _sampled_one_step(rmrt, prm, phi, None, "f32dev", "AA", 4096, 2)
    err = np.abs(got - expect).max() / np.abs(expect).max()
    say(f"   sampled max rel err {err:.2e}")
    assert err < 2e-6


def test_conservation_and_reductions(rmrt):
    say("[reductions] Q27 periodic with force, FP64")
    prm = dict(lattice="Q27", n=(17, 13, 11), dx=(1.0, 0.5, 2.0), nu=0.03, force=(1e-5, -2e-5, 3e-6))
    m = O.Model(prm)
    rho, u = random_fields(m, 5)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    r0 = dom.reduce()
    F = np.array(prm["force"])
    for k in range(1, 4):
        dom.step(7)
        r = dom.reduce()
        assert abs(r[0] - r0[0]) < 1e-13 * r0[0]
        np.testing.assert_allclose(r[1:], np.array(r0[1:]) + 7 * k * m.N * F, rtol=0, atol=1e-12)
    # the reduction equals the sum of the macroscopic fields
    rho_g, u_g = dom.moments()
    rho_g, u_g = rho_g.cpu().numpy(), u_g.cpu().numpy()
    r = dom.reduce()
    assert abs(r[0] - rho_g.sum()) < 1e-10
    np.testing.assert_allclose(r[1:], (rho_g[None] * u_g).sum(axis=1), atol=1e-12)
    # steady residual against numpy on the same fields
    assert dom.residual() == float("inf")
    prev = u_g.copy()
    dom.step(3)
    r_res = dom.residual()
    _, u2 = dom.moments()
    u2 = u2.cpu().numpy()
    expect = np.sqrt(((u2 - prev) ** 2).sum() / (u2**2).sum())
    assert abs(r_res - expect) < 1e-12 * max(1.0, expect)
    dom.close()


@pytest.mark.parametrize("case", ["q9_channel_solid_force", "q19_channel_force", "q27_periodic",
                                  "q9_heluo_walls_force", "q27_viscosity_tensor_heluo", "q19_viscosity_tensor"])
def test_init_with_nonequilibrium_part(rmrt, case):
    say(f"[init fne] {case}")
    prm, solid_fn, _ = CASES[case]
    m = O.Model(prm, solid=None if solid_fn is None else solid_fn(prm["n"]))
    rho, u = random_fields(m, 9)
    solid = None if solid_fn is None else m.solid.astype(np.uint8)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern="AB"), rho, u, solid=solid, with_fne=True)
    g = dom.populations().cpu().numpy()
    f = m.init(rho, u, with_fne=True)
    assert rel_err(g[:, m.fluid], f[:, m.fluid]) < 1e-13
    dom.close()


def test_nonfinite_detected_by_health_check(rmrt):
    say("[health] NaN in the initial density")
    prm = dict(lattice="Q9", n=(16, 8, 1), dx=(1.0, 0.5, 1.0), nu=0.05)
    rho = np.ones(128)
    rho[5] = np.nan
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", check_every=2), rho, np.zeros((2, 128)))
    with pytest.raises(rmrt.RMRTError) as ei:
        dom.step(4)
    assert ei.value.code == rmrt.ENONFINITE
    dom.close()


def test_launch_shapes_agree_and_match_oracle(rmrt):
    """Persistent grids of 1..8 workgroups per CU (XCD-ordered or not) and one
    workgroup per tile give bitwise-identical states that match the oracle,
    on a grid large enough (640 tiles) for the persistent walk."""
    say("[launch shapes] Q19 80x64x32 FP64")
    prm = dict(lattice="Q19", n=(80, 64, 32), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.05)
    m = O.Model(prm)
    rho, u = random_fields(m, 21)
    f_or = m.step(m.init(rho, u), 9)
    ref = None
    P, X, Wd = rmrt.LAUNCH_PERSISTENT, rmrt.LAUNCH_XCD_ORDER, rmrt.LAUNCH_WIDE_TILES
    B, A, Ch = rmrt.LAUNCH_BUFFER_OFFSETS, rmrt.LAUNCH_ALTERNATE_ORDER, rmrt.LAUNCH_XCD_CHUNKS
    for bpc, fl in [(0, 0), (0, X), (3, 0), (8, 0), (1, P | X), (2, P | X), (3, P), (8, P | X), (0, Wd),
                    (3, Wd | X), (2, Wd | P | X), (3, B), (0, B | X), (1, B | P | X), (2, B | Wd | P | X),
                    (3, B | A), (0, A | X), (1, A | P | X), (3, A | P), (0, B | Wd | A), (2, B | Wd | P | X | A),
                    (0, Ch), (4, B | A | Ch), (4, B | A | Wd | Ch), (2, B | A | P | Ch)]:
        dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern="AA"), rho, u)
        dom.set_launch(bpc, fl)
        assert dom.get_launch() == (bpc, fl)
        dom.step(9)
        g = dom.populations().cpu().numpy()
        dom.close()
        if ref is None:
            ref = g
            err = rel_err(g, f_or)
            say(f"   max rel |f - f_oracle| = {err:.3e}")
            assert err < 1e-12
        else:
            assert np.array_equal(g, ref), (bpc, fl)


@pytest.mark.parametrize("n", [(45, 37, 29), (64, 32, 40)])
def test_xcd_chunks_are_bitwise_the_plain_order(rmrt, n):
    """RMRT_LAUNCH_XCD_CHUNKS only permutes tiles among workgroups: a walled,
    forced rD3Q27 channel with a ragged tile count (189 tiles: 128 chunked, 61
    in the identity tail; 320 tiles: 256 + 64) steps bitwise as in the plain
    order, with 256- and 512-node tiles, both AA phases."""
    say(f"[xcd chunks] Q27 {n} f32dev")
    N = n[0] * n[1] * n[2]
    rng = np.random.default_rng(5)
    rho, u = 1 + 0.01 * rng.standard_normal(N), 0.02 * rng.standard_normal((3, N))
    W = rmrt.WALL_YM | rmrt.WALL_YP | rmrt.WALL_ZM | rmrt.WALL_ZP
    prm = rmrt.make_params(lattice="Q27", n=n, nu=0.05, force=(1e-5, 0.0, 0.0), wall_faces=W,
                           storage="f32dev", pattern="AA")
    B, A, Ch, Wd = (rmrt.LAUNCH_BUFFER_OFFSETS, rmrt.LAUNCH_ALTERNATE_ORDER, rmrt.LAUNCH_XCD_CHUNKS,
                    rmrt.LAUNCH_WIDE_TILES)
    out = []
    for bpc, fl in [(4, B | A), (4, B | A | Ch), (0, Ch), (3, B | A | Wd | Ch), (3, B | A | Wd)]:
        dom = rmrt.Domain(prm, rho, u)
        dom.set_launch(bpc, fl)
        dom.step(7)
        out.append(dom.populations().cpu().numpy())
        dom.close()
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    assert np.array_equal(out[3], out[4])


def test_tune_picks_a_valid_shape(rmrt):
    say("[tune] Q19 64x64x64 f32dev")
    prm = dict(lattice="Q19", n=(64, 64, 64), dx=(1.0, 1.0, 2.0), nu=0.01)
    N = 64 ** 3
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f32dev", pattern="AA"), np.ones(N), np.zeros((3, N)))
    k = dom.tune(steps=4)
    assert k in (0, 2, 3, 4, 5, 6, 8)
    bpc, fl = dom.get_launch()
    W, B, A = rmrt.LAUNCH_WIDE_TILES, rmrt.LAUNCH_BUFFER_OFFSETS, rmrt.LAUNCH_ALTERNATE_ORDER
    assert bpc == k and fl & A and (fl & ~A) in (0, W, B, W | B)   # 64-node rows: no XCD chunks
    r = dom.reduce()
    assert abs(r[0] - N) < 1e-6 * N
    dom.close()


def test_q27_with_zero_corner_weight_matches_q19(rmrt):
    """Cross-lattice check of the embedded rD3Q19 transform: rD3Q27 with
    omega_19 = 0 reproduces rD3Q19 and keeps its corners at zero."""
    say("[q27 w19=0 vs q19]")
    prm = dict(n=(13, 11, 9), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.07, force=(1e-5, 2e-5, 0.0))
    m = O.Model(dict(prm, lattice="Q19"))
    rho, u = random_fields(m, 17)
    d19 = rmrt.Domain(rmrt.make_params(**prm, lattice="Q19", storage="f64", pattern="AA"), rho, u)
    d27 = rmrt.Domain(rmrt.make_params(**prm, lattice="Q27", w_corner=0.0, storage="f64", pattern="AA"), rho, u)
    d19.step(11)
    d27.step(11)
    g19 = d19.populations().cpu().numpy()
    g27 = d27.populations().cpu().numpy()
    assert np.abs(g27[:19] - g19).max() < 1e-13
    assert np.abs(g27[19:]).max() < 1e-13
    d19.close()
    d27.close()


@pytest.mark.parametrize("lat,n", [("Q27", (1, 1, 1)), ("Q19", (1, 3, 1)), ("Q9", (1, 1, 1)), ("Q9", (5, 1, 1))])
def test_degenerate_single_node_extents(rmrt, lat, n):
    """Axes of one node: every link along them wraps to the node itself."""
    say(f"[degenerate] {lat} {n}")
    d = 2 if lat == "Q9" else 3
    prm = dict(lattice=lat, n=n, dx=(1.0, 0.5, 2.0)[:d] + ((1.0,) if d == 2 else ()), nu=0.04)
    m = O.Model(prm)
    rho, u = random_fields(m, 23)
    f_or = m.step(m.init(rho, u), 7)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage="f64", pattern="AA"), rho, u)
    dom.step(0)                                   # no-op
    assert dom.steps_taken() == 0
    dom.step(7)
    assert rel_err(dom.populations().cpu().numpy(), f_or) < 1e-12
    dom.close()


@pytest.mark.parametrize("lat,n,storage,buffer_offsets", [("Q9", (12000, 12000, 1), "f32dev", False),
                                                          ("Q27", (300, 300, 300), "f64", False),
                                                          ("Q9", (12000, 12000, 1), "f32dev", True)])
def test_byte_offsets_beyond_4_gib(rmrt, lat, n, storage, buffer_offsets):
    """Population buffers larger than 4 GiB (5.2 GB and 5.8 GB): the highest
    streams start beyond 2^32 bytes, so every stream offset must be formed in
    64 bits (buffer addressing, requested or not, must fall back to that form).
    One step, 4096 sampled nodes (and the last node) against the oracle."""
    say(f"[large buffers] {lat} {n} {storage} buffer offsets requested: {buffer_offsets}")
    N = n[0] * n[1] * n[2]
    d = 2 if lat == "Q9" else 3
    q = 9 if lat == "Q9" else 27
    es = 4 if storage == "f32dev" else 8
    prm = dict(lattice=lat, n=n, dx=(1.0, 0.5, 2.0)[:d] + ((1.0,) if d == 2 else ()), nu=0.03)
    assert (q - 1) * N * es > 2**32
    rng = np.random.default_rng(13)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, N)
    u = 0.02 * rng.uniform(-1, 1, (d, N))
    got, expect = _sampled_one_step(rmrt, prm, rho, u, storage, "AA", 4096, 13,
                                    flags=rmrt.LAUNCH_BUFFER_OFFSETS if buffer_offsets else None)
    del rho, u
    err = np.abs(got - expect).max() / np.abs(expect).max()
    say(f"   sampled max rel err {err:.2e}")
    assert err < (2e-6 if storage == "f32dev" else 1e-13)


@pytest.mark.parametrize("lat,storage", [("Q19", "f32dev"), ("Q19", "f16dev"), ("Q27", "f32dev"), ("Q27", "f16dev")])
def test_full_size_taylor_green_decay_rate(rmrt, lat, storage):
    """The benchmark's 256 x 256 x 128, dz = 2 dx, AA configuration (and its
    rD3Q27 / FP16 siblings) run for 2000 steps at U0 = 1e-3 (Re ~ 50, so the
    vortex stays in its linear decay): the kinetic energy decays at
    2 nu (kx^2 + ky^2 + kz^2) within 1%, a property of the recovered
    Navier-Stokes equations at any size."""
    say(f"[full size TG decay] {lat} 256x256x128 {storage}")
    n, dx, nu, U0 = (256, 256, 128), (1.0, 1.0, 2.0), 0.005, 1e-3
    prm = dict(lattice=lat, n=n, dx=dx, nu=nu, cs2=1.0 / 3.0)
    rho, u, (kx, ky, kz) = taylor_green_3d(n, dx, U0, 1.0 / 3.0)
    dom = rmrt.Domain(rmrt.make_params(**prm, storage=storage, pattern="AA"), rho, u)
    del rho, u
    ts, es = [], []
    for t in range(0, 2001, 250):
        if t:
            dom.step(250)
        _, uu = dom.moments()
        ts.append(t)
        es.append(float((uu * uu).sum()))
    dom.close()
    rate = -np.polyfit(ts, np.log(es), 1)[0]
    expect = 2.0 * nu * (kx * kx + ky * ky + kz * kz)
    say(f"   energy decay rate {rate:.6e}, expected {expect:.6e}, ratio {rate / expect:.5f}")
    assert abs(rate / expect - 1.0) < 0.01
