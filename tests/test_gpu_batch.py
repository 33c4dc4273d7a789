"""GPU parity of the batched persistent path (many uneven domains in one
launch per step, graph-replayed, tile shapes from the autotuner)."""
import sys

import numpy as np
import pytest

from gpu_util import WALLS, circle_mask, rel_err
from inputs import channel_batch, grid_coords
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


SMALL = [
    dict(lattice="Q27", n=(17, 9, 11), dx=(1.0, 0.5, 2.0), nu=0.03, nu_b=0.02, force=(2e-5, 0.0, 0.0), wall_faces=WALLS["yz"]),
    dict(lattice="Q27", n=(9, 13, 7), dx=(1.0, 2.0, 1.0), nu=0.08, force=(1e-5, 0.0, 0.0), wall_faces=WALLS["yz"]),
    dict(lattice="Q27", n=(23, 7, 5), dx=(1.0, 1.0, 0.5), nu=0.05, force=(3e-5, 0.0, 0.0), wall_faces=WALLS["yz"]),
    dict(lattice="Q27", n=(5, 6, 31), dx=(1.0, 0.5, 0.5), nu=0.02, force=(1e-5, 0.0, 0.0), wall_faces=WALLS["z"]),
]


def _fields(m, seed):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 1e-3 * rng.uniform(-1, 1, m.N)
    u = 0.01 * rng.uniform(-1, 1, (m.d, m.N))
    return rho, u


@pytest.fixture(scope="module")
def small_oracle():
    out = []
    for k, prm in enumerate(SMALL):
        m = O.Model(prm)
        rho, u = _fields(m, 100 + k)
        out.append((m, rho, u, m.step(m.init(rho, u), 21)))
    return out


@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_batch_every_tile_config_matches_oracle(rmrt, small_oracle, pattern):
    ncfg = len(rmrt.Batch.configs())
    for cfg in range(ncfg):
        say(f"[batch f64] {pattern} config {cfg} {rmrt.Batch.configs()[cfg]}")
        b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern=pattern) for p in SMALL])
        b.set_config(cfg)
        for d, (m, rho, u, _) in zip(b.domains, small_oracle):
            d.set_fields(rho, u)
        b.step(20)
        b.step(1)                               # odd total: AA ends on the swapped layout
        for d, (m, rho, u, f_or) in zip(b.domains, small_oracle):
            g = d.populations().cpu().numpy()
            err = rel_err(g, f_or)
            assert err < 1e-12, (cfg, err)
        b.close()


def test_batch_autotune_then_fp32_parity(rmrt, small_oracle):
    say("[batch f32] autotune + parity")
    b = rmrt.Batch([rmrt.make_params(**p, storage="f32dev", pattern="AA") for p in SMALL])
    cfg = b.autotune(steps=3)
    assert 0 <= cfg < len(rmrt.Batch.configs())
    for d, (m, rho, u, _) in zip(b.domains, small_oracle):
        d.set_fields(rho, u)          # the autotuner advanced the state; restart it
    b.step(21)
    for d, (m, rho, u, f_or) in zip(b.domains, small_oracle):
        r_g, u_g = d.moments()
        r_o, u_o = m.macroscopic(f_or)
        assert np.abs(r_g.cpu().numpy() - r_o).max() < 1e-5
        assert np.abs(u_g.cpu().numpy() - u_o).max() / np.abs(u_o).max() < 1e-5
    b.close()


def test_batch_plane_poiseuille(rmrt):
    """Plane channels inside one batch (walls on z or y faces, anisotropic spacing)
    reach the parabolic profile u = g y (H - y) / (2 nu) to O(dy^2)."""
    say("[batch] plane Poiseuille")
    specs = [
        dict(lattice="Q27", n=(4, 4, 24), dx=(1.0, 1.0, 0.5), nu=0.03, force=(1e-5, 0, 0), wall_faces=WALLS["z"]),
        dict(lattice="Q27", n=(4, 24, 4), dx=(1.0, 2.0, 1.0), nu=0.1, force=(3e-6, 0, 0), wall_faces=WALLS["y"]),
    ]
    b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern="AA") for p in specs])
    b.step(30000)
    for d, p in zip(b.domains, specs):
        _, u = d.moments()
        u = u.cpu().numpy()
        axis = 2 if p["wall_faces"] == WALLS["z"] else 1
        X, Y, Z = grid_coords(p["n"], p["dx"], centered=True)
        yc = (X, Y, Z)[axis]
        H = p["n"][axis] * p["dx"][axis]
        exact = O.poiseuille(yc, H, p["force"][0], p["nu"])
        err = np.abs(u[0] - exact).max() / exact.max()
        say(f"   {p['n']} dx={p['dx']}: profile error {err:.2e}")
        assert err < 1e-2
    b.close()


def test_q27_64_channel_batch_one_step_sampled(rmrt):
    """The 64-domain rD3Q27 channel batch (seed 4, about 2e8 nodes, FP32-dev, AA)
    in its autotuned launch: the 4 smallest domains restart from seeded random
    fields, the whole batch takes one step, and 256 random nodes of each (plus
    nodes on every wall face and both ends) are checked against the oracle
    collision at their upstream nodes, or bounced back at the node itself."""
    say("[batch] 64 rD3Q27 channels, sampled")
    doms = channel_batch(seed=4, nd=64)
    walls = WALLS["yz"]
    params = [rmrt.make_params(lattice="Q27", n=d["n"], dx=d["dx"], nu=d["nu"], nu_b=d["nu_b"], force=d["force"],
                               wall_faces=walls, storage="f32dev", pattern="AA") for d in doms]
    b = rmrt.Batch(params)
    b.autotune(steps=2)
    order = np.argsort([d["n"][0] * d["n"][1] * d["n"][2] for d in doms])[:4]
    rng = np.random.default_rng(4)
    fields = {}
    for k in order:                       # restart the 4 checked domains from a known state
        d = doms[k]
        N = d["n"][0] * d["n"][1] * d["n"][2]
        fields[k] = (1.0 + 1e-3 * rng.uniform(-1, 1, N), 0.02 * rng.uniform(-1, 1, (3, N)))
        b.domains[k].set_fields(*fields[k])
    b.step(1)
    E = O.unit_offsets("Q27")
    for k in order:
        d = doms[k]
        nx, ny, nz = d["n"]
        N = nx * ny * nz
        f_g = b.domains[k].populations()
        face = [(x, y, z) for x, y, z in ((3, 0, nz // 2), (4, ny - 1, nz // 3), (5, ny // 2, 0),
                                          (nx - 1, ny // 3, nz - 1), (0, 0, 0), (nx - 1, ny - 1, nz - 1))]
        idx = np.concatenate([rng.integers(0, N, 256), [x + nx * (y + ny * z) for x, y, z in face]])
        x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
        ups, wall = [], []
        for j in range(27):
            sx, sy, sz = (x - E[j, 0]) % nx, y - E[j, 1], z - E[j, 2]
            w = (sy < 0) | (sy >= ny) | (sz < 0) | (sz >= nz)
            ups.append(np.where(w, idx, sx + nx * (np.clip(sy, 0, ny - 1) + ny * np.clip(sz, 0, nz - 1))))
            wall.append(w)
        nodes, inv = np.unique(np.concatenate(ups), return_inverse=True)
        inv = inv.reshape(27, idx.size)
        # the collision is local: a model of just the needed nodes collides them
        prm = dict(lattice="Q27", n=(nodes.size, 1, 1), dx=d["dx"], nu=d["nu"], nu_b=d["nu_b"], force=d["force"])
        mo = O.Model(prm)
        rho, u = fields[k]
        fstar = mo.collide(mo.init(rho[nodes], u[:, nodes]))
        opp = mo.opp
        expect = np.empty((27, idx.size))
        for j in range(27):
            # pulled from the upstream node, or bounced back at this node (opp(j) leaving toward the wall)
            expect[j] = np.where(wall[j], fstar[opp[j], inv[j]], fstar[j, inv[j]])
        got = f_g[:, torch.as_tensor(idx, device=f_g.device)].cpu().numpy()
        err = np.abs(got - expect).max() / np.abs(expect).max()
        say(f"   domain {k} n={d['n']}: sampled max rel err {err:.2e}, {int(np.sum(wall))} bounced links")
        assert err < 2e-6
    b.close()


def test_batch_residuals_match_per_domain(rmrt):
    say("[batch] residuals")
    b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern="AA") for p in SMALL])
    for d, p in zip(b.domains, SMALL):
        m = O.Model(p)
        rho, u = _fields(m, 7)
        d.set_fields(rho, u)
    r0 = b.residuals()
    assert all(v == float("inf") for v in r0)
    prev = [d.moments()[1].cpu().numpy() for d in b.domains]
    b.step(5)
    r = b.residuals()
    for k, d in enumerate(b.domains):
        u = d.moments()[1].cpu().numpy()
        expect = np.sqrt(((u - prev[k]) ** 2).sum() / (u**2).sum())
        assert abs(r[k] - expect) < 1e-12 * max(1.0, expect)
    b.close()


@pytest.mark.parametrize("pattern", ["AA", "AB"])
def test_batch_set_fields_at_odd_parity(rmrt, small_oracle, pattern):
    """Re-initialising a batch domain after an odd number of steps writes the
    layout that parity expects (the swapped one for AA)."""
    say(f"[batch] set_fields at odd parity, {pattern}")
    b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern=pattern) for p in SMALL])
    b.step(3)                                   # odd: AA state is swapped
    for d, (m, rho, u, _) in zip(b.domains, small_oracle):
        d.set_fields(rho, u)
        assert d.steps_taken() == 3
    b.step(21)
    for d, (m, rho, u, f_or) in zip(b.domains, small_oracle):
        g = d.populations().cpu().numpy()
        assert rel_err(g, f_or) < 1e-12
    b.close()


SOLID_MIX = [
    (dict(lattice="Q27", n=(17, 13, 6), dx=(1.0, 0.5, 2.0), nu=0.04, force=(2e-5, 0.0, 0.0), wall_faces=WALLS["yz"]),
     ((6, 6), 3)),
    (dict(lattice="Q27", n=(20, 11, 5), dx=(1.0, 2.0, 1.0), nu=0.06, force=(1e-5, 3e-6, 0.0), wall_faces=0),
     ((9, 5), 2)),
    (dict(lattice="Q27", n=(9, 13, 7), dx=(1.0, 1.0, 0.5), nu=0.05, force=(3e-5, 0.0, 0.0), wall_faces=WALLS["z"]),
     None),
]


@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_batch_with_solid_masks_matches_oracle(rmrt, pattern):
    """A batch mixing domains with solid masks (cylinders), walls, periodic faces
    and one domain without a mask (the batch then steps every domain with link
    words): FP64, 21 steps, against the oracle on every fluid node, for a
    one-workgroup-per-tile, a persistent and a two-nodes-per-thread shape."""
    models, fields, solids, refs = [], [], [], []
    for k, (prm, cyl) in enumerate(SOLID_MIX):
        sol = None if cyl is None else circle_mask(prm["n"], *cyl)
        m = O.Model(prm, solid=sol)
        rho, u = _fields(m, 300 + k)
        if sol is not None:
            u[:, sol] = 0.0
        models.append(m)
        fields.append((rho, u))
        solids.append(None if sol is None else sol.astype(np.uint8))
        refs.append(m.step(m.init(rho, u), 21))
    shapes = rmrt.Batch.configs()
    picks = [0, next(i for i, c in enumerate(shapes) if c[3]), next(i for i, c in enumerate(shapes) if c[4] == 2)]
    for cfg in picks:
        say(f"[batch f64 solids] {pattern} tile shape {cfg} {shapes[cfg]}")
        b = rmrt.Batch([rmrt.make_params(**p, storage="f64", pattern=pattern) for p, _ in SOLID_MIX], solids=solids)
        b.set_config(cfg)
        for k, (rho, u) in enumerate(fields):
            b.domains[k].set_fields(rho, u)
        b.step(21)
        for k, m in enumerate(models):
            g = b.domains[k].populations().cpu().numpy()
            err = rel_err(g[:, m.fluid], refs[k][:, m.fluid])
            say(f"   domain {k}: max rel |f - f_oracle| = {err:.2e}")
            assert err < 1e-12
        b.close()


@pytest.mark.parametrize("storage", ["f32dev", "f16dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_batch_graph_replays_match_single_steps(rmrt, small_oracle, pattern, storage):
    """Batch graphs replayed several times, with eager work (per-domain moments
    and the batch residuals) and host synchronisations between the replays,
    leave the bits of the same number of eagerly launched single steps; with
    domain groups too."""
    for gb in (0, 1):
        bs = []
        for _ in range(2):
            b = rmrt.Batch([rmrt.make_params(**p, storage=storage, pattern=pattern) for p in SMALL])
            b.set_config(0)
            b.set_group_bytes(gb)
            for k, (m, rho, u, _) in enumerate(small_oracle):
                b.domains[k].set_fields(rho, u)
            bs.append(b)
        g, e = bs
        for it, n in enumerate((4, 4, 4, 3, 3)):
            if it == 3:
                # prepared graphs (captured ahead, no steps taken) replay the same bits
                before = g.domains[0].populations().cpu().numpy()
                g.prepare(n)
                torch.cuda.synchronize()
                assert np.array_equal(g.domains[0].populations().cpu().numpy(), before)
            g.step(n)
            for _ in range(n):
                e.step(1)
            g.domains[0].moments()
            g.residuals()
            torch.cuda.synchronize()
            for k in range(len(SMALL)):
                fg = g.domains[k].populations().cpu().numpy()
                fe = e.domains[k].populations().cpu().numpy()
                assert np.array_equal(fg, fe), (gb, it, n, k)
        say(f"[batch graph replay] {pattern} {storage} group bytes {gb}: bitwise")
        g.close()
        e.close()


@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("pattern", ["AB", "AA"])
def test_domain_groups_are_bitwise_identical(rmrt, small_oracle, pattern, storage):
    """Domain groups (each group advanced through all its steps before the next)
    give the bits of the one-group batch: graph chunks and single steps, odd
    totals, one-workgroup-per-tile and persistent shapes; FP64 also against the
    oracle."""
    nbytes = [rmrt.population_bytes(rmrt.make_params(**p, storage=storage, pattern=pattern))
              * (2 if pattern == "AB" else 1) for p in SMALL]
    shapes = rmrt.Batch.configs()
    persistent = next(i for i, c in enumerate(shapes) if c[3])
    for cfg in (0, persistent):
        out = {}
        for gb in (0, 1, max(nbytes[0], nbytes[1]) + min(nbytes)):
            b = rmrt.Batch([rmrt.make_params(**p, storage=storage, pattern=pattern) for p in SMALL])
            b.set_config(cfg)
            b.set_group_bytes(gb)
            lim, ng = b.group_bytes()
            assert lim == gb and (ng == 1 if gb == 0 else 1 < ng <= len(SMALL))
            for k, (m, rho, u, _) in enumerate(small_oracle):
                b.domains[k].set_fields(rho, u)
            b.step(20)
            b.step(1)
            out[gb] = [b.domains[k].populations().cpu().numpy() for k in range(len(SMALL))]
            b.close()
        say(f"[batch groups] {pattern} {storage} config {cfg}: group counts checked")
        for gb, res in out.items():
            for k in range(len(SMALL)):
                assert np.array_equal(res[k], out[0][k]), (gb, k)
        if storage == "f64":
            for k, (m, rho, u, f_or) in enumerate(small_oracle):
                assert rel_err(out[0][k], f_or) < 1e-12


def test_xcd_chunks_are_bitwise_identical(rmrt):
    """rmrt_batch_set_xcd_chunks only permutes tiles among workgroups: modes 0
    and 1 give the same bits, in one group and in one group per domain, with
    256- and 512-node tiles; only the groups whose rows straddle cache lines
    (n[0] x 4 B not a multiple of 128) qualify."""
    W = rmrt.WALL_YM | rmrt.WALL_YP | rmrt.WALL_ZM | rmrt.WALL_ZP
    dims = [(45, 37, 29), (64, 32, 40), (33, 50, 41)]
    prms = [rmrt.make_params(lattice="Q27", n=n, nu=0.04, force=(1e-5, 0.0, 0.0), wall_faces=W,
                             storage="f32dev", pattern="AA") for n in dims]
    rng = np.random.default_rng(8)
    init = []
    for n in dims:
        N = n[0] * n[1] * n[2]
        init.append((1 + 0.01 * rng.standard_normal(N), 0.02 * rng.standard_normal((3, N))))
    shapes = rmrt.Batch.configs()
    wide = next(i for i, c in enumerate(shapes) if not c[3] and c[4] == 2)
    for cfg in (0, wide):
        ref = None
        for gb, mode in ((0, 0), (0, 1), (1, 0), (1, 1)):
            b = rmrt.Batch(prms)
            b.set_config(cfg)
            b.set_group_bytes(gb)
            b.set_xcd_chunks(mode)
            m, g = b.xcd_chunks()
            assert m == mode and g == (1 if gb == 0 else 2)
            for k, (rho, u) in enumerate(init):
                b.domains[k].set_fields(rho, u)
            b.step(6)
            b.step(1)
            out = [b.domains[k].populations().cpu().numpy() for k in range(len(dims))]
            b.close()
            if ref is None:
                ref = out
            else:
                for k in range(len(dims)):
                    assert np.array_equal(out[k], ref[k]), (cfg, gb, mode, k)
        say(f"[batch xcd chunks] config {cfg}: modes and groups bitwise equal")
    b = rmrt.Batch(prms)
    with pytest.raises(rmrt.RMRTError) as e:
        b.set_xcd_chunks(2)
    assert e.value.code == rmrt.EINVAL
    b.close()
