"""GPU parity of the surrogate kernels (MFMA convolutions, their backward
passes, loss, Adam, feature/target/initial-field glue) against the FP64
oracle.  Inputs are rounded to bfloat16 on both sides; products of bf16
values are exact in fp32, so the bar for fp32 results is 1e-5 of the output
scale (accumulation order), and one bf16 rounding (2^-8) for bf16 outputs."""
import sys

import numpy as np
import pytest

from oracle import conv_oracle as C

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


def bf16_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").to(torch.bfloat16).contiguous()


def f32_dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("cin,cout", [(16, 16), (16, 32), (32, 16), (32, 32)])
@pytest.mark.parametrize("dil", [1, 2, 8])
@pytest.mark.parametrize("shape", [(2, 16, 24), (1, 7, 9)])
def test_conv_forward_matches_oracle(R, cin, cout, dil, shape):
    say(f"[nn fwd] cin={cin} cout={cout} dil={dil} shape={shape}")
    B, H, W = shape
    rng = np.random.default_rng(cin * 100 + cout + dil)
    x = C.to_bf16(rng.standard_normal((B, H, W, cin)))
    w = C.to_bf16(rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin))
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    y_or = C.conv_forward(x, w, b, dil)
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    a = torch.empty((B, H, W, cout), dtype=torch.bfloat16, device="cuda")
    R.nn_conv_forward(bf16_dev(x), bf16_dev(w), f32_dev(b), y, a, None, dil, R.NN_EPI_SILU)
    yg = host(y)
    assert np.abs(yg - y_or).max() < 1e-5 * np.abs(y_or).max()
    silu = C.silu(y_or)
    assert np.abs(host(a) - silu).max() <= 2.0**-7 * np.abs(silu).max() + 1e-6


@pytest.mark.parametrize("cin,cout,dil", [(16, 32, 1), (32, 32, 2), (32, 32, 4), (32, 16, 8)])
def test_conv_at_the_surrogate_shape(R, cin, cout, dil):
    """The four layers of the warm-start network at the shape it runs at: batches of
    16 images of 64 x 128 coarse cells (obstacle channels of 512 x 256 nodes coarsened
    4x).  Forward and weight gradient against the oracle on the whole output."""
    say(f"[nn surrogate shape] cin={cin} cout={cout} dil={dil}")
    B, H, W = 16, 64, 128
    rng = np.random.default_rng(31 * dil + cin)
    x = C.to_bf16(rng.standard_normal((B, H, W, cin)))
    w = C.to_bf16(rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin))
    b = rng.standard_normal(cout).astype(np.float32).astype(np.float64)
    y_or = C.conv_forward(x, w, b, dil)
    y = torch.empty((B, H, W, cout), dtype=torch.float32, device="cuda")
    a = torch.empty((B, H, W, cout), dtype=torch.bfloat16, device="cuda")
    R.nn_conv_forward(bf16_dev(x), bf16_dev(w), f32_dev(b), y, a, None, dil, R.NN_EPI_SILU)
    assert np.abs(host(y) - y_or).max() < 1e-5 * np.abs(y_or).max()
    dy = C.to_bf16(rng.standard_normal((B, H, W, cout)))
    dW_or, db_or = C.conv_backward_weight(x, dy, dil)
    dW = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    scr = torch.empty(R.nn_wgrad_scratch_floats(B, H, W, cin, cout), dtype=torch.float32, device="cuda")
    R.nn_conv_backward_weight(bf16_dev(x), bf16_dev(dy), dil, dW, db, scr)
    # sums of B H W = 131072 bf16 products: fp32 accumulation in another order
    assert np.abs(host(dW) - dW_or).max() < 1e-5 * np.abs(dW_or).max() + 1e-4
    assert np.abs(host(db) - db_or).max() < 1e-5 * np.abs(db_or).max() + 1e-4


@pytest.mark.parametrize("cin,cout,dil", [(32, 32, 4), (16, 32, 1), (32, 16, 2)])
def test_backward_data_with_silu_grad(R, cin, cout, dil):
    say(f"[nn bwd data] cin={cin} cout={cout} dil={dil}")
    B, H, W = 2, 12, 20
    rng = np.random.default_rng(7 + dil)
    dy = C.to_bf16(rng.standard_normal((B, H, W, cout)))
    w = C.to_bf16(rng.standard_normal((cout, 3, 3, cin)) / np.sqrt(9 * cin))
    aux = rng.standard_normal((B, H, W, cin)).astype(np.float32).astype(np.float64)
    ref = C.conv_backward_data(dy, w, dil)
    ref_g = ref * C.silu_grad(aux)
    wt = torch.empty((cin, 3, 3, cout), dtype=torch.bfloat16, device="cuda")
    R.nn_flip_weights(bf16_dev(w), wt)
    y = torch.empty((B, H, W, cin), dtype=torch.float32, device="cuda")
    g = torch.empty((B, H, W, cin), dtype=torch.bfloat16, device="cuda")
    R.nn_conv_forward(bf16_dev(dy), wt, None, y, g, f32_dev(aux), dil, R.NN_EPI_SILU_GRAD)
    assert np.abs(host(y) - ref).max() < 1e-5 * np.abs(ref).max()
    assert np.abs(host(g) - ref_g).max() <= 2.0**-7 * np.abs(ref_g).max() + 1e-6


@pytest.mark.parametrize("cin,cout,dil", [(32, 32, 8), (16, 32, 2), (32, 16, 1)])
@pytest.mark.parametrize("shape", [(2, 32, 64), (1, 9, 13)])
def test_backward_weight(R, cin, cout, dil, shape):
    say(f"[nn bwd weight] cin={cin} cout={cout} dil={dil} shape={shape}")
    B, H, W = shape
    rng = np.random.default_rng(11 + dil)
    x = C.to_bf16(rng.standard_normal((B, H, W, cin)))
    dy = C.to_bf16(rng.standard_normal((B, H, W, cout)))
    dW_or, db_or = C.conv_backward_weight(x, dy, dil)
    dW = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device="cuda")
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    scr = torch.empty(R.nn_wgrad_scratch_floats(B, H, W, cin, cout), dtype=torch.float32, device="cuda")
    R.nn_conv_backward_weight(bf16_dev(x), bf16_dev(dy), dil, dW, db, scr)
    scale = np.sqrt(B * H * W)
    assert np.abs(host(dW) - dW_or).max() < 1e-5 * scale * 10
    assert np.abs(host(db) - db_or).max() < 1e-5 * scale * 10


def test_masked_mse_and_adam(R):
    say("[nn loss + adam]")
    rng = np.random.default_rng(3)
    B, H, W = 2, 8, 16
    out = rng.standard_normal((B, H, W, 16)).astype(np.float32).astype(np.float64)
    tgt = rng.standard_normal((B, H, W, 3)).astype(np.float32).astype(np.float64)
    wgt = rng.uniform(0, 1, (B, H, W)).astype(np.float32).astype(np.float64)
    loss_or, dout_or = C.masked_mse(out[..., :3], tgt, wgt)
    dout = torch.empty((B, H, W, 16), dtype=torch.bfloat16, device="cuda")
    scr = torch.empty(1024, dtype=torch.float64, device="cuda")
    inv = torch.empty(1, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float64, device="cuda")
    R.nn_masked_mse(f32_dev(out), f32_dev(tgt), f32_dev(wgt), dout, scr, inv, loss)
    assert abs(loss.item() - loss_or) < 1e-6 * loss_or
    d = host(dout)
    assert np.abs(d[..., :3] - dout_or).max() <= 2.0**-7 * np.abs(dout_or).max()
    assert np.all(d[..., 3:] == 0)
    # Adam: three steps against the oracle
    n = 1000
    w = rng.standard_normal(n)
    wd, md, vd = f32_dev(w), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    wb = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    m, v = np.zeros(n), np.zeros(n)
    w_or = w.astype(np.float32).astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(n).astype(np.float32).astype(np.float64)
        w_or, m, v = C.adam_step(w_or, g, m, v, t, lr=1e-3)
        R.nn_adam(wd, wb, f32_dev(g), md, vd, 1e-3, t)
    assert np.abs(host(wd) - w_or).max() < 1e-6
    assert np.array_equal(host(wb), C.to_bf16(host(wd)))


def test_features_targets_and_warm_fields(R):
    say("[nn glue] features / targets / warm fields")
    B, nx, ny, k, dy, Ut, rs = 2, 32, 16, 4, 0.5, 0.03, 100.0
    rng = np.random.default_rng(5)
    solid = (rng.random((B, ny, nx)) < 0.2).astype(np.uint8)
    re = np.array([20.0, 80.0])
    Hh = ny * dy
    # features
    x0 = torch.empty((B, ny // k, nx // k, 16), dtype=torch.bfloat16, device="cuda")
    R.nn_features(torch.tensor(solid, device="cuda"), f32_dev(re), B, nx, ny, k, dy, 100.0, x0)
    f = host(x0)
    frac = C.avg_pool(solid[..., None].astype(np.float64), k)[..., 0]
    yc = (np.arange(ny // k) * k + 0.5 * k) * dy
    prior_c = 4 * yc * (Hh - yc) / Hh**2
    np.testing.assert_allclose(f[..., 0], C.to_bf16(frac), atol=0)
    np.testing.assert_allclose(f[..., 1], C.to_bf16(np.broadcast_to(prior_c[None, :, None], frac.shape)), atol=0)
    np.testing.assert_allclose(f[..., 2], C.to_bf16(np.broadcast_to((re / 100.0)[:, None, None], frac.shape)), atol=0)
    col = solid.astype(np.float64).mean(axis=1)                       # (B, nx): over the full height
    colc = col.reshape(B, nx // k, k).mean(axis=2)
    np.testing.assert_allclose(f[..., 3], np.broadcast_to(colc[:, None, :], frac.shape), rtol=2.0**-7, atol=1e-7)
    gf = solid.astype(np.float64).mean(axis=(1, 2))
    np.testing.assert_allclose(f[..., 4], np.broadcast_to(gf[:, None, None], frac.shape), rtol=2.0**-7, atol=1e-7)
    assert np.all(f[..., 5:] == 0)
    # targets: fluid means per block
    N = nx * ny
    rho = 1 + 0.01 * rng.standard_normal((B, N))
    u = 0.03 * rng.standard_normal((B, 2, N))
    tg = torch.empty((B, ny // k, nx // k, 3), dtype=torch.float32, device="cuda")
    wg = torch.empty((B, ny // k, nx // k), dtype=torch.float32, device="cuda")
    R.nn_targets(torch.tensor(rho, device="cuda"), torch.tensor(u, device="cuda"), torch.tensor(solid, device="cuda"),
                 B, nx, ny, k, dy, Ut, rs, tg, wg)
    yn = (np.arange(ny) + 0.5) * dy
    prior_n = 4 * yn * (Hh - yn) / Hh**2
    fl = 1.0 - solid.astype(np.float64)
    q0 = (u[:, 0].reshape(B, ny, nx) / Ut - prior_n[None, :, None]) * fl
    q1 = u[:, 1].reshape(B, ny, nx) / Ut * fl
    q2 = (rho.reshape(B, ny, nx) - 1) * rs * fl
    cnt = C.avg_pool(fl[..., None], k)[..., 0] * k * k
    exp = np.stack([C.avg_pool(q[..., None], k)[..., 0] * k * k / np.maximum(cnt, 1) for q in (q0, q1, q2)], -1)
    np.testing.assert_allclose(host(tg), exp, atol=1e-5)
    np.testing.assert_allclose(host(wg), cnt / (k * k), atol=1e-7)
    # warm fields: bilinear upsampling of the coarse output
    out = rng.standard_normal((B, ny // k, nx // k, 16)).astype(np.float32).astype(np.float64)
    r2 = torch.empty((B, N), dtype=torch.float64, device="cuda")
    u2 = torch.empty((B, 2, N), dtype=torch.float64, device="cuda")
    R.nn_warm_fields(f32_dev(out), B, nx, ny, k, dy, Ut, rs, torch.tensor(solid, device="cuda"), r2, u2)
    up = C.upsample_bilinear(out[..., :3], k)
    exp_u = Ut * (prior_n[None, :, None] + up[..., 0]) * fl
    exp_v = Ut * up[..., 1] * fl
    exp_r = 1 + up[..., 2] / rs
    np.testing.assert_allclose(u2.cpu().numpy()[:, 0].reshape(B, ny, nx), exp_u, atol=1e-6)
    np.testing.assert_allclose(u2.cpu().numpy()[:, 1].reshape(B, ny, nx), exp_v, atol=1e-6)
    np.testing.assert_allclose(r2.cpu().numpy().reshape(B, ny, nx), exp_r, atol=1e-6)


def test_network_gradients_match_oracle(R):
    """Full 4-layer forward + backward through the driver against the oracle in
    the network's own storage mode (bf16 stored activations and propagated
    gradients, the rest exact), every dW and db entry compared.  What remains
    is the fp32 accumulation of the GPU against the oracle's fp64: a few
    1e-7 relative per sum, plus an occasional bf16 rounding of a stored value
    that the two accumulations put on different sides of a rounding boundary."""
    say("[nn] network forward/backward vs oracle (bf16 storage mode)")
    from paper_2206_00366_amd.surrogate import Surrogate
    B, H, W = 2, 16, 32
    net = Surrogate(seed=1, B=B, H=H, W=W)
    rng = np.random.default_rng(2)
    x = C.to_bf16(np.concatenate([rng.standard_normal((B, H, W, 3)), np.zeros((B, H, W, 13))], -1))
    # fp32-representable targets and weights, the values the GPU sees
    tgt = (rng.standard_normal((B, H, W, 3)) * 0.1).astype(np.float32).astype(np.float64)
    wgt = rng.uniform(0, 1, (B, H, W)).astype(np.float32).astype(np.float64)
    loss = net.loss_and_grads(bf16_dev(x), f32_dev(tgt), f32_dev(wgt))
    Ws = [C.to_bf16(host(w)) for w in net.w32]
    bs = [host(b) for b in net.b32]
    out, cache = C.network_forward(x, Ws, bs, net.dils, store=C.to_bf16)
    loss_or, dout = C.masked_mse(out[..., :3], tgt, wgt)
    dout_full = np.zeros_like(out)
    dout_full[..., :3] = dout
    grads = C.network_backward(dout_full, cache, Ws, net.dils, store=C.to_bf16)
    say(f"   loss gpu {loss:.9e} oracle {loss_or:.9e}")
    assert abs(loss - loss_or) < 1e-5 * loss_or
    stats = []
    for l in range(4):
        for name, got, ref in (("dW", host(net.gw[l]), grads[l][0]), ("db", host(net.gb[l]), grads[l][1])):
            scale = np.abs(ref).max()
            err = np.abs(got - ref)
            norm = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            frac = float((err <= 1e-5 * scale).mean())
            say(f"   layer {l} {name}: max |d - d_oracle| / max |d_oracle| = {err.max() / scale:.3e}, "
                f"norm {norm:.3e}, entries within 1e-5: {frac:.3f} of {err.size}")
            stats.append((l, name, err.max() / scale, norm, frac))
    for l, name, emax, norm, frac in stats:
        assert emax <= 2e-3, (l, name, emax)
        assert norm <= 5e-4, (l, name, norm)
