"""Pins of the surrogate's FP64 oracle: library special cases (scipy
correlation, torch bfloat16 rounding), the adjoint identity of the convolution,
central finite differences of the full network loss, closed forms of Adam's
first step and of pooling/upsampling."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from inputs import conv_problem
from oracle import conv_oracle as C


@pytest.mark.parametrize("d", [1, 2, 3])
def test_single_channel_conv_is_scipy_correlation(d):
    rng = np.random.default_rng(d)
    x = rng.standard_normal((1, 13, 17, 1))
    W = rng.standard_normal((1, 3, 3, 1))
    k = np.zeros((2 * d + 1, 2 * d + 1))
    k[::d, ::d] = W[0, :, :, 0]            # dilated kernel
    ref = correlate2d(x[0, :, :, 0], k, mode="same", boundary="fill", fillvalue=0.0)
    got = C.conv_forward(x, W, np.zeros(1), d)[0, :, :, 0]
    np.testing.assert_allclose(got, ref, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 4])
def test_multichannel_conv_matches_brute_force(d):
    rng = np.random.default_rng(10 + d)
    x = rng.standard_normal((2, 6, 7, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    got = C.conv_forward(x, W, b, d)
    ref = np.zeros_like(got)
    for bb in range(2):
        for h in range(6):
            for w in range(7):
                for o in range(4):
                    s = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            hh, ww = h + (ky - 1) * d, w + (kx - 1) * d
                            if 0 <= hh < 6 and 0 <= ww < 7:
                                s += (x[bb, hh, ww, :] * W[o, ky, kx, :]).sum()
                    ref[bb, h, w, o] = s
    np.testing.assert_allclose(got, ref, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 8])
def test_backward_data_is_the_adjoint(d):
    rng = np.random.default_rng(20 + d)
    x = rng.standard_normal((2, 11, 9, 5))
    W = rng.standard_normal((6, 3, 3, 5))
    dy = rng.standard_normal((2, 11, 9, 6))
    y = C.conv_forward(x, W, np.zeros(6), d)
    dx = C.conv_backward_data(dy, W, d)
    assert abs((y * dy).sum() - (x * dx).sum()) < 1e-10


def test_network_gradients_match_finite_differences():
    p = conv_problem(seed=3, B=1, H=7, W=8, cin=2, chid=3, cout=2)
    dils = (1, 2, 1, 2)
    Ws, bs = [w.copy() for w in p["W"]], [b.copy() for b in p["b"]]

    def loss_of(Ws, bs):
        out, _ = C.network_forward(p["x"], Ws, bs, dils)
        return C.masked_mse(out, p["target"], p["mask"])[0]

    out, cache = C.network_forward(p["x"], Ws, bs, dils)
    _, dout = C.masked_mse(out, p["target"], p["mask"])
    grads = C.network_backward(dout, cache, Ws, dils)
    rng = np.random.default_rng(4)
    h = 1e-6
    for l in range(4):
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in Ws[l].shape)
            Wp = [w.copy() for w in Ws]
            Wm = [w.copy() for w in Ws]
            Wp[l][idx] += h
            Wm[l][idx] -= h
            fd = (loss_of(Wp, bs) - loss_of(Wm, bs)) / (2 * h)
            assert abs(fd - grads[l][0][idx]) < 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        k = int(rng.integers(0, bs[l].size))
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][k] += h
        bm[l][k] -= h
        fd = (loss_of(Ws, bp) - loss_of(Ws, bm)) / (2 * h)
        assert abs(fd - grads[l][1][k]) < 1e-6 * max(1.0, abs(fd))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    w1, m, v = C.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=1e-8)
    np.testing.assert_allclose(w1, w - 1e-2 * g / (np.abs(g) + 1e-8), atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_pooling_and_upsampling_closed_forms():
    x = np.full((2, 8, 12, 3), 1.25)
    np.testing.assert_allclose(C.avg_pool(x, 4), 1.25)
    # a field linear in the coarse index is reproduced exactly away from the clamped edges
    h, w, k = 6, 5, 4
    I, J = np.meshgrid(np.arange(h), np.arange(w), indexing="ij")
    coarse = (0.3 * I - 0.7 * J + 0.1)[None, :, :, None]
    fine = C.upsample_bilinear(coarse, k)[0, :, :, 0]
    pi = (np.arange(h * k) + 0.5) / k - 0.5
    pj = (np.arange(w * k) + 0.5) / k - 0.5
    PI, PJ = np.meshgrid(pi, pj, indexing="ij")
    inner = (PI >= 0) & (PI <= h - 1) & (PJ >= 0) & (PJ <= w - 1)
    np.testing.assert_allclose(fine[inner], (0.3 * PI - 0.7 * PJ + 0.1)[inner], atol=1e-12)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    a = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-5, 5, 1000),
                        [1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, -2.5, 0.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.to_bf16(a), ref)


def test_bf16_storage_mode_matches_torch_autograd():
    """The oracle's bf16-storage mode (stored activations and propagated
    gradients rounded to bf16, everything else exact) against the same network
    built from torch's float64 conv2d and autograd on the CPU: a rounding op
    whose gradient passes straight through stores the activations, and
    gradient hooks round dL/dout and every hidden dL/dy."""
    torch = pytest.importorskip("torch")
    p = conv_problem(seed=8, B=2, H=6, W=7, cin=4, chid=8, cout=3)
    dils = (1, 2, 1, 3)
    Ws = [C.to_bf16(w) for w in p["W"]]
    x = C.to_bf16(p["x"])

    class Store(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v):
            return torch.from_numpy(C.to_bf16(v.detach().numpy()))

        @staticmethod
        def backward(ctx, g):
            return g

    def round_grad(g):
        return torch.from_numpy(C.to_bf16(g.numpy()))

    a = torch.tensor(x).permute(0, 3, 1, 2)
    tw = [torch.tensor(w).permute(0, 3, 1, 2).requires_grad_(True) for w in Ws]
    tb = [torch.tensor(b).requires_grad_(True) for b in p["b"]]
    for l in range(4):
        y = torch.nn.functional.conv2d(a, tw[l], tb[l], padding=dils[l], dilation=dils[l])
        y.register_hook(round_grad)
        a = Store.apply(torch.nn.functional.silu(y)) if l < 3 else y
    out_t = a.permute(0, 2, 3, 1)
    m = torch.tensor(p["mask"])
    loss_t = (m[..., None] * (out_t - torch.tensor(p["target"])) ** 2).sum() / m.sum()
    loss_t.backward()

    out, cache = C.network_forward(x, Ws, p["b"], dils, store=C.to_bf16)
    loss, dout = C.masked_mse(out, p["target"], p["mask"])
    grads = C.network_backward(dout, cache, Ws, dils, store=C.to_bf16)
    assert abs(loss - loss_t.item()) < 1e-13 * loss
    for l in range(4):
        gw = tw[l].grad.permute(0, 2, 3, 1).numpy()
        assert np.abs(grads[l][0] - gw).max() < 1e-12 * np.abs(gw).max(), l
        assert np.abs(grads[l][1] - tb[l].grad.numpy()).max() < 1e-12 * np.abs(gw).max(), l
    # the stored activations are bf16 numbers; without rounding the mode is the FP64 network
    for a_l, _ in cache[1:]:
        np.testing.assert_array_equal(a_l, C.to_bf16(a_l))
    out64, _ = C.network_forward(x, Ws, p["b"], dils)
    out_id, _ = C.network_forward(x, Ws, p["b"], dils, store=lambda v: v)
    np.testing.assert_array_equal(out64, out_id)
