"""Pins of the warm-start network oracle: the convolution by its sum written
out, the backward pass by central finite differences and by adjoint
identities, bfloat16 rounding by torch's conversion, Adam by torch.optim."""
import numpy as np
import pytest

from oracle import cnn


def brute_conv(x, W, b):
    n, H, Wd, cin = x.shape
    y = np.zeros((n, H, Wd, W.shape[3]))
    for a in range(n):
        for i in range(H):
            for j in range(Wd):
                for dy in range(3):
                    for dx in range(3):
                        ii, jj = i + dy - 1, j + dx - 1
                        if 0 <= ii < H and 0 <= jj < Wd:
                            y[a, i, j] += x[a, ii, jj] @ W[dy, dx]
    return y + b


def test_conv_matches_sum_definition():
    rs = np.random.default_rng(0)
    x = rs.standard_normal((2, 5, 4, 3))
    W = rs.standard_normal((3, 3, 3, 4))
    b = rs.standard_normal(4)
    np.testing.assert_allclose(cnn.conv3x3(x, W, b), brute_conv(x, W, b), atol=1e-12)


def test_conv_backward_adjoint_identities():
    rs = np.random.default_rng(1)
    x = rs.standard_normal((2, 6, 5, 3))
    W = rs.standard_normal((3, 3, 3, 4))
    gy = rs.standard_normal((2, 6, 5, 4))
    gx, gW, gb = cnn.conv3x3_backward(x, W, gy)
    zero = np.zeros(4)
    # <conv(x), gy> = <x, gx> = <W, gW> (bilinear, no bias)
    v = np.sum(cnn.conv3x3(x, W, zero) * gy)
    assert abs(v - np.sum(x * gx)) < 1e-10 * abs(v)
    assert abs(v - np.sum(W * gW)) < 1e-10 * abs(v)
    np.testing.assert_allclose(gb, gy.sum(axis=(0, 1, 2)))


def test_network_gradients_by_finite_differences():
    rs = np.random.default_rng(2)
    params = cnn.init_params(3)
    params[4] = (params[4][0] * 10.0, rs.standard_normal(2) * 0.1)
    zf = rs.standard_normal((1, 6, 6)) + 1j * rs.standard_normal((1, 6, 6))
    label = zf + 0.3 * (rs.standard_normal((1, 6, 6)) + 1j * rs.standard_normal((1, 6, 6)))
    x0, cache = cnn.forward(params, zf)
    grads = cnn.backward(cache, cnn.loss_grad(x0, label))
    h = 1e-6
    for layer in (0, 2, 4):
        W, b = params[layer]
        for _ in range(6):
            idx = tuple(rs.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = list(params); pp[layer] = (Wp, b)
            pm = list(params); pm[layer] = (Wm, b)
            fd = (cnn.loss(cnn.forward(pp, zf)[0], label) - cnn.loss(cnn.forward(pm, zf)[0], label)) / (2 * h)
            an = grads[layer][0][idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)), (layer, idx, fd, an)
        k = int(rs.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[k] += h
        bm[k] -= h
        pp = list(params); pp[layer] = (W, bp)
        pm = list(params); pm[layer] = (W, bm)
        fd = (cnn.loss(cnn.forward(pp, zf)[0], label) - cnn.loss(cnn.forward(pm, zf)[0], label)) / (2 * h)
        assert abs(fd - grads[layer][1][k]) <= 1e-6 * max(1e-3, abs(fd))


def test_parameter_count():
    n = sum(W.size + b.size for W, b in cnn.init_params(0))
    assert n == 28930


def test_bf16_matches_torch_conversion():
    torch = pytest.importorskip("torch")
    rs = np.random.default_rng(4)
    a = np.concatenate([rs.standard_normal(10000) * 10.0 ** rs.integers(-6, 6, 10000),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0])])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(a), ref)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rs = np.random.default_rng(5)
    p0 = rs.standard_normal(50)
    gs = [rs.standard_normal(50) for _ in range(5)]
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = cnn.adam(p, g, m, v, t, lr=1e-2)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)
