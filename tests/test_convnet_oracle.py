"""Pins of the network reference: brute force, torch library routines and
finite differences (CPU only)."""

import numpy as np
import pytest
import torch

from oracle import convnet_ref as N

rng = np.random.default_rng(0)


def test_bf16_rounding_is_torch_bfloat16():
    a = np.concatenate([rng.normal(size=1000) * 10.0 ** rng.integers(-5, 5, size=1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(N.bf16_round(a), ref)


def test_conv_brute_force():
    B, T, Cin, Cout = 2, 11, 3, 4
    x = rng.normal(size=(B, T, Cin))
    W = rng.normal(size=(Cout, 9, Cin))
    b = rng.normal(size=Cout)
    y = N.conv1d_same(x, W, b)
    for bb in range(B):
        for t in range(T):
            for co in range(Cout):
                acc = b[co]
                for k in range(9):
                    s = t + k - 4
                    if 0 <= s < T:
                        for ci in range(Cin):
                            acc += W[co, k, ci] * x[bb, s, ci]
                assert abs(acc - y[bb, t, co]) < 1e-12


def test_conv_and_gradients_match_torch():
    B, T, Cin, Cout = 3, 40, 5, 6
    x = torch.tensor(rng.normal(size=(B, T, Cin)), requires_grad=True)
    W = torch.tensor(rng.normal(size=(Cout, 9, Cin)), requires_grad=True)
    b = torch.tensor(rng.normal(size=Cout), requires_grad=True)
    y = torch.nn.functional.conv1d(x.transpose(1, 2), W.transpose(1, 2), b, padding=4).transpose(1, 2)
    g = torch.tensor(rng.normal(size=(B, T, Cout)))
    (y * g).sum().backward()
    np.testing.assert_allclose(N.conv1d_same(x.detach().numpy(), W.detach().numpy(), b.detach().numpy()),
                               y.detach().numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(N.conv1d_dgrad(g.numpy(), W.detach().numpy()), x.grad.numpy(), rtol=1e-12,
                               atol=1e-12)
    gW, gb = N.conv1d_wgrad(x.detach().numpy(), g.numpy())
    np.testing.assert_allclose(gW, W.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_network_backward_finite_differences():
    widths = (2, 5, 4, 1)
    params = N.init_params(np.random.default_rng(1), widths)
    params = [(W, rng.normal(size=W.shape[0]) * 0.1) for W, _ in params]
    x = rng.normal(size=(2, 25, 2))
    r = rng.normal(size=(2, 25))
    h, acts = N.forward(params, x, rounding=False)
    grads = N.backward(params, acts, r, rounding=False)
    for li in range(len(params)):
        W, b = params[li]
        for idx in [(0, 0, 0), (W.shape[0] - 1, 4, W.shape[2] - 1), (0, 8, 0)]:
            e = 1e-6
            Wp = W.copy(); Wp[idx] += e
            Wm = W.copy(); Wm[idx] -= e
            pp = list(params); pp[li] = (Wp, b)
            pm = list(params); pm[li] = (Wm, b)
            fd = ((N.forward(pp, x, rounding=False)[0] * r).sum() - (N.forward(pm, x, rounding=False)[0] * r).sum()) / (2 * e)
            assert abs(fd - grads[li][0][idx]) < 1e-6 * max(1.0, abs(fd)), (li, idx, fd, grads[li][0][idx])
        e = 1e-6
        bp = b.copy(); bp[0] += e
        bm = b.copy(); bm[0] -= e
        pp = list(params); pp[li] = (W, bp)
        pm = list(params); pm[li] = (W, bm)
        fd = ((N.forward(pp, x, rounding=False)[0] * r).sum() - (N.forward(pm, x, rounding=False)[0] * r).sum()) / (2 * e)
        assert abs(fd - grads[li][1][0]) < 1e-6 * max(1.0, abs(fd))


def test_head_and_loss_gradients():
    h = rng.normal(size=(3, 30))
    d = 2
    g_rows = rng.normal(size=(3, 28))
    gh = N.head_backward(h, g_rows, d)
    e = 1e-6
    for (i, t) in [(0, 1), (1, 15), (2, 28), (0, 0), (2, 29)]:
        hp = h.copy(); hp[i, t] += e
        hm = h.copy(); hm[i, t] -= e
        fd = ((N.head_rows(N.head(hp), d) - N.head_rows(N.head(hm), d)) * g_rows).sum() / (2 * e)
        assert abs(fd - gh[i, t]) <= 1e-6 * max(1.0, abs(fd))
    lam = N.head(h)
    assert (lam >= 0.1 * (1 - 1e-12)).all() and (lam <= 1e5 * (1 + 1e-12)).all()
    z, x = rng.normal(size=(2, 4, 9))
    mask = rng.random((4, 9)) < 0.4
    L, gz = N.masked_mse(z, x, mask)
    assert abs(L - ((z - x)[mask] ** 2).mean()) < 1e-14
    zp = z.copy(); zp[mask][0]
    i, j = np.argwhere(mask)[0]
    zp[i, j] += e
    assert abs((N.masked_mse(zp, x, mask)[0] - L) / e - gz[i, j]) < 1e-5


def test_adam_matches_torch():
    p0 = rng.normal(size=50)
    p = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2)
    q, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(size=50)
        opt.zero_grad()
        p.grad = torch.tensor(g)
        opt.step()
        q, m, v = N.adam_step(q, g, m, v, step, 1e-2)
    np.testing.assert_allclose(q, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_scalar_head_bounds_and_gradient_through_the_smoother():
    from oracle import whs_ref as R
    # midpoint and limits of the bounded parametrisation
    np.testing.assert_allclose(N.scalar_head(0.0, 3), 10.0 ** 2.0, rtol=1e-14)
    assert abs(np.log10(N.scalar_head(60.0, 1)[0]) - 5.0) < 1e-12
    assert abs(np.log10(N.scalar_head(-60.0, 1)[0]) + 1.0) < 1e-12
    # d/dtheta of the held-out MSE of the smoothed series, every series sharing lambda(theta)
    r = np.random.default_rng(3)
    P, T, d = 3, 60, 2
    x = r.normal(size=(P, T)) * 0.1 + 0.3
    w = (r.random((P, T)) < 0.4).astype(np.uint8)
    w[:, :3] = 1
    hold = ((r.random((P, T)) < 0.3) & (w != 0)).astype(np.uint8)
    wtr = w * (1 - hold)

    def loss(theta):
        z, _ = R.solve_band(np.where(wtr != 0, x, 0.0), wtr, N.scalar_head(theta, P), d)
        return N.masked_mse(z, x, hold)[0]

    theta = 0.3
    z, _ = R.solve_band(np.where(wtr != 0, x, 0.0), wtr, N.scalar_head(theta, P), d)
    _, gz = N.masked_mse(z, x, hold)
    _, glam, _ = R.vjp(np.where(wtr != 0, x, 0.0), wtr, N.scalar_head(theta, P), d, gz, z=z)
    an = N.scalar_head_backward(theta, glam)
    h = 1e-5
    fd = (loss(theta + h) - loss(theta - h)) / (2 * h)
    assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12, (fd, an)
