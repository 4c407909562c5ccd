"""Pins of the transformer weight-network reference (oracle/transformer_ref.py)
against things other than itself: PyTorch's own pre-norm encoder layer,
attention and layer norm in float64 (independent library routines with the
same definitions), its autograd for every parameter gradient, central finite
differences, closed forms of attention and of the sinusoidal encoding, and
permutation equivariance of an encoder without masks."""

import numpy as np
import pytest
import torch

from oracle import transformer_ref as X
from oracle.convnet_ref import bf16_round

rng = np.random.default_rng(7)


def case(B=2, T=9, C=3, seed=0):
    r = np.random.default_rng(seed)
    p = X.init_params(r, C + 1)
    # non-trivial norms and biases so every parameter matters
    for L in p["layers"]:
        for k in ("g1", "g2"):
            L[k] = 1.0 + 0.2 * r.normal(size=X.E)
        for k in ("b1", "b2", "bqkv", "bo", "bf1", "bf2"):
            L[k] = 0.1 * r.normal(size=L[k].shape)
    p["gf"] = 1.0 + 0.2 * r.normal(size=X.E)
    p["bf"] = 0.1 * r.normal(size=X.E)
    p["be"] = 0.1 * r.normal(size=X.E)
    p["bh"] = np.array([0.3])
    x = r.normal(size=(B, T, C))
    w = (r.random((B, T)) < 0.7).astype(np.uint8)
    times = np.sort(r.choice(np.arange(0, 400, 5), size=T, replace=False)).astype(np.float64)
    return p, X.features(x, w, 0.1, 1.3), times


def torch_model(p):
    """The same network assembled from PyTorch modules (float64)."""
    layers = []
    for L in p["layers"]:
        m = torch.nn.TransformerEncoderLayer(X.E, X.H, X.FF, dropout=0.0, activation="relu",
                                             layer_norm_eps=X.LN_EPS, batch_first=True, norm_first=True,
                                             dtype=torch.float64)
        with torch.no_grad():
            m.norm1.weight.copy_(torch.tensor(L["g1"]))
            m.norm1.bias.copy_(torch.tensor(L["b1"]))
            m.self_attn.in_proj_weight.copy_(torch.tensor(L["Wqkv"]))
            m.self_attn.in_proj_bias.copy_(torch.tensor(L["bqkv"]))
            m.self_attn.out_proj.weight.copy_(torch.tensor(L["Wo"]))
            m.self_attn.out_proj.bias.copy_(torch.tensor(L["bo"]))
            m.norm2.weight.copy_(torch.tensor(L["g2"]))
            m.norm2.bias.copy_(torch.tensor(L["b2"]))
            m.linear1.weight.copy_(torch.tensor(L["W1"]))
            m.linear1.bias.copy_(torch.tensor(L["bf1"]))
            m.linear2.weight.copy_(torch.tensor(L["W2"]))
            m.linear2.bias.copy_(torch.tensor(L["bf2"]))
        m.train()   # the math path, no fused fast path
        layers.append(m)
    return layers


def torch_forward(p, feats, times, layers):
    We = torch.tensor(p["We"], requires_grad=True)
    be = torch.tensor(p["be"], requires_grad=True)
    gf = torch.tensor(p["gf"], requires_grad=True)
    bf = torch.tensor(p["bf"], requires_grad=True)
    wh = torch.tensor(p["wh"], requires_grad=True)
    bh = torch.tensor(p["bh"], requires_grad=True)
    h = torch.tensor(feats) @ We.T + be + torch.tensor(X.sinusoidal(times))[None]
    for m in layers:
        h = m(h)
    s = torch.nn.functional.layer_norm(h, (X.E,), gf, bf, X.LN_EPS) @ wh + bh[0]
    return s, dict(We=We, be=be, gf=gf, bf=bf, wh=wh, bh=bh)


def test_forward_matches_torch_encoder():
    p, f, t = case()
    s, _ = X.forward(p, f, t, rounding=False)
    st, _ = torch_forward(p, f, t, torch_model(p))
    np.testing.assert_allclose(s, st.detach().numpy(), rtol=0, atol=1e-12)


def test_backward_matches_torch_autograd():
    p, f, t = case(seed=3)
    s, cache = X.forward(p, f, t, rounding=False)
    gs = np.random.default_rng(4).normal(size=s.shape)
    g = X.backward(p, cache, gs, rounding=False)
    layers = torch_model(p)
    st, top = torch_forward(p, f, t, layers)
    (st * torch.tensor(gs)).sum().backward()
    for k in ("We", "be", "gf", "bf", "wh", "bh"):
        np.testing.assert_allclose(g[k], top[k].grad.numpy(), rtol=0, atol=1e-11, err_msg=k)
    names = {"g1": "norm1.weight", "b1": "norm1.bias", "Wqkv": "self_attn.in_proj_weight",
             "bqkv": "self_attn.in_proj_bias", "Wo": "self_attn.out_proj.weight", "bo": "self_attn.out_proj.bias",
             "g2": "norm2.weight", "b2": "norm2.bias", "W1": "linear1.weight", "bf1": "linear1.bias",
             "W2": "linear2.weight", "bf2": "linear2.bias"}
    for gl, m in zip(g["layers"], layers):
        params = dict(m.named_parameters())
        for k, n in names.items():
            np.testing.assert_allclose(gl[k], params[n].grad.numpy(), rtol=0, atol=1e-11, err_msg=k)


def test_backward_finite_differences():
    p, f, t = case(B=1, T=6, C=2, seed=5)
    gs = np.random.default_rng(6).normal(size=(1, 6))
    s, cache = X.forward(p, f, t, rounding=False)
    g = X.backward(p, cache, gs, rounding=False)
    r = np.random.default_rng(8)
    eps = 1e-6

    def loss(q):
        return float((X.forward(q, f, t, rounding=False)[0] * gs).sum())

    def perturbed(path, delta):
        import copy
        q = copy.deepcopy(p)
        if len(path) == 1:
            q[path[0]] = q[path[0]] + delta
        else:
            q["layers"][path[0]][path[1]] = q["layers"][path[0]][path[1]] + delta
        return q

    paths = [("We",), ("be",), ("gf",), ("bf",), ("wh",), ("bh",)]
    paths += [(i, k) for i in range(X.NL) for k in ("g1", "Wqkv", "bqkv", "Wo", "g2", "b2", "W1", "bf1", "W2")]
    for path in paths:
        base = p[path[0]] if len(path) == 1 else p["layers"][path[0]][path[1]]
        gg = g[path[0]] if len(path) == 1 else g["layers"][path[0]][path[1]]
        dirn = r.normal(size=np.shape(base))
        fd = (loss(perturbed(path, eps * dirn)) - loss(perturbed(path, -eps * dirn))) / (2 * eps)
        an = float((gg * dirn).sum())
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (path, fd, an)


def test_attention_matches_torch_sdpa():
    q, k, v = (rng.normal(size=(2, X.H, 11, X.DH)) for _ in range(3))
    o, lse = X.attention(q, k, v)
    ot = torch.nn.functional.scaled_dot_product_attention(torch.tensor(q), torch.tensor(k), torch.tensor(v))
    np.testing.assert_allclose(o, ot.numpy(), rtol=0, atol=1e-13)
    s = np.einsum("bhqd,bhkd->bhqk", q, k) / np.sqrt(X.DH)
    np.testing.assert_allclose(lse, torch.logsumexp(torch.tensor(s), -1).numpy(), rtol=0, atol=1e-13)


def test_attention_two_keys_is_logistic():
    # two keys: the first key's weight is the logistic function of the scaled score gap
    q = rng.normal(size=(1, 1, 1, X.DH))
    k = rng.normal(size=(1, 1, 2, X.DH))
    v = np.zeros((1, 1, 2, X.DH))
    v[..., 0, 0] = 1.0
    o, _ = X.attention(q, k, v)
    gap = float(q[0, 0, 0] @ (k[0, 0, 0] - k[0, 0, 1])) / np.sqrt(X.DH)
    assert abs(o[0, 0, 0, 0] - 1.0 / (1.0 + np.exp(-gap))) < 1e-15


def test_attention_equal_keys_average_values():
    q = rng.normal(size=(1, 2, 5, X.DH))
    k = np.repeat(rng.normal(size=(1, 2, 1, X.DH)), 7, axis=2)
    v = rng.normal(size=(1, 2, 7, X.DH))
    o, lse = X.attention(q, k, v)
    np.testing.assert_allclose(o, np.broadcast_to(v.mean(axis=2, keepdims=True), o.shape), atol=1e-15)
    s0 = np.einsum("bhqd,bhd->bhq", q, k[:, :, 0]) / np.sqrt(X.DH)
    np.testing.assert_allclose(lse, s0 + np.log(7.0), atol=1e-13)


def test_layernorm_matches_torch_and_normalises():
    h = rng.normal(size=(3, 5, X.E)) * 3 + 1
    g = rng.normal(size=X.E)
    b = rng.normal(size=X.E)
    y, xhat, _ = X.layernorm(h, g, b)
    yt = torch.nn.functional.layer_norm(torch.tensor(h), (X.E,), torch.tensor(g), torch.tensor(b), X.LN_EPS)
    np.testing.assert_allclose(y, yt.numpy(), atol=1e-13)
    np.testing.assert_allclose(xhat.mean(-1), 0.0, atol=1e-14)
    np.testing.assert_allclose((xhat ** 2).mean(-1), h.var(-1) / (h.var(-1) + X.LN_EPS), atol=1e-13)


def test_sinusoidal_inner_product_depends_on_lag_only():
    t = np.array([0.0, 5.0, 35.0, 1200.0, 3285.0])
    pe = X.sinusoidal(t)
    om = 10000.0 ** (-2.0 * np.arange(X.E // 2) / X.E)
    gram = pe @ pe.T
    lag = t[:, None] - t[None, :]
    np.testing.assert_allclose(gram, np.cos(lag[..., None] * om).sum(-1), atol=1e-10)
    np.testing.assert_allclose(np.diag(gram), X.E / 2, atol=1e-12)
    assert pe[0, 0] == 0.0 and pe[0, 1] == 1.0


def test_permutation_equivariance():
    # no masks and per-token layers: permuting tokens with their times permutes the output
    p, f, t = case(B=2, T=10, seed=9)
    perm = np.random.default_rng(10).permutation(10)
    s, _ = X.forward(p, f, t, rounding=False)
    s2, _ = X.forward(p, f[:, perm], t[perm], rounding=False)
    np.testing.assert_allclose(s2, s[:, perm], atol=1e-12)


def test_rounded_forward_close_to_exact_and_bf16_valued():
    p, f, t = case(seed=11)
    s_r, c = X.forward(p, f, t, rounding=True)
    s_e, _ = X.forward(p, f, t, rounding=False)
    assert np.abs(s_r - s_e).max() < 0.05 * np.abs(s_e).max()
    for k in ("a", "qkv", "o", "a2", "f"):
        a = c["layers"][0][k]
        np.testing.assert_array_equal(a, bf16_round(a))


def test_features_and_flatten():
    x = np.array([[[1.0, 2.0], [np.nan, 7.0]]])
    w = np.array([[1, 0]])
    f = X.features(x, w, np.array([1.0, 0.0]), np.array([2.0, 4.0]))
    np.testing.assert_array_equal(f, [[[0.0, 0.5, 1.0], [0.0, 0.0, 0.0]]])
    p = X.init_params(np.random.default_rng(0), 3)
    n = X.flatten(p).size
    per_layer = 2 * X.E + 3 * X.E * X.E + 3 * X.E + X.E * X.E + X.E + 2 * X.E + 2 * X.FF * X.E + X.FF + X.E
    assert n == X.E * 3 + X.E + X.NL * per_layer + 3 * X.E + 1
