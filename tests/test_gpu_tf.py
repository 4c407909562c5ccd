"""GPU parity of the transformer weight-network kernels against the FP64
reference (oracle/transformer_ref.py) on the same bfloat16 inputs.

Bars: bfloat16 results within one bfloat16 step of the reference rounded the
same way; for attention, plus 1e-4 of the magnitude of the terms summed into
each element (the probabilities travel as a 16-bit split, and sums of terms of
both signs can cancel to nothing, as at T = 1 where dq and dk vanish exactly); FP32 results within 1e-5 relative to the
tensor's largest value (1e-6 for single dot products).  The whole network:
head value within 1e-2 of the reference's own forward; every parameter
gradient within 5e-3 of the reference backward run on the activations the GPU
saved (the wiring of the backward), and within 1e-1 end to end, where
one-step differences in stored bfloat16 values flip ReLU-mask entries.  Sizes span several
64-row tiles, 32-token chunks and 128-row attention chunks with ragged tails;
T = 1, T = 128 and 129 (one staged chunk, and one more row) and T = 643 (the
longest series in the paper's data: six 128-row blocks of queries or keys, the
last ragged) are the edge cases of the attention launch; the embedding runs
with 3 and 10 bands."""

import numpy as np
import pytest
import torch

from oracle import convnet_ref as N
from oracle import transformer_ref as X
from paper_2604_00048_amd import synth, tf

pytestmark = pytest.mark.gpu
rng = np.random.default_rng(2604)
dev = "cuda"
E, FF = X.E, X.FF


def to_bf(a) -> torch.Tensor:
    return torch.tensor(np.asarray(a), dtype=torch.float32).to(torch.bfloat16).view(torch.int16).to(dev)


def from_bf(t: torch.Tensor) -> np.ndarray:
    return t.cpu().view(torch.bfloat16).to(torch.float64).numpy()


def f32(a) -> torch.Tensor:
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)


def ulp_diff(a: np.ndarray, b: np.ndarray) -> int:
    def key(x):
        u = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).view(torch.int16).to(torch.int32).numpy()
        return np.where(u < 0, -(u & 0x7FFF), u)
    return int(np.abs(key(a) - key(b)).max())


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def bfv(shape, scale=1.0):
    return N.bf16_round(rng.normal(size=shape) * scale)


@pytest.mark.parametrize("C", [3, 10])
def test_encoding_and_embedding(C):
    P, T, S = 70, 45, 64
    times = np.sort(rng.choice(np.arange(3300), size=T, replace=False)).astype(np.float64)
    pe = tf.pe(torch.tensor(times, device=dev))
    np.testing.assert_allclose(pe.cpu().double().numpy(), X.sinusoidal(times), atol=2e-7, rtol=0)
    x = rng.normal(size=(P, T, C)).astype(np.float32).astype(np.float64)
    w = (rng.random((P, T)) < 0.6).astype(np.uint8)
    x[w == 0] = np.nan   # never read where unused
    mean = np.float32(rng.uniform(-0.3, 0.3, size=C)).astype(np.float64)
    inv_sd = np.float32(rng.uniform(0.5, 2.0, size=C))
    F = C + 1
    web = rng.normal(size=E * F + E).astype(np.float32)
    feats = torch.empty((P * T, F), dtype=torch.float32, device=dev)
    h = torch.empty((P * T, E), dtype=torch.float32, device=dev)
    xi = synth.pack_series(torch.tensor(x, dtype=torch.float32), S).to(dev)
    wi = synth.pack_rows(torch.tensor(w), S).to(dev)
    tf.embed(xi, wi, P, T, C, S, f32(mean), f32(inv_sd), pe, f32(web), feats, h)
    fr = X.features(x, w, mean, 1.0 / inv_sd.astype(np.float64))
    np.testing.assert_allclose(feats.cpu().double().numpy().reshape(P, T, F), fr, atol=1e-6, rtol=0)
    We = web[:E * F].reshape(E, F).astype(np.float64)
    hr = fr @ We.T + web[E * F:] + X.sinusoidal(times)[None]
    assert rel(h.cpu().double().numpy().reshape(P, T, E), hr) < 1e-6


def test_layernorm_forward_backward():
    M = 1000
    h = rng.normal(size=(M, E)) * 2 + 0.5
    gb = np.concatenate([1 + 0.3 * rng.normal(size=E), 0.2 * rng.normal(size=E)]).astype(np.float32)
    ht = f32(h)
    out = torch.empty((M, E), dtype=torch.int16, device=dev)
    mu = torch.empty(M, dtype=torch.float32, device=dev)
    rs = torch.empty(M, dtype=torch.float32, device=dev)
    tf.ln_fwd(ht, M, f32(gb), out, mu, rs)
    h32 = h.astype(np.float32).astype(np.float64)
    y, xhat, rstd = X.layernorm(h32, gb[:E].astype(np.float64), gb[E:].astype(np.float64))
    assert ulp_diff(from_bf(out), N.bf16_round(y)) <= 1
    assert rel(rs.cpu().double().numpy(), rstd[:, 0]) < 1e-5
    ga = rng.normal(size=(M, E))
    gh0 = rng.normal(size=(M, E))
    gh = f32(gh0)
    dgb = torch.empty(2 * E, dtype=torch.float32, device=dev)
    ws = torch.empty(tf.lib().whs_tf_ln_bwd_workspace_bytes(37) // 4, dtype=torch.float32, device=dev)
    tf.ln_bwd(f32(ga), ht, mu, rs, f32(gb), M, gh, dgb, ws, parts=37)
    ga32 = ga.astype(np.float32).astype(np.float64)
    d, gg, gbb = X.layernorm_backward(ga32, xhat, rstd, gb[:E].astype(np.float64))
    assert rel(gh.cpu().double().numpy() - gh0.astype(np.float32), d) < 1e-5
    assert rel(dgb.cpu().double().numpy(), np.concatenate([gg, gbb])) < 1e-5


LIN_CASES = [(64, 0, 0, 192), (64, 0, 1, 128), (64, 0, 2, 64), (128, 0, 2, 64), (64, 1, 4, 128), (128, 0, 3, 64),
             (64, 1, 0, 64), (192, 0, 3, 64), (64, 0, 3, 64)]


@pytest.mark.parametrize("K,xf32,mode,Nout", LIN_CASES)
def test_linear_modes(K, xf32, mode, Nout):
    M = 200   # four 64-row tiles, the last one ragged
    x = rng.normal(size=(M, K)) if xf32 else bfv((M, K))
    W = bfv((Nout, K), 0.2)
    b = rng.normal(size=Nout).astype(np.float32).astype(np.float64)
    xin = f32(x) if xf32 else to_bf(x)
    xr = N.bf16_round(x.astype(np.float32).astype(np.float64)) if xf32 else x
    acc = xr @ W.T
    mask = bfv((M, Nout)) if mode == 4 else None
    res = rng.normal(size=(M, Nout)).astype(np.float32).astype(np.float64) if mode == 2 else None
    bias = None if mode in (3, 4) or (mode == 0 and xf32) else b
    bterm = 0.0 if bias is None else bias
    if mode in (0, 1, 4):
        out = torch.empty((M, Nout), dtype=torch.int16, device=dev)
    else:
        out = f32(res) if mode == 2 else torch.empty((M, Nout), dtype=torch.float32, device=dev)
    tf.linear(xin, xf32, K, to_bf(W), None if bias is None else f32(bias), Nout, mode,
              None if mask is None else to_bf(mask), out if mode == 2 else None, out, M)
    if mode == 0:
        assert ulp_diff(from_bf(out), N.bf16_round(acc + bterm)) <= 1
    elif mode == 1:
        assert ulp_diff(from_bf(out), N.bf16_round(np.maximum(acc + bterm, 0))) <= 1
    elif mode == 4:
        assert ulp_diff(from_bf(out), N.bf16_round(acc * (mask > 0))) <= 1
    elif mode == 2:
        assert rel(out.cpu().double().numpy(), res + acc + bterm) < 1e-6
    else:
        assert rel(out.cpu().double().numpy(), acc) < 1e-6


@pytest.mark.parametrize("Nout,K,dyf32", [(64, 128, 1), (128, 64, 0), (64, 64, 1), (192, 64, 0)])
def test_weight_gradient(Nout, K, dyf32):
    M = 1000   # 32-token chunks with a ragged tail; more workgroups than chunks per workgroup
    dy = rng.normal(size=(M, Nout)) if dyf32 else bfv((M, Nout))
    x = bfv((M, K))
    dwb = torch.empty(Nout * K + Nout, dtype=torch.float32, device=dev)
    ws = torch.empty(tf.lib().whs_tf_wgrad_workspace_bytes(Nout, K, 13) // 4, dtype=torch.float32, device=dev)
    tf.wgrad(f32(dy) if dyf32 else to_bf(dy), dyf32, Nout, to_bf(x), K, M, dwb, ws, parts=13)
    dy32 = dy.astype(np.float32).astype(np.float64)
    dyr = N.bf16_round(dy32)
    g = dwb.cpu().double().numpy()
    assert rel(g[:Nout * K].reshape(Nout, K), dyr.T @ x) < 1e-5
    assert rel(g[Nout * K:], dy32.sum(0)) < 1e-5


def attn_inputs(P, T):
    qkv = bfv((P, T, 3 * E))
    heads = lambda a: a.reshape(P, T, X.H, X.DH).transpose(0, 2, 1, 3)   # noqa: E731
    return qkv, [heads(qkv[:, :, i * E:(i + 1) * E]) for i in range(3)]


def merge(a):
    P, _, T, _ = a.shape
    return a.transpose(0, 2, 1, 3).reshape(P, T, E)


def close_terms(got, ref, scale, frac=1e-4):
    """Within one bfloat16 step of ref, plus ``frac`` of the magnitude of the
    terms summed into each element (``scale``, the same sums over absolute
    values): FP32 sums and the 16-bit split of the probabilities err relative to
    the terms, not to a result that cancels."""
    return bool((np.abs(got - ref) <= 2.0 ** -7 * np.abs(ref) + frac * scale).all())


def attention_term_scales(q, k, v, lse, go, o):
    """Per element, the sums of absolute terms behind o, dq, dk and dv."""
    sc = 1.0 / np.sqrt(X.DH)
    p = np.exp(np.einsum("bhqd,bhkd->bhqk", q, k) * sc - lse[..., None])
    o_s = np.einsum("bhqk,bhkd->bhqd", p, np.abs(v))
    dp = np.einsum("bhqd,bhkd->bhqk", go, v)
    dsa = p * (np.abs(dp) + np.abs((go * o).sum(-1, keepdims=True))) * sc
    return (o_s, np.einsum("bhqk,bhkd->bhqd", dsa, np.abs(k)), np.einsum("bhqk,bhqd->bhkd", dsa, np.abs(q)),
            np.einsum("bhqk,bhqd->bhkd", p, np.abs(go)))


@pytest.mark.parametrize("T", [1, 37, 128, 129, 300, 643])
def test_attention_forward_backward(T):
    check_attention(2, T)


def test_attention_longest_sequence():
    # the largest T the attention calls accept: 32 staged key chunks, 32 query blocks
    check_attention(1, 4096)


def check_attention(P, T):
    qkv, (q, k, v) = attn_inputs(P, T)
    o = torch.empty((P * T, E), dtype=torch.int16, device=dev)
    lse = torch.empty((P, X.H, T), dtype=torch.float32, device=dev)
    qt = to_bf(qkv.reshape(P * T, 3 * E))
    tf.attn_fwd(qt, P, T, o, lse)
    o_ref, lse_ref = X.attention(q, k, v)
    got_o = from_bf(o).reshape(P, T, E)
    go = bfv((P, T, E))
    heads = lambda a: a.reshape(P, T, X.H, X.DH).transpose(0, 2, 1, 3)   # noqa: E731
    o_s, dq_s, dk_s, dv_s = attention_term_scales(q, k, v, lse_ref, heads(go), heads(got_o))
    assert close_terms(got_o, N.bf16_round(merge(o_ref)), merge(o_s))
    assert np.abs(lse.cpu().double().numpy() - lse_ref).max() < 1e-5 * max(1.0, np.abs(lse_ref).max())
    dqkv = torch.empty((P * T, 3 * E), dtype=torch.int16, device=dev)
    tf.attn_bwd(qt, o, to_bf(go.reshape(P * T, E)), lse, P, T, dqkv)
    dq, dk, dv = X.attention_backward(q, k, v, heads(got_o), lse_ref, heads(go))
    got = from_bf(dqkv).reshape(P, T, 3 * E)
    for i, (ref, sc) in enumerate(((dq, dq_s), (dk, dk_s), (dv, dv_s))):
        assert close_terms(got[:, :, i * E:(i + 1) * E], N.bf16_round(merge(ref)), merge(sc)), i


def test_head_forward_backward():
    P, T, S, d = 70, 41, 64, 2
    M = P * T
    h = rng.normal(size=(M, E)) * 1.5
    hp = np.concatenate([1 + 0.3 * rng.normal(size=E), 0.2 * rng.normal(size=E), 0.3 * rng.normal(size=E),
                         [0.4]]).astype(np.float32)
    s = torch.empty(M, dtype=torch.float32, device=dev)
    mu = torch.empty(M, dtype=torch.float32, device=dev)
    rs = torch.empty(M, dtype=torch.float32, device=dev)
    nb = (P + S - 1) // S
    lam = torch.empty((nb, T - d, S), dtype=torch.float32, device=dev)
    ht = f32(h)
    tf.head_fwd(ht, P, T, f32(hp), S, d, X.LO, X.HI, s, mu, rs, lam)
    h32 = h.astype(np.float32).astype(np.float64)
    hp64 = hp.astype(np.float64)
    y, xhat, rstd = X.layernorm(h32, hp64[:E], hp64[E:2 * E])
    s_ref = y @ hp64[2 * E:3 * E] + hp64[3 * E]
    assert rel(s.cpu().double().numpy(), s_ref) < 1e-5
    s32 = s.cpu().double().numpy().reshape(P, T)
    lam_ref = N.head_rows(N.head(s32, X.LO, X.HI), d)
    assert np.max(np.abs(synth.unpack_rows(lam.cpu(), P).double().numpy() / lam_ref - 1)) < 1e-6
    glam = rng.normal(size=(P, T - d)) * 1e-3
    gl = synth.pack_rows(torch.tensor(glam, dtype=torch.float32), S).to(dev)
    gh = torch.empty((M, E), dtype=torch.float32, device=dev)
    dhp = torch.empty(3 * E + 1, dtype=torch.float32, device=dev)
    ws = torch.empty(tf.lib().whs_tf_head_bwd_workspace_bytes(29) // 4, dtype=torch.float32, device=dev)
    tf.head_bwd(ht, s, mu, rs, f32(hp), gl, P, T, S, d, X.LO, X.HI, gh, dhp, ws, parts=29)
    gs = N.head_backward(s32, glam.astype(np.float32).astype(np.float64), d, X.LO, X.HI).reshape(M)
    gy = gs[:, None] * hp64[2 * E:3 * E]
    ghr, dgf, dbf = X.layernorm_backward(gy, xhat, rstd, hp64[:E])
    assert rel(gh.cpu().double().numpy(), ghr) < 1e-5
    ref = np.concatenate([dgf, dbf, (gs[:, None] * y).sum(0), [gs.sum()]])
    assert rel(dhp.cpu().double().numpy(), ref) < 1e-5


def test_embedding_gradient_and_cast():
    M, F = 1000, 5
    gh = rng.normal(size=(M, E))
    feats = rng.normal(size=(M, F))
    dweb = torch.empty(E * F + E, dtype=torch.float32, device=dev)
    ws = torch.empty(tf.lib().whs_tf_embed_bwd_workspace_bytes(F, 17) // 4, dtype=torch.float32, device=dev)
    tf.embed_bwd(f32(gh), f32(feats), M, F, dweb, ws, parts=17)
    g32, f32_ = gh.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64)
    g = dweb.cpu().double().numpy()
    assert rel(g[:E * F].reshape(E, F), g32.T @ f32_) < 1e-5
    assert rel(g[E * F:], g32.sum(0)) < 1e-5
    W = rng.normal(size=(192, 64)).astype(np.float32)
    out = torch.empty((192, 64), dtype=torch.int16, device=dev)
    out_t = torch.empty((64, 192), dtype=torch.int16, device=dev)
    tf.cast(f32(W), 192, 64, out, out_t)
    Wb = N.bf16_round(W.astype(np.float64))
    np.testing.assert_array_equal(from_bf(out), Wb)
    np.testing.assert_array_equal(from_bf(out_t), Wb.T)


def oracle_params(model: tf.TransformerNet):
    th = model.theta.cpu().double().numpy()

    def get(name):
        off, shp = model.lay[name]
        return th[off:off + int(np.prod(shp))].reshape(shp).copy()
    p = {"We": get("We"), "be": get("be"), "gf": get("gf"), "bf": get("bf"), "wh": get("wh"), "bh": get("bh"),
         "layers": [{k: get(f"{i}.{k}") for k, _ in tf.LAYER_KEYS} for i in range(model.nl)]}
    return p


def test_whole_network_forward_backward():
    P, T, C, S, d = 3, 150, 2, 64, 2
    model = tf.TransformerNet(dev, C, seed=5)
    # non-trivial norms and biases
    for name, (off, shp) in model.lay.items():
        n = int(np.prod(shp))
        key = name.split(".")[-1]
        if key in ("g1", "g2", "gf"):
            model.theta[off:off + n] += f32(0.2 * rng.normal(size=n))
        elif not key.startswith("W") and key != "wh":
            model.theta[off:off + n] = f32(0.1 * rng.normal(size=n))
    model.cast()
    p = oracle_params(model)
    times = np.sort(rng.choice(np.arange(0, 3300, 5), size=T, replace=False)).astype(np.float64)
    x = (rng.normal(size=(P, T, C)) * 0.1 + 0.3).astype(np.float32).astype(np.float64)
    w = (rng.random((P, T)) < 0.7).astype(np.uint8)
    mean = np.float32([0.3, 0.3]).astype(np.float64)
    inv_sd = np.float32([10.0, 10.0])
    xi = synth.pack_series(torch.tensor(x, dtype=torch.float32), S).to(dev)
    wi = synth.pack_rows(torch.tensor(w), S).to(dev)
    pe = tf.pe(torch.tensor(times, device=dev))
    lam = model.forward(xi, wi, P, T, S, f32(mean), f32(inv_sd), pe, d)
    feats = X.features(x, w, mean, 1.0 / inv_sd.astype(np.float64))
    s_ref, cache = X.forward(p, feats, times, rounding=True)
    s_gpu = model.cache["s"].cpu().double().numpy().reshape(P, T)
    assert rel(s_gpu, s_ref) < 1e-2
    lam_own = N.head_rows(N.head(s_gpu, X.LO, X.HI), d)
    assert np.max(np.abs(synth.unpack_rows(lam.cpu(), P).double().numpy() / lam_own - 1)) < 1e-6
    # dL/dlambda chosen so every token's dL/ds is of order one: with bounds
    # 1e-6 .. 1e10 dlambda/ds spans many decades, and a few tokens would
    # otherwise carry the whole gradient (and any ReLU-mask flip in them)
    sg = 1.0 / (1.0 + np.exp(-s_gpu))
    dl = 10.0 ** (X.LO + (X.HI - X.LO) * sg) * np.log(10.0) * (X.HI - X.LO) * sg * (1.0 - sg)
    glam = (rng.normal(size=(P, T)) / dl)[:, d // 2:d // 2 + T - d]
    gl = synth.pack_rows(torch.tensor(glam, dtype=torch.float32), S).to(dev)
    model.backward(gl)
    gs = N.head_backward(s_gpu, glam.astype(np.float32).astype(np.float64), d, X.LO, X.HI)
    G = model.grad.cpu().double().numpy()

    def got(name):
        off, shp = model.lay[name]
        return G[off:off + int(np.prod(shp))].reshape(shp)

    def compare(g, tol):
        for k in ("We", "be", "gf", "bf", "wh", "bh"):
            assert rel(got(k), g[k]) < tol, k
        for i in range(model.nl):
            for k, _ in tf.LAYER_KEYS:
                assert rel(got(f"{i}.{k}"), g["layers"][i][k]) < tol, (i, k)

    # the backward kernels on the GPU's own saved activations: differences are
    # FP32 sums and one-step roundings of gradient values only
    compare(X.backward(p, gpu_cache(model, p), gs, rounding=True), 5e-3)
    # end to end against the reference's own forward: a pre-activation that
    # lands on the other side of zero flips a ReLU mask entry, an error of
    # about the square root of the flip rate in the weight gradients
    compare(X.backward(p, cache, gs, rounding=True), 1e-1)


def gpu_cache(model: tf.TransformerNet, p):
    """The reference backward's cache built from the activations the GPU saved."""
    c0 = model.cache
    P, T = c0["P"], c0["T"]
    M = P * T

    def f64(t):
        return t.cpu().double().numpy()

    def xh(h, mu, rs):
        return ((f64(h) - f64(mu)[:, None]) * f64(rs)[:, None]).reshape(P, T, E), f64(rs).reshape(P, T, 1)
    cache = {"feats": f64(c0["feats"]).reshape(P, T, model.F), "layers": []}
    for c in c0["acts"]:
        x1, r1 = xh(c["h_in"], c["mu1"], c["rs1"])
        x2, r2 = xh(c["h_mid"], c["mu2"], c["rs2"])
        cache["layers"].append(dict(h_in=f64(c["h_in"]).reshape(P, T, E), xhat1=x1, rstd1=r1, xhat2=x2, rstd2=r2,
                                    a=from_bf(c["a"]).reshape(P, T, E), qkv=from_bf(c["qkv"]).reshape(P, T, 3 * E),
                                    o=from_bf(c["o"]).reshape(P, T, E), lse=f64(c["lse"]),
                                    a2=from_bf(c["a2"]).reshape(P, T, E), f=from_bf(c["f"]).reshape(P, T, FF)))
    cache["xhatf"], cache["rstdf"] = xh(c0["h"], c0["muf"], c0["rsf"])
    cache["af"] = cache["xhatf"] * p["gf"] + p["bf"]
    assert M == P * T
    return cache


def test_bfloat16_rounding_is_nearest_even():
    # exact ties at several exponents and signs, their neighbours, values that
    # round up into the next binade and past the largest finite value, plus
    # random values over many binades (FP32 denormals are not used anywhere)
    one = np.float32(1.0)
    e = [np.float32(2.0 ** k) for k in (-20, -3, 0, 5, 40)]
    ties = []
    for s in e:
        for m in range(8):
            t = s * (one + np.float32((2 * m + 1) * 2.0 ** -8))      # halfway between two bfloat16 values
            ties += [t, -t, np.nextafter(t, np.float32(0)), np.nextafter(t, np.float32(np.inf))]
    special = [np.float32(1.9999999), np.float32(3.3e38), np.float32(3.4e38), np.float32(0.0), np.float32(-0.0)]
    rnd = (rng.normal(size=4000) * 10.0 ** rng.uniform(-30, 30, size=4000)).astype(np.float32)
    v = np.concatenate([np.array(ties + special, dtype=np.float32), rnd])
    out = torch.empty((1, v.size), dtype=torch.int16, device=dev)
    tf.cast(f32(v), 1, v.size, out)
    got = out.cpu().view(torch.bfloat16).to(torch.float64).numpy()[0]
    np.testing.assert_array_equal(got, N.bf16_round(v.astype(np.float64)))
