"""FP64 reference of the transformer weight network and its backward pass.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s
``cpu_baseline`` leg, never by the GPU library.

The paper's heteroscedastic model estimates one weight per acquisition with a
transformer that reads the raw series and encodes the acquisition times with
sinusoids; a final sigmoid bounds the weight between a minimum and a maximum
(Sec. IV-B, with Lambda = g_theta(x, t) of Sec. II-C).  The paper gives no
widths or depth.  This reference fixes them as the GPU kernels do:

* tokens are the acquisitions of a series; features ``f_t`` are the C
  standardised bands where the acquisition is used (0 elsewhere) and the flag
  ``w_t``;
* embedding ``h = f W_e^T + b_e + PE(t)``, with ``PE(t)[2i] = sin(t w_i)``,
  ``PE(t)[2i+1] = cos(t w_i)``, ``w_i = 10000^(-2i/E)`` and t the day of the
  acquisition;
* ``NL`` pre-norm encoder layers, width ``E``, ``H`` heads of ``DH``, ReLU
  feed-forward of width ``FF``::

      a = LN1(h);  [q k v] = a Wqkv^T + bqkv
      h += softmax(q k^T / sqrt(DH)) v  Wo^T + bo        (per head)
      a2 = LN2(h); h += relu(a2 W1^T + b1) W2^T + b2

* head: ``s = LNf(h) wh + bh`` and ``log10 lambda = lo + (hi - lo) sigmoid(s)``
  (the paper's typical bounds are 1e-6 and 1e10).

Precision follows the kernels.  The residual stream and its gradient are FP32
there (FP64 here).  Values that feed a bfloat16 matrix product are rounded to
bfloat16 (round to nearest even) at the same points: weight matrices,
``LN1``/``LN2`` outputs, q/k/v, the attention output, the ReLU output, the
residual gradient where it enters a product, the gradient of the ReLU input,
the attention output gradient and dq/dk/dv.  Sums are exact here (FP32
accumulators there).  Bias and layer-norm parameter gradients are sums of the
unrounded gradients.

Layouts: tokens ``(B, T, ·)``; ``Wqkv`` ``(3E, E)`` with rows q, then k, then
v, head ``j`` owning rows ``j*DH .. j*DH+DH-1`` of each; attention tensors
``(B, H, T, DH)``.
"""

from __future__ import annotations

import numpy as np

from .convnet_ref import bf16_round

E = 64
H = 2
DH = E // H
FF = 128
NL = 2
LN_EPS = 1e-5
LO, HI = -6.0, 10.0


def _id(a):
    return np.asarray(a, dtype=np.float64)


def sinusoidal(times, e: int = E) -> np.ndarray:
    """Sinusoidal encoding of the acquisition days: ``(T, e)``."""
    t = np.asarray(times, dtype=np.float64)[:, None]
    i = np.arange(e // 2, dtype=np.float64)[None, :]
    om = 10000.0 ** (-2.0 * i / e)
    pe = np.zeros((t.shape[0], e))
    pe[:, 0::2] = np.sin(t * om)
    pe[:, 1::2] = np.cos(t * om)
    return pe


def features(x: np.ndarray, w: np.ndarray, mean, sd) -> np.ndarray:
    """Token features ``(B, T, C + 1)``: bands standardised per band where
    ``w`` is set (0 elsewhere), then the flag (Sec. IV-C standardises the
    spectral values).  ``x``: ``(B, T, C)``; ``w``: ``(B, T)``."""
    obs = (np.asarray(w) != 0)[:, :, None]
    xs = np.where(obs, (np.asarray(x, dtype=np.float64) - np.asarray(mean)) / np.asarray(sd), 0.0)
    return np.concatenate([xs, obs.astype(np.float64)], axis=2)


def init_params(rng: np.random.Generator, F: int, nl: int = NL):
    """Uniform(+-1/sqrt(fan_in)) matrices, zero biases, unit LN gains; FP32-valued."""
    def mat(n, k):
        b = 1.0 / np.sqrt(k)
        return rng.uniform(-b, b, size=(n, k)).astype(np.float32).astype(np.float64)
    p = {"We": mat(E, F), "be": np.zeros(E), "layers": []}
    for _ in range(nl):
        p["layers"].append({
            "g1": np.ones(E), "b1": np.zeros(E),
            "Wqkv": mat(3 * E, E), "bqkv": np.zeros(3 * E),
            "Wo": mat(E, E), "bo": np.zeros(E),
            "g2": np.ones(E), "b2": np.zeros(E),
            "W1": mat(FF, E), "bf1": np.zeros(FF),
            "W2": mat(E, FF), "bf2": np.zeros(E),
        })
    p["gf"] = np.ones(E)
    p["bf"] = np.zeros(E)
    p["wh"] = mat(1, E)[0]
    p["bh"] = np.zeros(1)
    return p


def layernorm(h: np.ndarray, g: np.ndarray, b: np.ndarray):
    """``y = (h - mean) / sqrt(var + eps) * g + b`` over the last axis (biased
    variance).  Returns ``(y, xhat, rstd)``."""
    mu = h.mean(axis=-1, keepdims=True)
    var = ((h - mu) ** 2).mean(axis=-1, keepdims=True)
    rstd = 1.0 / np.sqrt(var + LN_EPS)
    xhat = (h - mu) * rstd
    return xhat * g + b, xhat, rstd


def layernorm_backward(gy: np.ndarray, xhat: np.ndarray, rstd: np.ndarray, g: np.ndarray):
    """Gradients of ``layernorm`` w.r.t. its input, gain and bias."""
    gx = gy * g
    n = xhat.shape[-1]
    gh = rstd * (gx - gx.sum(-1, keepdims=True) / n - xhat * (gx * xhat).sum(-1, keepdims=True) / n)
    red = tuple(range(gy.ndim - 1))
    return gh, (gy * xhat).sum(axis=red), gy.sum(axis=red)


def attention(q: np.ndarray, k: np.ndarray, v: np.ndarray):
    """Scaled dot-product attention per (series, head), all keys visible.
    Returns the output and the log-sum-exp of each query's scaled scores."""
    s = np.einsum("bhqd,bhkd->bhqk", q, k) / np.sqrt(q.shape[-1])
    m = s.max(axis=-1, keepdims=True)
    e = np.exp(s - m)
    l = e.sum(axis=-1, keepdims=True)
    return np.einsum("bhqk,bhkd->bhqd", e / l, v), (m + np.log(l))[..., 0]


def attention_backward(q, k, v, o, lse, go):
    """Gradients of ``attention`` w.r.t. q, k, v from ``go`` (``o`` and ``lse``
    as returned by the forward; the softmax Jacobian uses ``sum_d go*o``)."""
    sc = 1.0 / np.sqrt(q.shape[-1])
    p = np.exp(np.einsum("bhqd,bhkd->bhqk", q, k) * sc - lse[..., None])
    dv = np.einsum("bhqk,bhqd->bhkd", p, go)
    dp = np.einsum("bhqd,bhkd->bhqk", go, v)
    delta = (go * o).sum(-1, keepdims=True)
    ds = p * (dp - delta) * sc
    return np.einsum("bhqk,bhkd->bhqd", ds, k), np.einsum("bhqk,bhqd->bhkd", ds, q), dv


def _heads(a: np.ndarray) -> np.ndarray:
    B, T, _ = a.shape
    return a.reshape(B, T, H, DH).transpose(0, 2, 1, 3)


def _merge(a: np.ndarray) -> np.ndarray:
    B, _, T, _ = a.shape
    return a.transpose(0, 2, 1, 3).reshape(B, T, E)


def forward(p, feats: np.ndarray, times, rounding: bool = True):
    """Network forward: returns the head's pre-sigmoid value ``s`` ``(B, T)``
    and the cache the backward pass reads."""
    rnd = bf16_round if rounding else _id
    h = feats @ p["We"].T + p["be"] + sinusoidal(times)[None]
    cache = {"feats": feats, "layers": []}
    for L in p["layers"]:
        c = {"h_in": h}
        y, c["xhat1"], c["rstd1"] = layernorm(h, L["g1"], L["b1"])
        a = rnd(y)
        qkv = rnd(a @ rnd(L["Wqkv"]).T + L["bqkv"])
        q, k, v = (_heads(qkv[:, :, i * E:(i + 1) * E]) for i in range(3))
        o, lse = attention(q, k, v)
        o = rnd(_merge(o))
        h = h + o @ rnd(L["Wo"]).T + L["bo"]
        y2, c["xhat2"], c["rstd2"] = layernorm(h, L["g2"], L["b2"])
        a2 = rnd(y2)
        f = rnd(np.maximum(a2 @ rnd(L["W1"]).T + L["bf1"], 0.0))
        h = h + f @ rnd(L["W2"]).T + L["bf2"]
        c.update(a=a, qkv=qkv, o=o, lse=lse, a2=a2, f=f)
        cache["layers"].append(c)
    yf, cache["xhatf"], cache["rstdf"] = layernorm(h, p["gf"], p["bf"])
    cache["af"] = yf
    return yf @ p["wh"] + p["bh"][0], cache


def backward(p, cache, gs: np.ndarray, rounding: bool = True):
    """Parameter gradients from ``dL/ds`` ``(B, T)``; same structure as ``p``."""
    rnd = bf16_round if rounding else _id
    red = (0, 1)
    g = {"wh": (gs[:, :, None] * cache["af"]).sum(axis=red), "bh": np.array([gs.sum()]), "layers": []}
    gh, g["gf"], g["bf"] = layernorm_backward(gs[:, :, None] * p["wh"], cache["xhatf"], cache["rstdf"], p["gf"])
    for L, c in zip(reversed(p["layers"]), reversed(cache["layers"])):
        gl = {}
        ghb = rnd(gh)
        gl["W2"] = np.einsum("bte,btf->ef", ghb, c["f"])
        gl["bf2"] = gh.sum(axis=red)
        gf = rnd((ghb @ rnd(L["W2"])) * (c["f"] > 0))
        gl["W1"] = np.einsum("btf,bte->fe", gf, c["a2"])
        gl["bf1"] = gf.sum(axis=red)
        d2, gl["g2"], gl["b2"] = layernorm_backward(gf @ rnd(L["W1"]), c["xhat2"], c["rstd2"], L["g2"])
        gh = gh + d2
        ghb = rnd(gh)
        gl["Wo"] = np.einsum("bte,btf->ef", ghb, c["o"])
        gl["bo"] = gh.sum(axis=red)
        go = rnd(ghb @ rnd(L["Wo"]))
        q, k, v = (_heads(c["qkv"][:, :, i * E:(i + 1) * E]) for i in range(3))
        dq, dk, dv = attention_backward(q, k, v, _heads(c["o"]), c["lse"], _heads(go))
        gqkv = rnd(np.concatenate([_merge(dq), _merge(dk), _merge(dv)], axis=2))
        gl["Wqkv"] = np.einsum("btn,bte->ne", gqkv, c["a"])
        gl["bqkv"] = gqkv.sum(axis=red)
        d1, gl["g1"], gl["b1"] = layernorm_backward(gqkv @ rnd(L["Wqkv"]), c["xhat1"], c["rstd1"], L["g1"])
        gh = gh + d1
        g["layers"].insert(0, gl)
    g["We"] = np.einsum("bte,btf->ef", gh, cache["feats"])
    g["be"] = gh.sum(axis=red)
    return g


def flatten(p) -> np.ndarray:
    """Parameters in the order the GPU side keeps them in one FP32 buffer:
    We, be, then per layer g1 b1 Wqkv bqkv Wo bo g2 b2 W1 bf1 W2 bf2, then gf bf wh bh."""
    parts = [p["We"], p["be"]]
    for L in p["layers"]:
        parts += [L[k] for k in ("g1", "b1", "Wqkv", "bqkv", "Wo", "bo", "g2", "b2", "W1", "bf1", "W2", "bf2")]
    parts += [p["gf"], p["bf"], p["wh"], p["bh"]]
    return np.concatenate([np.ravel(a) for a in parts])
