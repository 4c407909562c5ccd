"""FP64 reference of the learned-weight network and its training step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s
``cpu_baseline`` leg, never by the GPU library.

The paper estimates the weights with a network g_theta of the series and its
times (Sec. II-C, Sec. IV-B), bounded by a final sigmoid between a minimum
and a maximum (Sec. IV-B), trained by masking observed times and taking the
MSE on them (Sec. IV-C).  The network here is a small 1-D convolution stack
(4 layers, kernel 9, 64 channels, ReLU, "same" zero padding) mapping
(standardised x, w, day-of-year harmonics) over time to a per-day value h; the head maps
``log10 lambda = lo + (hi - lo) sigmoid(h)``.

Precision follows the kernels: weights and stored activations are rounded to
bfloat16 (round to nearest even) at the same points, sums are exact (FP64
here, FP32 accumulators there), the last layer's output h is FP32.

Array layouts: activations ``(B, T, C)``; weights ``(Cout, 9, Cin)``; bias
``(Cout,)``.
"""

from __future__ import annotations

import numpy as np

K = 9
PAD = 4
WIDTHS = (8, 64, 64, 64, 1)


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


def conv1d_same(x: np.ndarray, W: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """``y[b,t,co] = bias[co] + sum_{k,ci} W[co,k,ci] x[b, t+k-4, ci]`` with zero padding."""
    B, T, Cin = x.shape
    Cout = W.shape[0]
    xp = np.zeros((B, T + 2 * PAD, Cin))
    xp[:, PAD:PAD + T] = x
    y = np.zeros((B, T, Cout))
    for k in range(K):
        y += np.einsum("btc,oc->bto", xp[:, k:k + T], W[:, k, :])
    if b is not None:
        y += b
    return y


def conv1d_dgrad(gy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Gradient w.r.t. the input of ``conv1d_same``: ``gx[b,s,ci] = sum_{k,co} W[co,k,ci] gy[b, s-k+4, co]``."""
    B, T, Cout = gy.shape
    Cin = W.shape[2]
    gp = np.zeros((B, T + 2 * PAD, Cout))
    gp[:, PAD:PAD + T] = gy
    gx = np.zeros((B, T, Cin))
    for k in range(K):
        # y[t] uses x[t+k-4]  =>  x[s] receives gy[s-k+4]
        gx += np.einsum("bto,oc->btc", gp[:, 2 * PAD - k:2 * PAD - k + T], W[:, k, :])
    return gx


def conv1d_wgrad(x: np.ndarray, gy: np.ndarray):
    """Gradients of ``conv1d_same`` w.r.t. weights and bias."""
    B, T, Cin = x.shape
    xp = np.zeros((B, T + 2 * PAD, Cin))
    xp[:, PAD:PAD + T] = x
    gW = np.zeros((gy.shape[2], K, Cin))
    for k in range(K):
        gW[:, k, :] = np.einsum("bto,btc->oc", gy, xp[:, k:k + T])
    return gW, gy.sum(axis=(0, 1))


def init_params(rng: np.random.Generator, widths=WIDTHS):
    """He-uniform weights, zero bias (FP32 master copies as float64 arrays)."""
    params = []
    for cin, cout in zip(widths[:-1], widths[1:]):
        bound = np.sqrt(6.0 / (cin * K))
        W = rng.uniform(-bound, bound, size=(cout, K, cin)).astype(np.float32).astype(np.float64)
        params.append((W, np.zeros(cout)))
    return params


def _id(a):
    return np.asarray(a, dtype=np.float64)


def forward(params, x_in: np.ndarray, rounding: bool = True):
    """Network forward with the kernels' rounding points.

    ``x_in``: ``(B, T, 2)`` already bfloat16-valued.  Returns ``(h, acts)``:
    ``h`` ``(B, T)`` FP32-valued output of the last layer and ``acts`` the
    stored bfloat16 activations (inputs of every layer).
    """
    rnd = bf16_round if rounding else _id
    acts = [x_in]
    a = x_in
    n = len(params)
    for i, (W, b) in enumerate(params):
        y = conv1d_same(a, rnd(W), b)
        if i < n - 1:
            a = rnd(np.maximum(y, 0.0))
            acts.append(a)
        else:
            h = y[:, :, 0].astype(np.float32).astype(np.float64) if rounding else y[:, :, 0]
    return h, acts


def backward(params, acts, gh: np.ndarray, rounding: bool = True):
    """Gradients of the parameters from ``dL/dh`` (``(B, T)``), FP64 sums of
    bfloat16 stored values; the gradient flowing between layers is rounded to
    bfloat16 where the kernels store it."""
    rnd = bf16_round if rounding else _id
    grads = [None] * len(params)
    g = rnd(gh)[:, :, None]   # the head's gradient is stored in bfloat16
    for i in range(len(params) - 1, -1, -1):
        W, b = params[i]
        gW, gb = conv1d_wgrad(acts[i], g)
        grads[i] = (gW, gb)
        if i > 0:
            gx = conv1d_dgrad(g, rnd(W))
            g = rnd(gx * (acts[i] > 0))   # ReLU of the layer that produced acts[i]
    return grads


def head(h: np.ndarray, lo: float = -1.0, hi: float = 5.0) -> np.ndarray:
    """Bounded weight per day: ``log10 lambda = lo + (hi - lo) sigmoid(h)`` (Sec. IV-B)."""
    s = 1.0 / (1.0 + np.exp(-h))
    return 10.0 ** (lo + (hi - lo) * s)


def head_rows(lam_day: np.ndarray, d: int) -> np.ndarray:
    """Per-day weights to one weight per row of D: row k takes day ``k + d // 2``."""
    T = lam_day.shape[1]
    o = d // 2
    return lam_day[:, o:o + T - d]


def head_backward(h: np.ndarray, glam_rows: np.ndarray, d: int, lo: float = -1.0, hi: float = 5.0):
    """``dL/dh`` from ``dL/dlambda_k`` (rows) through the head and the row mapping."""
    s = 1.0 / (1.0 + np.exp(-h))
    lam = 10.0 ** (lo + (hi - lo) * s)
    dlam_dh = lam * np.log(10.0) * (hi - lo) * s * (1.0 - s)
    gh = np.zeros_like(h)
    T = h.shape[1]
    o = d // 2
    gh[:, o:o + T - d] = glam_rows * dlam_dh[:, o:o + T - d]
    return gh


def scalar_head(theta: float, P: int, lo: float = -1.0, hi: float = 5.0) -> np.ndarray:
    """Homoscedastic model (Sec. IV-B): one learned scalar weight for every series,
    through the same bounded parametrisation, ``log10 lambda = lo + (hi - lo) sigmoid(theta)``."""
    return np.full(P, head(np.array([float(theta)]), lo, hi)[0])


def scalar_head_backward(theta: float, glam: np.ndarray, lo: float = -1.0, hi: float = 5.0) -> float:
    """``dL/dtheta`` from the per-series ``dL/dlambda`` (every series shares lambda)."""
    s = 1.0 / (1.0 + np.exp(-float(theta)))
    lam = 10.0 ** (lo + (hi - lo) * s)
    return float(np.sum(glam)) * lam * np.log(10.0) * (hi - lo) * s * (1.0 - s)


def masked_mse(z: np.ndarray, x: np.ndarray, mask: np.ndarray):
    """Mean of ``(z - x)^2`` over ``mask`` and its gradient w.r.t. ``z``."""
    m = np.asarray(mask) != 0
    n = max(int(m.sum()), 1)
    r = np.where(m, z - x, 0.0)
    return float((r ** 2).sum() / n), 2.0 * r / n


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba) with bias correction; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def time_features(T: int, start_year: int = 2016) -> np.ndarray:
    """Per-day time encoding ``(T, 4)``: sine and cosine of the first two
    harmonics of the day of year (the paper encodes time with sinusoids, Sec. IV-B)."""
    doy = []
    y = start_year
    while len(doy) < T:
        n = 366 if (y % 4 == 0 and (y % 100 != 0 or y % 400 == 0)) else 365
        doy.extend(range(n))
        y += 1
    a = 2.0 * np.pi * np.asarray(doy[:T], dtype=np.float64) / 365.25
    return np.stack([np.sin(a), np.cos(a), np.sin(2 * a), np.cos(2 * a)], axis=1)


def standardize(x: np.ndarray, w: np.ndarray, mean: float, sd: float, feat: np.ndarray | None = None) -> np.ndarray:
    """Network input ``(B, T, 8)``: standardised x at observed times (0 elsewhere),
    w, four time features and two zero channels, rounded to bfloat16
    (Sec. IV-C standardises the spectral values)."""
    obs = np.asarray(w) != 0
    B, T = obs.shape
    xs = np.where(obs, (x - mean) / sd, 0.0)
    f = time_features(T) if feat is None else feat
    out = np.zeros((B, T, 8))
    out[:, :, 0] = xs
    out[:, :, 1] = obs
    out[:, :, 2:6] = f[None]
    return bf16_round(out)
