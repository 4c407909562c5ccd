"""Heteroscedastic (transformer) against homoscedastic (one learned weight)
smoothing of irregular multi-band series, both trained through the smoother.

The paper's setting (Sec. II-C, Sec. IV): series of acquisitions at uneven
dates, D the divided-difference operator on those dates, the weight either
one learned scalar for all series or one per acquisition from a transformer
that reads the raw series and its dates; training hides 10 % of the valid
acquisitions of every series (their weight set to 0) and takes the MSE on
them.  Pixels of one batch share their acquisition dates (one patch of a
tile), each with its own validity mask.

Every numerical step runs in the library's kernels; this module draws the
synthetic batches, allocates tensors and orders the calls.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import torch

from . import net, synth, tf, whs

D = 2
S = 64
T_ACQ = 280
C_BANDS = 4


@dataclass
class SitsBatch:
    P: int
    T: int
    C: int
    days: torch.Tensor      # (T,) float64 acquisition days
    coef: torch.Tensor      # (T - d, d + 1) rows of D on those days
    x_train: torch.Tensor   # interleaved (nb, T, C, S) FP32, held-out acquisitions removed
    w_train: torch.Tensor   # interleaved (nb, T, S) uint8
    x_true: torch.Tensor    # interleaved observations (targets at held-out acquisitions)
    hold: torch.Tensor      # interleaved (nb, T, C, S) held-out mask
    n_hold: int             # held-out values (acquisitions x bands)
    x_clean: torch.Tensor | None = None


def make_batch(P: int, seed: int, chunk: int, device, T: int = T_ACQ, C: int = C_BANDS, frac: float = 0.1,
               clouds: float = 0.0) -> SitsBatch:
    """One patch of irregular series with a held-out split.  ``clouds > 0``:
    that fraction of the valid acquisitions is cloud-contaminated and kept
    valid (the mask is withheld); the noise-free signal is kept for scoring."""
    days, b = synth.irregular_sits(P, T, C, seed, device, chunk)
    gen = synth._gen(seed * 7 + chunk * 13 + 1, device)
    x_obs = b.x
    if clouds > 0:
        x_obs, _ = synth.cloud_contaminate(b.x, b.w, clouds, synth._gen(seed * 11 + chunk * 17 + 5, device))
        x_obs = synth._finish(x_obs, b.w)
    hold = synth.holdout_split(b.w, frac, gen)
    w_tr = (b.w != 0) & (hold == 0)
    x_tr = torch.where(w_tr[:, :, None], x_obs, torch.zeros((), dtype=b.x.dtype, device=b.x.device))
    hold_x = hold[:, :, None].expand(P, T, C).contiguous()
    return SitsBatch(P=P, T=T, C=C, days=days, coef=whs.whs_diff_coef(days.contiguous(), D),
                     x_train=synth.pack_series(x_tr.float(), S),
                     w_train=synth.pack_rows(w_tr.to(torch.uint8), S),
                     x_true=synth.pack_series(x_obs.float(), S),
                     hold=synth.pack_series(hold_x, S),
                     n_hold=int(hold.sum().item()) * C,
                     x_clean=synth.pack_series(b.clean.float(), S) if clouds > 0 else None)


def band_stats(batch: SitsBatch):
    """Per-band mean and sd of the valid training values (Sec. IV-C standardises the values)."""
    x = synth.unpack_series(batch.x_train, batch.P).double()
    m = synth.unpack_rows(batch.w_train, batch.P) != 0
    v = x[m]                                    # (n, C)
    return v.mean(0), v.std(0)


class Hetero:
    """Transformer weights per acquisition, trained through the smoother."""

    def __init__(self, device, C: int, mean, sd, seed: int = 0):
        self.device = torch.device(device)
        self.model = tf.TransformerNet(self.device, C, seed=seed)
        self.mean = mean.float().to(self.device)
        self.inv_sd = (1.0 / sd).float().to(self.device)
        self.sd2 = float((sd ** 2).mean())

    def weights(self, b: SitsBatch, keep: bool = False):
        pe = tf.pe(b.days)
        return self.model.forward(b.x_train, b.w_train, b.P, b.T, S, self.mean, self.inv_sd, pe, D, keep=keep)

    def train_step(self, b: SitsBatch, lr: float) -> float:
        lam = self.weights(b, keep=True)
        z, _ = whs.whs_solve(b.x_train, b.w_train, lam, D, b.P, coef=b.coef)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        g = net.mse(z, b.x_true, b.hold, 1.0 / (max(b.n_hold, 1) * self.sd2), loss=loss)
        _, glam, _ = whs.whs_backward(b.w_train, lam, z, g, D, b.P, need_x=False, coef=b.coef)
        self.model.backward(glam)
        self.model.adam(lr)
        return loss.item() / max(b.n_hold, 1) / self.sd2


class Homo:
    """One learned weight for every series (Sec. IV-B), same bounded parametrisation."""

    def __init__(self, device, sd2: float, theta0: float = 0.0):
        self.device = torch.device(device)
        self.theta = torch.full((1,), theta0, dtype=torch.float32, device=self.device)
        self.m = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.sd2 = sd2
        self.step = 0

    def weights(self, b: SitsBatch):
        return net.scalar_head_fwd(self.theta, b.P, lo=tf.LO, hi=tf.HI)

    def train_step(self, b: SitsBatch, lr: float) -> float:
        lam = self.weights(b)
        z, _ = whs.whs_solve(b.x_train, b.w_train, lam, D, b.P, coef=b.coef)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        g = net.mse(z, b.x_true, b.hold, 1.0 / (max(b.n_hold, 1) * self.sd2), loss=loss)
        _, glam, _ = whs.whs_backward(b.w_train, lam, z, g, D, b.P, need_x=False, coef=b.coef)
        gt = net.scalar_head_bwd(self.theta, glam, b.P, lo=tf.LO, hi=tf.HI)
        self.step += 1
        net._chk(net.lib().whs_net_adam(net._p(self.theta), net._p(gt), net._p(self.m), net._p(self.v), 1, lr, 0.9,
                                        0.999, 1e-8, self.step, net._s(self.device)), "whs_net_adam")
        return loss.item() / max(b.n_hold, 1) / self.sd2

    def log10_lambda(self) -> float:
        s = 1.0 / (1.0 + math.exp(-float(self.theta.item())))
        return tf.LO + (tf.HI - tf.LO) * s


def train(device, steps: int = 200, batch_size: int = 4096, lr: float = 1e-3, lr_homo: float = 3e-2,
          seed: int = 2604004807, T: int = T_ACQ, C: int = C_BANDS, clouds: float = 0.0, log=None):
    """Train both models on the same batches (Adam, cosine-decayed learning
    rates).  Returns ``(hetero, homo, seconds_per_hetero_step)``."""
    first = make_batch(batch_size, seed, 0, device, T=T, C=C, clouds=clouds)
    mean, sd = band_stats(first)
    het = Hetero(device, C, mean, sd)
    hom = Homo(device, het.sd2)
    t_het = 0.0
    for s in range(steps):
        b = first if s == 0 else make_batch(batch_size, seed, s, device, T=T, C=C, clouds=clouds)
        c = 0.5 * (1.0 + math.cos(math.pi * s / steps))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lh = het.train_step(b, lr * c)
        torch.cuda.synchronize()
        t_het += time.perf_counter() - t0
        lo = hom.train_step(b, lr_homo * c)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"step {s} loss hetero {lh:.4f} homo {lo:.4f} (log10 lambda {hom.log10_lambda():.2f})")
    return het, hom, t_het / max(steps, 1)


def _sse(z, target, hold) -> float:
    loss = torch.zeros(1, dtype=torch.float64, device=z.device)
    net.mse(z, target, hold, 1.0, loss=loss)
    return loss.item()


def evaluate(het: Hetero, hom: Homo, device, n_series: int = 16384, chunk: int = 4096, seed: int = 2604004808,
             T: int = T_ACQ, C: int = C_BANDS, clouds: float = 0.0):
    """Held-out RMSE (data units) of both models on fresh patches (each with
    its own dates), and the inference throughput of the transformer form."""
    sse_h = sse_o = cl_h = cl_o = 0.0
    n = 0
    t_h = 0.0
    lam_sd = []
    for i, p0 in enumerate(range(0, n_series, chunk)):
        P = min(chunk, n_series - p0)
        b = make_batch(P, seed, i, device, T=T, C=C, clouds=clouds)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam = het.weights(b)
        z_h, _ = whs.whs_solve(b.x_train, b.w_train, lam, D, P, coef=b.coef)
        torch.cuda.synchronize()
        t_h += time.perf_counter() - t0
        z_o, _ = whs.whs_solve(b.x_train, b.w_train, hom.weights(b), D, P, coef=b.coef)
        sse_h += _sse(z_h, b.x_true, b.hold)
        sse_o += _sse(z_o, b.x_true, b.hold)
        if b.x_clean is not None:
            cl_h += _sse(z_h, b.x_clean, b.hold)
            cl_o += _sse(z_o, b.x_clean, b.hold)
        n += b.n_hold
        lam_sd.append(torch.log10(lam.double()).std().item())
    out = {
        "n_series": n_series,
        "acquisitions": T,
        "bands": C,
        "heldout_values": n,
        "rmse_hetero_transformer": math.sqrt(sse_h / n),
        "rmse_homo_scalar": math.sqrt(sse_o / n),
        "gain": 1.0 - math.sqrt(sse_h / n) / math.sqrt(sse_o / n),
        "log10_lambda_homo": hom.log10_lambda(),
        "sd_log10_lambda_hetero": sum(lam_sd) / len(lam_sd),
        "series_per_s_hetero": n_series / t_h,
    }
    if clouds > 0:
        out["clouds"] = clouds
        out["rmse_clean_hetero_transformer"] = math.sqrt(cl_h / n)
        out["rmse_clean_homo_scalar"] = math.sqrt(cl_o / n)
    return out
