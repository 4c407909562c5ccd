"""Training and evaluation of the learned-weight form against the plain form.

Learned form (Sec. II-C, Sec. IV-B, Sec. IV-C): per-day weights from the
network, one weight per difference row, trained end to end through the
smoother by hiding 10 % of the observed points of every series and taking
the MSE on them.  Plain form: one scalar weight per series chosen by GCV over
a grid.  Both forms see the same inputs (held-out points removed) and are
scored on the same held-out points of fresh series.

Every numerical step runs in the library's kernels; this module draws the
synthetic batches, allocates tensors and orders the calls.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import torch

from . import net, synth, whs

D = 2
S = 64                # interleave of the evaluation chunks (one lane per series fills the chip)
SMALL_BATCH = 8192    # training batches up to this size are series-contiguous
T_DAYS = 3288
GRID = [10.0 ** (-1.0 + 0.3 * i) for i in range(21)]


def layout_for(P: int) -> int:
    """Interleave of a batch of P series.  Up to a few thousand series, one lane
    per series leaves most of the chip idle and the smoother calls wait on the
    sequential recurrence (about 0.64 ms for the solve of 4096 or of 16384 series
    of 3288 days); series-contiguous tensors (interleave 1) take the partition
    kernel instead, 256 lanes per series (0.26 ms for 4096), and the network's
    input and head kernels read them coalesced."""
    return 1 if P <= SMALL_BATCH else S


@dataclass
class Batch:
    P: int
    x_train: torch.Tensor   # interleaved (nb, T, 1, S) FP32, held-out points removed
    w_train: torch.Tensor   # interleaved (nb, T, S) uint8
    x_true: torch.Tensor    # interleaved observations (targets at held-out points)
    hold: torch.Tensor      # interleaved held-out mask
    n_hold: int
    x_clean: torch.Tensor | None = None   # interleaved noise-free signal (cloud experiments)
    S: int = S              # interleave of every series-side tensor of the batch


def make_batch(P: int, seed: int, chunk: int, device, T: int = T_DAYS, frac: float = 0.1,
               clouds: float = 0.0, S: int | None = None) -> Batch:
    """One batch of the nine-year daily generator (band 0), with a held-out split,
    interleave ``S`` (``layout_for(P)`` when None).

    ``clouds > 0``: that fraction of the acquisitions is cloud-contaminated and
    still marked observed (the cloud mask is withheld, Sec. IV-C); the held-out
    targets are the observed values, as in training on real series, and the
    noise-free signal is kept for evaluation."""
    b = synth.multiband_homoscedastic(P, T=T, C=1, d=D, seed=seed, device=device, chunk=chunk)
    gen = synth._gen(seed * 7 + chunk * 13 + 1, device)
    x_obs = b.x
    if clouds > 0:
        x_obs, _ = synth.cloud_contaminate(b.x, b.w, clouds, synth._gen(seed * 11 + chunk * 17 + 5, device))
        x_obs = synth._finish(x_obs, b.w)
    hold = synth.holdout_split(b.w, frac, gen)
    w_tr = (b.w != 0) & (hold == 0)
    if S is None:
        S = layout_for(P)
    x_tr = torch.where(w_tr[:, :, None], x_obs, torch.zeros((), dtype=b.x.dtype, device=b.x.device))
    return Batch(P=P,
                 x_train=synth.pack_series(x_tr.float(), S),
                 w_train=synth.pack_rows(w_tr.to(torch.uint8), S),
                 x_true=synth.pack_series(x_obs.float(), S),
                 hold=synth.pack_rows(hold, S),
                 n_hold=int(hold.sum().item()),
                 x_clean=synth.pack_series(b.clean.float(), S) if clouds > 0 else None,
                 S=S)


def input_stats(batch: Batch):
    """Global mean and sd of the observed training values (Sec. IV-C standardises the values)."""
    m = batch.w_train != 0
    v = batch.x_train[:, :, 0, :][m].double()
    return float(v.mean()), float(v.std())


class Learned:
    """The network plus the statistics and scratch tensors of one batch size."""

    def __init__(self, device, mean: float, sd: float, seed: int = 0):
        self.device = torch.device(device)
        self.model = net.ConvNet(self.device, seed=seed)
        self.mean, self.sd = mean, sd
        self.feat = net.time_features(T_DAYS).to(self.device)

    def weights(self, batch: Batch, keep: bool = False):
        """h and the per-difference weights of a batch."""
        x8 = net.net_input(batch.x_train, batch.w_train, batch.P, T_DAYS, batch.S, self.mean, self.sd, self.feat)
        h = self.model.forward(x8, batch.P, T_DAYS) if keep else self.model.infer(x8, batch.P, T_DAYS)
        lam = net.head_fwd(h, batch.P, T_DAYS, batch.S, D)
        return h, lam

    def train_step(self, batch: Batch, lr: float) -> float:
        h, lam = self.weights(batch, keep=True)
        # series-contiguous batches: the in-place partition kernel (staged=False)
        z, info = whs.whs_solve(batch.x_train, batch.w_train, lam, D, batch.P, staged=False)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        # MSE in standardised units: (z - x)^2 / sd^2 averaged over held-out points
        g = net.mse(z, batch.x_true, batch.hold, 1.0 / (max(batch.n_hold, 1) * self.sd ** 2), loss=loss)
        _, glam, _ = whs.whs_backward(batch.w_train, lam, z, g, D, batch.P, need_x=False, staged=False)
        gh = net.head_bwd1(h, glam, batch.P, T_DAYS, batch.S, D)
        self.model.backward1(gh, batch.P, T_DAYS)
        self.model.adam(lr)
        return loss.item() / max(batch.n_hold, 1) / self.sd ** 2


class LearnedScalar:
    """Homoscedastic model (Sec. IV-B): one learned weight shared by every series,
    through the same bounded parametrisation as the per-day head."""

    def __init__(self, device, theta0: float = 0.0):
        self.device = torch.device(device)
        self.theta = torch.full((1,), theta0, dtype=torch.float32, device=self.device)
        self.m = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.v = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0

    def weights(self, batch: Batch):
        return net.scalar_head_fwd(self.theta, batch.P)

    def train_step(self, batch: Batch, lr: float, sd: float) -> float:
        lam = self.weights(batch)
        z, _ = whs.whs_solve(batch.x_train, batch.w_train, lam, D, batch.P, staged=False)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        g = net.mse(z, batch.x_true, batch.hold, 1.0 / (max(batch.n_hold, 1) * sd ** 2), loss=loss)
        _, glam, _ = whs.whs_backward(batch.w_train, lam, z, g, D, batch.P, need_x=False, staged=False)
        gt = net.scalar_head_bwd(self.theta, glam, batch.P)
        self.step += 1
        net._chk(net.lib().whs_net_adam(net._p(self.theta), net._p(gt), net._p(self.m), net._p(self.v), 1, lr, 0.9,
                                        0.999, 1e-8, self.step, net._s(self.device)), "whs_net_adam")
        return loss.item() / max(batch.n_hold, 1) / sd ** 2

    def log10_lambda(self) -> float:
        return math.log10(net.scalar_head_fwd(self.theta, 1).item())


def train_scalar(device, steps: int = 400, batch_size: int = 4096, lr: float = 3e-2, seed: int = 2604004805,
                 log=None, clouds: float = 0.0) -> LearnedScalar:
    """Train the one shared weight through the smoother on the same batches as ``train``."""
    first = make_batch(batch_size, seed, 0, device, clouds=clouds)
    _, sd = input_stats(first)
    L = LearnedScalar(device)
    for s in range(steps):
        b = first if s == 0 else make_batch(batch_size, seed, s, device, clouds=clouds)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
        loss = L.train_step(b, lr_s, sd)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"scalar step {s} loss {loss:.4f} log10 lambda {L.log10_lambda():.3f}")
    return L


def heldout_sse(z: torch.Tensor, batch: Batch, target: torch.Tensor | None = None) -> float:
    loss = torch.zeros(1, dtype=torch.float64, device=z.device)
    net.mse(z, batch.x_true if target is None else target, batch.hold, 1.0, loss=loss)
    return loss.item()


def train(device, steps: int = 400, batch_size: int = 4096, lr: float = 1e-3, seed: int = 2604004805,
          log=None, clouds: float = 0.0) -> Learned:
    """Train the network end to end through the smoother (Adam; cosine-decayed learning rate)."""
    first = make_batch(batch_size, seed, 0, device, clouds=clouds)
    mean, sd = input_stats(first)
    L = Learned(device, mean, sd)
    for s in range(steps):
        b = first if s == 0 else make_batch(batch_size, seed, s, device, clouds=clouds)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
        loss = L.train_step(b, lr_s)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"step {s} loss {loss:.4f} lr {lr_s:.2e}")
    return L


def evaluate(L: Learned, device, n_series: int = 262144, chunk: int = 65536, seed: int = 2604004806,
             Ls: LearnedScalar | None = None, clouds: float = 0.0):
    """Held-out RMSE (data units) and throughput of the learned and the plain forms on fresh series
    (and of the learned shared weight, if given)."""
    grid = torch.tensor(GRID, dtype=torch.float64, device=device)
    sse_l = sse_p = sse_s = 0.0
    cl_l = cl_p = cl_s = 0.0
    n = 0
    t_l = t_p = 0.0
    lam_dev = []
    for i, p0 in enumerate(range(0, n_series, chunk)):
        P = min(chunk, n_series - p0)
        b = make_batch(P, seed, i, device, clouds=clouds, S=S)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, lam = L.weights(b)
        z_l, _ = whs.whs_solve(b.x_train, b.w_train, lam, D, P)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lam_best, _, _ = whs.whs_gcv(b.x_train, b.w_train, grid, D, P)
        z_p, _ = whs.whs_solve(b.x_train, b.w_train, lam_best, D, P)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_l += t1 - t0
        t_p += t2 - t1
        sse_l += heldout_sse(z_l, b)
        sse_p += heldout_sse(z_p, b)
        if Ls is not None:
            z_s, _ = whs.whs_solve(b.x_train, b.w_train, Ls.weights(b), D, P)
            sse_s += heldout_sse(z_s, b)
        if b.x_clean is not None:
            cl_l += heldout_sse(z_l, b, b.x_clean)
            cl_p += heldout_sse(z_p, b, b.x_clean)
            if Ls is not None:
                cl_s += heldout_sse(z_s, b, b.x_clean)
        n += b.n_hold
        lam_dev.append(torch.log10(lam_best.double()).mean().item())
    out = {
        "n_series": n_series,
        "heldout_points": n,
        "rmse_learned": math.sqrt(sse_l / n),
        "rmse_plain_gcv": math.sqrt(sse_p / n),
        "gain": 1.0 - math.sqrt(sse_l / n) / math.sqrt(sse_p / n),
        "series_per_s_learned": n_series / t_l,
        "series_per_s_plain_gcv": n_series / t_p,
        "mean_log10_lambda_gcv": sum(lam_dev) / len(lam_dev),
    }
    if Ls is not None:
        out["rmse_learned_scalar"] = math.sqrt(sse_s / n)
        out["log10_lambda_learned_scalar"] = Ls.log10_lambda()
    if clouds > 0:
        # error against the noise-free signal at the held-out days (cloudy or not)
        out["clouds"] = clouds
        out["rmse_clean_learned"] = math.sqrt(cl_l / n)
        out["rmse_clean_plain_gcv"] = math.sqrt(cl_p / n)
        if Ls is not None:
            out["rmse_clean_learned_scalar"] = math.sqrt(cl_s / n)
    return out
