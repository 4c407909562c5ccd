"""Seeded synthetic inputs shaped like the paper's Sentinel-2 workloads.

This module holds no arithmetic of the smoother itself: it draws series,
observation masks and smoothing weights, and converts between the natural
layout ``(P, T, C)`` and the interleaved layout the library reads.  Both the
GPU path and the CPU reference are fed from it.

Recipe (each choice is one reading of the workload description):

* phenology: a double logistic per year,
  ``x(t) = base + a_y [s(r_g (tau - g)) - s(r_s (tau - s_d))]`` with ``s`` the
  logistic function and ``tau`` the 0-based day of year of day ``t``
  (``T = 3288`` is 2016-01-01 .. 2024-12-31, leap years included; a single
  year uses ``tau = t``); ``base ~ U[0.05, 0.2]``, ``a ~ U[0.2, 0.8]``,
  ``g ~ U[80, 140]``, ``s_d ~ U[230, 300]``, ``r_g, r_s ~ U[0.03, 0.1]``;
  ``a_y = a * U[0.9, 1.1]`` per year (multi-year series);
* bands share the phenology dates, slopes and mask; base, amplitude and noise
  are drawn per band;
* noise ``N(0, 0.02^2)``; ``w_t ~ Bernoulli(p)``; ``x_t = 0`` where ``w_t = 0``;
* scalar weights are log-uniform; the per-difference field is a stationary
  Gaussian process in ``log10`` (squared-exponential kernel, length scale 60
  days, mean 2, sd 0.5) sampled as white noise convolved with a Gaussian of
  sd ``60/sqrt(2)`` days truncated at 4 sd, then 2 % of the entries lowered
  by 3 (abrupt single-day changes); a field over days maps to difference row
  ``k`` at day ``k + d // 2``.

Every draw comes from a ``torch.Generator`` seeded from ``(seed, chunk)``, so
chunked generation on one device is reproducible.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import torch

SEED_BASE = 2604004800


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFF_FFFF_FFFF_FFFF)
    return g


def _u(gen, shape, lo, hi, device, dtype=torch.float64):
    return lo + (hi - lo) * torch.rand(shape, generator=gen, device=device, dtype=dtype)


def day_of_year(T: int, start_year: int = 2016, single_year: bool = False):
    """``(tau, year_index)`` for ``T`` consecutive days from 1 January ``start_year``."""
    if single_year:
        t = torch.arange(T, dtype=torch.float64)
        return t, torch.zeros(T, dtype=torch.long)
    tau = []
    yr = []
    y = start_year
    while len(tau) < T:
        n = 366 if (y % 4 == 0 and (y % 100 != 0 or y % 400 == 0)) else 365
        tau.extend(range(n))
        yr.extend([y - start_year] * n)
        y += 1
    return (torch.tensor(tau[:T], dtype=torch.float64), torch.tensor(yr[:T], dtype=torch.long))


def phenology(P: int, T: int, C: int, gen, device, single_year: bool = False,
              noise_sd: float = 0.02):
    """Noisy double-logistic reflectance ``(P, T, C)`` in float64 and the clean signal."""
    tau, yr = day_of_year(T, single_year=single_year)
    tau = tau.to(device)
    yr = yr.to(device)
    ny = int(yr.max().item()) + 1
    g = _u(gen, (P, 1, 1), 80.0, 140.0, device)
    s = _u(gen, (P, 1, 1), 230.0, 300.0, device)
    rg = _u(gen, (P, 1, 1), 0.03, 0.1, device)
    rs = _u(gen, (P, 1, 1), 0.03, 0.1, device)
    base = _u(gen, (P, 1, C), 0.05, 0.2, device)
    amp = _u(gen, (P, 1, C), 0.2, 0.8, device)
    if single_year:
        jit = torch.ones((P, 1, C), dtype=torch.float64, device=device)
        amp_t = amp.expand(P, T, C)
    else:
        jit = _u(gen, (P, ny, C), 0.9, 1.1, device)
        amp_t = (amp * jit)[:, yr, :]
    tt = tau.view(1, T, 1)
    clean = base + amp_t * (torch.sigmoid(rg * (tt - g)) - torch.sigmoid(rs * (tt - s)))
    noisy = clean + noise_sd * torch.randn((P, T, C), generator=gen, device=device, dtype=torch.float64)
    return noisy, clean


def bernoulli_mask(P: int, T: int, p, gen, device) -> torch.Tensor:
    """0/1 observation mask ``(P, T)`` as uint8; ``p`` scalar or ``(P,)``."""
    if not torch.is_tensor(p):
        p = torch.full((P, 1), float(p), dtype=torch.float64, device=device)
    else:
        p = p.view(P, 1).to(device=device, dtype=torch.float64)
    r = torch.rand((P, T), generator=gen, device=device, dtype=torch.float64)
    return (r < p).to(torch.uint8)


def log_uniform(shape, lo: float, hi: float, gen, device) -> torch.Tensor:
    return 10.0 ** _u(gen, shape, math.log10(lo), math.log10(hi), device)


def gp_log10_field(P: int, n: int, gen, device, mean=2.0, sd=0.5, ell=60.0,
                   drop_p=0.02, drop=3.0) -> torch.Tensor:
    """Per-day ``log10`` weights ``(P, n)``: squared-exponential GP plus sparse drops."""
    ks = ell / math.sqrt(2.0)
    half = int(math.ceil(4.0 * ks))
    tk = torch.arange(-half, half + 1, dtype=torch.float64, device=device)
    ker = torch.exp(-0.5 * (tk / ks) ** 2)
    ker = ker / torch.sqrt((ker ** 2).sum())  # unit-variance output
    wn = torch.randn((P, n + 2 * half), generator=gen, device=device, dtype=torch.float64)
    # valid cross-correlation f[i] = sum_j ker[j] wn[i + j], by one batched FFT
    L = 1 << int(math.ceil(math.log2(n + 4 * half + 1)))
    spec = torch.fft.rfft(wn, L) * torch.conj(torch.fft.rfft(ker, L))
    f = torch.fft.irfft(spec, L)[:, :n]
    f = mean + sd * f
    hit = torch.rand((P, n), generator=gen, device=device, dtype=torch.float64) < drop_p
    return f - drop * hit.to(torch.float64)


# ---------------------------------------------------------------------------
# layout
# ---------------------------------------------------------------------------


def n_blocks(P: int, S: int) -> int:
    return (P + S - 1) // S


def pack_series(x: torch.Tensor, S: int) -> torch.Tensor:
    """``(P, T, C)`` -> interleaved ``[P/S][T][C][S]`` (zero-padded tail)."""
    P, T, C = x.shape
    nb = n_blocks(P, S)
    if nb * S != P:
        pad = torch.zeros((nb * S - P, T, C), dtype=x.dtype, device=x.device)
        x = torch.cat([x, pad], 0)
    return x.view(nb, S, T, C).permute(0, 2, 3, 1).contiguous()


def unpack_series(xi: torch.Tensor, P: int) -> torch.Tensor:
    """Interleaved ``[P/S][T][C][S]`` -> ``(P, T, C)``."""
    nb, T, C, S = xi.shape
    return xi.permute(0, 3, 1, 2).reshape(nb * S, T, C)[:P]


def pack_rows(v: torch.Tensor, S: int) -> torch.Tensor:
    """``(P, n)`` -> interleaved ``[P/S][n][S]`` (mask, per-row weights)."""
    P, n = v.shape
    nb = n_blocks(P, S)
    if nb * S != P:
        pad = torch.zeros((nb * S - P, n), dtype=v.dtype, device=v.device)
        v = torch.cat([v, pad], 0)
    return v.view(nb, S, n).permute(0, 2, 1).contiguous()


def unpack_rows(vi: torch.Tensor, P: int) -> torch.Tensor:
    nb, n, S = vi.shape
    return vi.permute(0, 2, 1).reshape(nb * S, n)[:P]


def pack_bits(wi: torch.Tensor) -> torch.Tensor:
    """Interleaved 0/1 weights ``[nb][T][S]`` (uint8) -> eight per byte,
    ``[nb][T][S/8]``: bit ``s % 8`` of byte ``s / 8`` of each row."""
    nb, T, S = wi.shape
    if S % 8:
        raise ValueError("the interleave must be a multiple of 8")
    b = (wi != 0).to(torch.uint8).view(nb, T, S // 8, 8)
    shifts = torch.arange(8, dtype=torch.uint8, device=wi.device)
    return (b << shifts).sum(dim=3, dtype=torch.int32).to(torch.uint8)


def unpack_bits(wb: torch.Tensor) -> torch.Tensor:
    """Inverse of ``pack_bits``: ``[nb][T][S/8]`` -> ``[nb][T][S]`` (0/1 uint8)."""
    nb, T, S8 = wb.shape
    shifts = torch.arange(8, dtype=torch.uint8, device=wb.device)
    return ((wb.unsqueeze(3) >> shifts) & 1).reshape(nb, T, S8 * 8)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------


@dataclass
class Batch:
    """One workload in natural layout: ``x (P,T,C)``, ``w (P,T)`` uint8,
    ``lam`` ``(P,)`` or ``(P, T-d)``, all on ``device``; ``clean`` the noise-free signal."""
    x: torch.Tensor
    w: torch.Tensor
    lam: torch.Tensor
    d: int
    clean: torch.Tensor | None = None

    @property
    def P(self):
        return self.x.shape[0]

    @property
    def T(self):
        return self.x.shape[1]

    @property
    def C(self):
        return self.x.shape[2]


def _finish(x, w):
    return torch.where(w[:, :, None] != 0, x, torch.zeros((), dtype=x.dtype, device=x.device))


def small_homoscedastic(P=64, T=365, d=2, seed=SEED_BASE + 1, device="cpu", p_obs=0.2,
                        lam_lo=1.0, lam_hi=1e4, C=1) -> Batch:
    """Single-year daily series, Bernoulli(0.2) mask, scalar log-uniform weight."""
    gen = _gen(seed, device)
    x, clean = phenology(P, T, C, gen, device, single_year=True)
    w = bernoulli_mask(P, T, p_obs, gen, device)
    lam = log_uniform((P,), lam_lo, lam_hi, gen, device)
    return Batch(_finish(x, w), w, lam, d, clean)


def multiband_homoscedastic(P, T=3288, C=10, d=2, seed=SEED_BASE + 2, device="cpu", chunk=0,
                            p_obs=0.08, lam_lo=1.0, lam_hi=1e4) -> Batch:
    """Nine years daily, ``C`` bands sharing one mask, scalar log-uniform weight."""
    gen = _gen(seed * 1_000_003 + chunk, device)
    x, clean = phenology(P, T, C, gen, device)
    w = bernoulli_mask(P, T, p_obs, gen, device)
    lam = log_uniform((P,), lam_lo, lam_hi, gen, device)
    return Batch(_finish(x, w), w, lam, d, clean)


def heteroscedastic(P, T=3288, d=2, seed=SEED_BASE + 3, device="cpu", chunk=0, p_obs=0.08) -> Batch:
    """Nine years daily, one band, per-difference weights from the GP field."""
    gen = _gen(seed * 1_000_003 + chunk, device)
    x, clean = phenology(P, T, 1, gen, device)
    w = bernoulli_mask(P, T, p_obs, gen, device)
    field = gp_log10_field(P, T, gen, device)
    lo = d // 2
    lam = 10.0 ** field[:, lo:lo + T - d]
    return Batch(_finish(x, w), w, lam, d, clean)


def uneven_groups(n_series=100_000, seed=SEED_BASE + 4, lengths=(365, 730, 1461, 3288),
                  orders=(1, 2, 3), device="cpu", lam_lo=0.1, lam_hi=1e5):
    """Uneven batch: lengths and orders drawn uniformly per series, grouped by ``(T, d)``.

    Returns a list of ``((T, d), Batch)`` in draw order of the groups
    (lengths ascending, orders ascending); every series has its own
    ``p ~ U[0.05, 0.3]``.
    """
    gen = _gen(seed, device)
    li = torch.randint(0, len(lengths), (n_series,), generator=gen, device=device)
    oi = torch.randint(0, len(orders), (n_series,), generator=gen, device=device)
    groups = []
    for a, T in enumerate(lengths):
        for b, d in enumerate(orders):
            n = int(((li == a) & (oi == b)).sum().item())
            if n == 0:
                continue
            g2 = _gen(seed * 7919 + a * 31 + b, device)
            x, clean = phenology(n, 3288, 1, g2, device)
            x = x[:, :T].contiguous()
            clean = clean[:, :T].contiguous()
            p = _u(g2, (n,), 0.05, 0.3, device)
            w = bernoulli_mask(n, T, p, g2, device)
            lam = log_uniform((n,), lam_lo, lam_hi, g2, device)
            groups.append(((T, d), Batch(_finish(x, w), w, lam, d, clean)))
    return groups


def acquisition_days(T: int, gen, device, revisit: int = 5, n_days: int = 3288) -> torch.Tensor:
    """``T`` distinct acquisition days (float64, ascending) drawn from a nominal
    ``revisit``-day pass calendar over ``n_days`` days: the dates one patch of
    pixels shares (the paper's series have median length 280 over about nine
    years, Sec. IV-A)."""
    passes = n_days // revisit
    if not 1 <= T <= passes:
        raise ValueError(f"T must be in [1, {passes}]")
    r = torch.rand(passes, generator=gen, device=device, dtype=torch.float64)
    pick = torch.sort(torch.argsort(r)[:T]).values
    return (pick * revisit + 1).to(torch.float64)


def irregular_sits(P: int, T: int, C: int, seed: int, device, chunk: int = 0, p_valid=(0.3, 0.8), days=None):
    """Irregular multi-band series: ``P`` pixels sharing ``T`` acquisition days,
    double-logistic bands sampled at those days with N(0, 0.02) noise, and a
    per-pixel validity mask ``w ~ Bernoulli(p)``, ``p ~ U[p_valid]`` (the
    masks a cloud detector provides).  Returns ``(days, Batch)``, the batch in
    natural layout with ``x`` zero where ``w`` is 0.  ``days``: the acquisition
    days to use (ascending, within the 3288-day span) instead of drawing them,
    so that chunks of one batch share their dates."""
    gen = _gen(seed * 1_000_003 + chunk, device)
    if days is None:
        days = acquisition_days(T, gen, device)
    elif days.numel() != T:
        raise ValueError(f"days must hold T={T} values")
    x_day, clean_day = phenology(P, 3288, C, gen, device)
    idx = days.long()
    x = x_day[:, idx, :].contiguous()
    clean = clean_day[:, idx, :].contiguous()
    del x_day, clean_day
    pv = _u(gen, (P,), p_valid[0], p_valid[1], device)
    w = bernoulli_mask(P, T, pv, gen, device)
    return days, Batch(_finish(x, w), w, None, 2, clean)


def cloud_contaminate(x: torch.Tensor, w: torch.Tensor, frac: float, gen):
    """Cloud-contaminated acquisitions kept as observed (their mask withheld):
    each observed sample is cloudy with probability ``frac``; a cloudy value is
    pulled towards a low cloud value, ``x (1 - a) + a c`` with opacity
    ``a ~ U[0.5, 1]`` and ``c ~ U[-0.05, 0.1]`` (a vegetation index drops
    under clouds).  ``x (P, T, C)``; returns ``(x_observed, cloudy (P, T) uint8)``."""
    P, T, C = x.shape
    dev = x.device
    cloudy = ((torch.rand((P, T), generator=gen, device=dev, dtype=torch.float64) < frac) & (w != 0))
    a = _u(gen, (P, T, 1), 0.5, 1.0, dev).to(x.dtype)
    c = _u(gen, (P, T, 1), -0.05, 0.1, dev).to(x.dtype)
    xo = torch.where(cloudy[:, :, None], x * (1 - a) + a * c, x)
    return xo, cloudy.to(torch.uint8)


def holdout_split(w: torch.Tensor, frac: float, gen) -> torch.Tensor:
    """Each observed point is held out independently with probability ``frac``
    (one uniform draw per point, no sort); returns the held-out mask (uint8), a
    subset of ``w``."""
    r = torch.rand(w.shape, generator=gen, device=w.device, dtype=torch.float64)
    return ((r < frac) & (w != 0)).to(torch.uint8)


# ---------------------------------------------------------------------------
# full-size workloads, generated chunk by chunk straight into the interleaved layout
# ---------------------------------------------------------------------------


@dataclass
class Packed:
    """A workload in the interleaved layout: ``x (nb,T,C,S)``, ``w (nb,T,S)``,
    ``lam`` ``(P,)`` or ``(nb,T-d,S)``."""
    x: torch.Tensor
    w: torch.Tensor
    lam: torch.Tensor
    d: int
    P: int
    S: int

    @property
    def T(self):
        return self.x.shape[1]

    @property
    def C(self):
        return self.x.shape[2]

    def series(self, idx) -> "Batch":
        """Natural-layout copy (float64, on the CPU) of the series in ``idx``."""
        idx = torch.as_tensor(idx, dtype=torch.long)
        b, s = idx // self.S, idx % self.S
        x = self.x[b.to(self.x.device), :, :, s.to(self.x.device)].to("cpu", torch.float64)
        w = self.w[b.to(self.w.device), :, s.to(self.w.device)].to("cpu")
        if self.lam.dim() == 1:
            lam = self.lam[idx.to(self.lam.device)].to("cpu", torch.float64)
        else:
            lam = self.lam[b.to(self.lam.device), :, s.to(self.lam.device)].to("cpu", torch.float64)
        return Batch(x, w, lam, self.d)


def generate_packed(kind: str, P: int, S: int = 64, dtype=torch.float32, device="cpu", chunk: int = 8192,
                    **kw) -> Packed:
    """Generate ``kind`` in ``{"multiband", "heteroscedastic"}`` chunk by chunk.

    Chunk ``i`` covers series ``[i*chunk, (i+1)*chunk)`` and is drawn from its
    own generator, so the result depends on ``chunk`` (a multiple of ``S``).
    """
    assert chunk % S == 0
    maker = {"multiband": multiband_homoscedastic, "heteroscedastic": heteroscedastic}[kind]
    nb = n_blocks(P, S)
    first = maker(min(chunk, P), device=device, chunk=0, **kw)
    T, C, d = first.T, first.C, first.d
    x = torch.zeros((nb, T, C, S), dtype=dtype, device=device)
    w = torch.zeros((nb, T, S), dtype=torch.uint8, device=device)
    per_diff = first.lam.dim() == 2
    lam = torch.zeros((nb, T - d, S) if per_diff else (P,), dtype=dtype, device=device)
    for i, p0 in enumerate(range(0, P, chunk)):
        n = min(chunk, P - p0)
        bt = first if i == 0 else maker(n, device=device, chunk=i, **kw)
        b0, b1 = p0 // S, n_blocks(p0 + n, S)
        x[b0:b1] = pack_series(bt.x.to(dtype), S)
        w[b0:b1] = pack_rows(bt.w, S)
        if per_diff:
            lam[b0:b1] = pack_rows(bt.lam.to(dtype), S)
        else:
            lam[p0:p0 + n] = bt.lam.to(dtype)
        del bt
    return Packed(x, w, lam, d, P, S)


def pack_groups(groups, S: int = 64, dtype=torch.float32, device="cpu"):
    """Pack ``[((T, d), Batch), ...]`` into flat interleaved buffers.

    Returns ``(x, w, lam, descs)``: 1-D tensors holding every group's
    interleaved blocks back to back, and one descriptor dict per group with
    the element offsets ``x_off, w_off, lam_off, info_off`` (scalar weights:
    one per series, concatenated).
    """
    xs, ws, ls, descs = [], [], [], []
    xo = wo = lo = io = 0
    for (T, d), b in groups:
        xi = pack_series(b.x.to(dtype), S).reshape(-1)
        wi = pack_rows(b.w, S).reshape(-1)
        if b.lam.dim() == 2:
            li = pack_rows(b.lam.to(dtype), S).reshape(-1)
        else:
            li = b.lam.to(dtype).reshape(-1)
        descs.append({"n_series": b.P, "T": T, "d": d, "x_off": xo, "w_off": wo, "lam_off": lo, "info_off": io})
        xs.append(xi)
        ws.append(wi)
        ls.append(li)
        xo += xi.numel()
        wo += wi.numel()
        lo += li.numel()
        io += b.P
    return (torch.cat(xs).to(device), torch.cat(ws).to(device), torch.cat(ls).to(device), descs)


def unpack_group(buf: torch.Tensor, desc: dict, C: int = 1, S: int = 64) -> torch.Tensor:
    """Natural-layout ``(n, T, C)`` view of one group inside a flat buffer from ``pack_groups``."""
    n, T = desc["n_series"], desc["T"]
    nb = n_blocks(n, S)
    blk = buf[desc["x_off"]:desc["x_off"] + nb * T * C * S].view(nb, T, C, S)
    return unpack_series(blk, n)
