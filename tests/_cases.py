"""Seeded cases shared by the GPU parity tests: inputs from the generator
module, expected values from the CPU oracle only."""

from __future__ import annotations

import numpy as np
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import synth


def random_case(P, T, d, C=1, per_diff=True, seed=0, p_obs=0.3, lam_lo=0.0, lam_hi=4.0, dtype=torch.float64):
    """Natural-layout float64 numpy inputs, rounded through ``dtype`` (what the GPU sees)."""
    r = np.random.default_rng(seed)
    x = r.normal(size=(P, T, C)) * 0.1 + 0.3
    w = (r.random((P, T)) < p_obs).astype(np.uint8)
    w[:, ::max(T // (d + 2), 1)] = 1  # at least d+1 observations in every series
    if per_diff:
        lam = 10.0 ** r.uniform(lam_lo, lam_hi, size=(P, T - d))
    else:
        lam = 10.0 ** r.uniform(lam_lo, lam_hi, size=P)
    x = np.where(w[:, :, None] != 0, x, 0.0)
    x = torch.tensor(x).to(dtype).double().numpy()
    lam = torch.tensor(lam).to(dtype).double().numpy()
    return x, w, lam


def to_device(x, w, lam, S, dtype, device="cuda"):
    xt = synth.pack_series(torch.tensor(x, dtype=dtype), S).to(device)
    wt = synth.pack_rows(torch.tensor(w), S).to(device)
    lam = np.asarray(lam)
    if lam.ndim == 1:
        lt = torch.tensor(lam, dtype=dtype).to(device)
    else:
        lt = synth.pack_rows(torch.tensor(lam, dtype=dtype), S).to(device)
    return xt, wt, lt


def from_device_series(zt, P):
    return synth.unpack_series(zt.cpu(), P).double().numpy()


def from_device_rows(lt, P):
    if lt.dim() == 1:
        return lt.cpu().double().numpy()[:P]
    return synth.unpack_rows(lt.cpu(), P).double().numpy()


# Backward error assumed for an FP64 result that is not output in full (the
# adjoint's u = Omega^{-1} g is seen only through W u and (D u)(D z); the
# variance is a diagonal of Omega^{-1}): 1e-15, about five times what banded
# LDL^T reaches on these systems (the oracle's own solutions sit near 2e-16).
BETA_UNSEEN = 1e-15


def solve_bar(z, zref, x, w, lam, d, floor=1e-10, coef=None):
    """The FP64 parity bar of a solve, per series.  A series passes if its
    norm-wise error against the oracle is <= ``floor``; otherwise its error
    against the solution refined in extended precision must stay within twice
    what its own componentwise backward error allows (the exact Oettli-Prager
    bound ``beta |Omega^{-1}| (|Omega||z| + |Wx|)``): forward errors of any
    backward-stable FP64 solver grow with the conditioning of Omega, and two
    such solvers can share most of theirs, so neither 1e-10 nor their distance
    bounds a third.  Returns (failing rows, error, allowed)."""
    err = R.rel_err(z, zref)
    bad = np.nonzero(err > floor)[0]
    if bad.size == 0:
        return bad, err[bad], np.full(0, floor)
    b = np.where(np.asarray(w)[bad][:, :, None] != 0, np.asarray(x)[bad].reshape(bad.size, w.shape[1], -1), 0.0)
    lb = np.asarray(lam)[bad]
    zt = R.solve_band_refined(b, w[bad], lb, d, coef).astype(np.float64)
    et = R.rel_err(z[bad], zt)
    allow = np.maximum(floor, 2 * R.solution_error_bound(b, w[bad], lb, d, z[bad], coef))
    fail = et > allow
    return bad[fail], et[fail], allow[fail]


def adjoint_tol(g, w, lam, d, floor=1e-9, coef=None):
    """Per-series FP64 bar for the adjoint against the oracle's: ``floor``, or
    twice the Oettli-Prager bound of ``u = Omega^{-1} g`` for a backward error of
    ``BETA_UNSEEN`` on each of the two sides, whichever is larger."""
    g3 = g if g.ndim == 3 else g[:, :, None]
    u, _ = R.solve_band_rhs(g3, w, lam, d, coef)
    return np.maximum(floor, 2 * R.solution_error_bound(g3, w, lam, d, u, coef, beta=2 * BETA_UNSEEN))


def inverse_diag_tol(w, lam, d, floor=1e-9, coef=None):
    """Per-series FP64 bar for diag(Omega^{-1}) against the oracle's: ``floor``,
    or twice the first-order error bound of the diagonal under a componentwise
    perturbation of ``BETA_UNSEEN`` on each side, whichever is larger."""
    return np.maximum(floor, 2 * R.inverse_diag_error_bound(w, lam, d, 2 * BETA_UNSEEN, coef))


def assert_solution(z, zref, x, w, lam, d, f64: bool, info=None, coef=None):
    """``solve_bar`` at 1e-10 (FP64 storage) or 1e-4 (FP32 storage): that error
    against the oracle, or, on series so ill-conditioned that the FP64 oracle
    itself is farther than that from the exact solution, the bound the stored
    result's own backward error gives (its FP32 rounding included).  Always:
    componentwise backward error <= 1e-13 (FP64) / 1e-6 (FP32), which does not
    depend on the conditioning."""
    ok = np.ones(z.shape[0], bool) if info is None else (info == 0)
    err = R.rel_err(z[ok], zref[ok])
    if f64:
        fail, et, allow = solve_bar(z[ok], zref[ok], x[ok], w[ok], np.asarray(lam)[ok], d, 1e-10, coef)
        assert fail.size == 0, ("rows", fail, "err", et, "allowed", allow)
        be = R.backward_error(x[ok], w[ok], np.asarray(lam)[ok], d, z[ok], coef)
        assert be.max() <= 1e-13, be.max()
    else:
        fail, et, allow = solve_bar(z[ok], zref[ok], x[ok], w[ok], np.asarray(lam)[ok], d, 1e-4, coef)
        assert fail.size == 0, ("rows", fail, "err", et, "allowed", allow)
        be = R.backward_error(x[ok], w[ok], np.asarray(lam)[ok], d, z[ok], coef)
        assert be.max() <= 1e-6, be.max()
    return err


def backward_error_interleaved(x, w, lam, z, d, chunk_blocks=256):
    """Componentwise backward error ``max_t |Omega z - W x|_t / (|Omega||z| + |W x|)_t``
    of every series of an interleaved batch, on the tensors' own device in float64
    (plain torch elementwise operations from the definition, daily grid):
    ``Omega z = W z + D^T (lambda * (D z))``, and with lambda >= 0 every band entry of
    Omega is a sum of terms of one sign, so ``|Omega| = W + |D|^T Lambda |D|``.
    x, z: (nb, T, C, S); w: (nb, T, S) uint8; lam: (nb, T-d, S) or (P,).
    Returns float64 (nb*S,) on the host; padding slots of the last block read 0."""
    nb, T, C, S = x.shape
    c = torch.tensor(R.diff_coeffs(d), dtype=torch.float64, device=x.device)
    out = []
    for b0 in range(0, nb, chunk_blocks):
        sl = slice(b0, min(nb, b0 + chunk_blocks))
        xs = x[sl].double()
        zs = z[sl].double()
        ws = (w[sl] != 0).double()[:, :, None, :]
        if lam.dim() == 1:
            ln = lam.double()
            ln = torch.nn.functional.pad(ln, (0, nb * S - ln.numel()))
            ls = ln.view(nb, 1, 1, S)[sl].expand(-1, T - d, 1, S)
        else:
            ls = lam[sl].double()[:, :, None, :]
        b = ws * xs
        dz = sum(c[j] * zs[:, j:T - d + j] for j in range(d + 1))
        adz = sum(abs(c[j]) * zs[:, j:T - d + j].abs() for j in range(d + 1))
        v, av = ls * dz, ls * adz
        om_z = ws * zs
        aom_z = ws * zs.abs()
        for j in range(d + 1):
            om_z[:, j:T - d + j] += c[j] * v
            aom_z[:, j:T - d + j] += abs(c[j]) * av
        num = (om_z - b).abs()
        den = aom_z + b.abs()
        q = torch.where(den > 0, num / den, torch.zeros_like(num))
        out.append(q.amax(dim=(1, 2)).reshape(-1))
    return torch.cat(out).cpu().numpy()
