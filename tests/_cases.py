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


def lapack_spread(x, w, lam, d, zref, coef=None):
    """Norm-wise distance between the oracle and LAPACK's banded solver per series
    (how far two correct FP64 solvers already differ on this input)."""
    import scipy.linalg
    AB = R.omega_band(w, lam, d, coef)
    out = np.zeros(x.shape[0])
    for p in range(x.shape[0]):
        ref = scipy.linalg.solveh_banded(AB[p], np.where(w[p][:, None] != 0, x[p], 0.0), lower=True)
        out[p] = np.abs(ref - zref[p]).max() / max(np.abs(ref).max(), 1e-300)
    return out


def adjoint_spread(g, w, lam, d, coef=None):
    """Norm-wise distance per series between the oracle's u = Omega^{-1} g and
    LAPACK's banded solve of the same system."""
    import scipy.linalg
    g3 = g if g.ndim == 3 else g[:, :, None]
    u, _ = R.solve_band_rhs(g3, w, lam, d, coef)
    AB = R.omega_band(w, lam, d, coef)
    out = np.zeros(g3.shape[0])
    for p in range(g3.shape[0]):
        ref = scipy.linalg.solveh_banded(AB[p], g3[p], lower=True)
        out[p] = np.abs(ref - u[p]).max() / max(np.abs(ref).max(), 1e-300)
    return out


def inverse_diag_spread(w, lam, d, ref, coef=None):
    """Norm-wise distance per series between the oracle's diag(Omega^{-1}) and the
    diagonal of LAPACK's banded solve against the identity."""
    import scipy.linalg
    AB = R.omega_band(w, lam, d, coef)
    out = np.zeros(w.shape[0])
    for p in range(w.shape[0]):
        inv = scipy.linalg.solveh_banded(AB[p], np.eye(w.shape[1]), lower=True)
        dg = np.diagonal(inv)
        out[p] = np.abs(dg - ref[p]).max() / max(np.abs(dg).max(), 1e-300)
    return out


def spread_bar(err, spread, floor):
    """The FP64 parity bar: per series, err <= max(floor, 10 x the distance between
    two correct FP64 solvers on the same input).  Returns the failing rows."""
    allow = np.maximum(floor, 10 * spread)
    return np.nonzero(err > allow)[0], allow


def assert_solution(z, zref, x, w, lam, d, f64: bool, info=None, coef=None):
    """FP64: per-series error <= max(1e-10, 10 x LAPACK spread); FP32 storage:
    <= 1e-4.  Always: componentwise backward error <= 1e-13 (FP64) / 1e-6 (FP32),
    which does not depend on the conditioning."""
    ok = np.ones(z.shape[0], bool) if info is None else (info == 0)
    err = R.rel_err(z[ok], zref[ok])
    if f64:
        bad = err > 1e-10
        if bad.any():
            spread = lapack_spread(x[ok][bad], w[ok][bad], np.asarray(lam)[ok][bad], d, zref[ok][bad], coef)
            fail, allow = spread_bar(err[bad], spread, 1e-10)
            assert fail.size == 0, ("err", err[bad][fail], "allowed", allow[fail], "spread", spread[fail])
        be = R.backward_error(x[ok], w[ok], np.asarray(lam)[ok], d, z[ok], coef)
        assert be.max() <= 1e-13, be.max()
    else:
        assert err.max() <= 1e-4, err.max()
        be = R.backward_error(x[ok], w[ok], np.asarray(lam)[ok], d, z[ok], coef)
        assert be.max() <= 1e-6, be.max()
    return err
