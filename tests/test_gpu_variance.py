"""GPU parity of whs_variance (diagonal of Omega^{-1}, the posterior variance)
against the oracle's selected inverse.  FP64 storage: per-series max-norm
relative error <= max(1e-9, twice the first-order error of diag(Omega^{-1})
under componentwise perturbations of Omega of 1e-15 on each side).  FP32
storage: 1e-5 (both sides see the same FP32-rounded weights; the kernel's
arithmetic is FP64, only the stored result is rounded)."""

import numpy as np
import pytest
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import synth, whs
from tests._cases import inverse_diag_tol, random_case, to_device

pytestmark = pytest.mark.gpu


def _assert_close(var, ref, w, lam, d, f64):
    rel = np.abs(var - ref).max(axis=1) / np.abs(ref).max(axis=1)
    if not f64:
        assert rel.max() < 1e-5, rel.max()
        return
    bad = np.nonzero(rel > 1e-9)[0]
    if bad.size:
        allow = inverse_diag_tol(w[bad], np.asarray(lam)[bad], d)
        fail = rel[bad] > allow
        assert not fail.any(), ("rows", bad[fail], "err", rel[bad][fail], "allowed", allow[fail])


def _run(w, lam, d, P, dt):
    _, wt, lt = to_device(np.zeros(w.shape + (1,)), w, lam, 64, dt)
    var, info = whs.whs_variance(wt, lt, d, P)
    torch.cuda.synchronize()
    return synth.unpack_series(var.cpu(), P).double().numpy()[:, :, 0], info.cpu().numpy()


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("per_diff", [True, False])
@pytest.mark.parametrize("P,T,d", [(130, 200, 2), (64, 37, 1), (70, 101, 3), (65, 90, 4), (1, 17, 2)])
def test_variance_parity(P, T, d, per_diff, dt):
    _, w, lam = random_case(P, T, d, per_diff=per_diff, seed=3 * P + T + d, p_obs=0.25, dtype=dt)
    var, info = _run(w, lam, d, P, dt)
    ref, rinfo = R.posterior_variance(w, lam, d)
    np.testing.assert_array_equal(info, rinfo)
    _assert_close(var, ref, w, lam, d, dt == torch.float64)
    assert (var > 0).all()


def test_variance_failures_and_heavy_smoothing():
    P, T, d = 64, 80, 2
    _, w, lam = random_case(P, T, d, per_diff=True, seed=11)
    w[5] = 0
    w[5, 40] = 1                 # one observation: singular, info = T
    lam[9, 30] = -1e6            # a large negative weight: Omega is indefinite by a wide margin, so the
                                 # first failing pivot is not a rounding decision
    lam[12, :] = 1e8             # heavy smoothing: variance of the straight-line fit
    var, info = _run(w, lam, d, P, torch.float64)
    ref, rinfo = R.posterior_variance(w, lam, d)
    np.testing.assert_array_equal(info, rinfo)
    assert info[5] == T and info[9] > 0
    assert np.isnan(var[5]).all() and np.isnan(var[9]).all()
    ok = rinfo == 0
    _assert_close(var[ok], ref[ok], w[ok], lam[ok], d, True)
    assert abs((var[12] * w[12]).sum() - d) < 1e-3
