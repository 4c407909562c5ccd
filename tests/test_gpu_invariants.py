"""Invariants the paper's mathematics fixes, checked on the GPU path itself
(no oracle values involved), in the interleaved layout and in the contiguous
one (run on interleaved copies, and read in place by the partition kernel for
order <= 2 or the one-lane kernel otherwise): identity for lambda = 0 with every
sample observed (P1), exact reproduction of polynomials of degree < d (P2),
O(1/lambda) approach to the least-squares polynomial fit (P3), symmetry and
time reversal (P4), padding with unobserved samples (P5), linearity and
polynomial shift (P6), the DCT closed form of the first-order smoother (P7),
and for the adjoint the dot-product identity and grad_lambda = 0 on
low-degree data (P11).  FP64 storage; tolerances as in the oracle's own pins."""

import numpy as np
import pytest
import scipy.fft
import torch

from paper_2604_00048_amd import synth, whs
from tests._cases import from_device_rows, from_device_series, to_device

pytestmark = pytest.mark.gpu
# interleaved; series-contiguous run through the interleaved kernels on copies;
# series-contiguous read in place (partition kernel for one band of order <= 2)
LAYOUTS = [64, 1, "1-in-place"]


def _s(S):
    return 1 if S == "1-in-place" else S


def _st(S):
    return S != "1-in-place"


def solve(x, w, lam, d, S):
    x3 = x[:, :, None] if x.ndim == 2 else x
    xt, wt, lt = to_device(x3, w, lam, _s(S), torch.float64)
    z, info = whs.whs_solve(xt, wt, lt, d, x.shape[0], staged=_st(S))
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    z = from_device_series(z, x.shape[0])
    return z[:, :, 0] if x.ndim == 2 else z


def case(P, T, d, seed, p_obs=0.4, per_diff=True):
    r = np.random.default_rng(seed)
    w = (r.random((P, T)) < p_obs).astype(np.uint8)
    w[:, :d + 1] = 1
    lam = 10.0 ** r.uniform(0, 3, size=(P, T - d) if per_diff else P)
    return w, lam, r


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P1_identity(d, S):
    x = np.random.default_rng(d).normal(size=(5, 300))
    w = np.ones((5, 300), np.uint8)
    for lam in (np.zeros(5), np.zeros((5, 300 - d))):
        np.testing.assert_allclose(solve(x, w, lam, d, S), x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P2_polynomials_reproduced(d, S):
    T = 400
    w, lam, r = case(6, T, d, 10 + d, p_obs=0.3)
    t = np.arange(T) / T
    coef = r.normal(size=(6, d))
    p = sum(coef[:, j:j + 1] * t ** j for j in range(d))
    z = solve(np.where(w != 0, p, 0.0), w, lam, d, S)
    np.testing.assert_allclose(z, p, rtol=0, atol=1e-9 if d <= 3 else 1e-7)


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P3_heavy_smoothing_tends_to_polynomial_fit(d, S):
    T = 14
    r = np.random.default_rng(100 + d)
    x = r.normal(size=(1, T))
    w = (r.random((1, T)) < 0.6).astype(np.uint8)
    w[0, :d + 2] = 1
    t = np.arange(T, dtype=np.float64)
    obs = w[0] != 0
    fit = np.polyval(np.polyfit(t[obs], x[0, obs], d - 1), t)
    lam0 = 30.0 * (T / np.pi) ** (2 * d)
    errs = [np.abs(solve(np.where(w != 0, x, 0.0), w, np.array([lam]), d, S)[0] - fit).max()
            for lam in (lam0, 10 * lam0, 100 * lam0)]
    assert errs[2] < 1e-3 * np.abs(x).max()
    for a, b in zip(errs, errs[1:]):
        assert 7.0 < a / b < 14.0, errs


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P4_symmetry_and_time_reversal(d, S):
    T = 500
    w, lam, r = case(4, T, d, 20 + d)
    a, b = r.normal(size=(4, T)), r.normal(size=(4, T))
    za, zb = solve(a, w, lam, d, S), solve(b, w, lam, d, S)
    np.testing.assert_allclose((a * w * zb).sum(1), (b * w * za).sum(1), rtol=1e-10)
    zr = solve(a[:, ::-1].copy(), w[:, ::-1].copy(), lam[:, ::-1].copy(), d, S)
    np.testing.assert_allclose(zr[:, ::-1], za, rtol=0, atol=1e-10 * np.abs(za).max())


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P5_padding_with_unobserved_samples(d, S):
    # long unobserved tails make Omega ill-conditioned (the oracle itself moves by
    # 3e-6 at T = 350 with 90 padded days, d = 3); at T = 120 with 12 it moves by 1e-10
    T, pad = 120, 12
    w, lam, r = case(4, T, d, 30 + d, per_diff=False)
    x = np.where(w != 0, r.normal(size=(4, T)), 0.0)
    z = solve(x, w, lam, d, S)
    zp = solve(np.concatenate([x, np.zeros((4, pad))], 1), np.concatenate([w, np.zeros((4, pad), np.uint8)], 1),
               lam, d, S)
    np.testing.assert_allclose(zp[:, :T], z, rtol=0, atol=1e-8 * np.abs(z).max())


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P6_linearity_and_polynomial_shift(d, S):
    T = 450
    w, lam, r = case(3, T, d, 40 + d)
    a, b = r.normal(size=(3, T)), r.normal(size=(3, T))
    za, zb = solve(a, w, lam, d, S), solve(b, w, lam, d, S)
    zab = solve(2.5 * a - 0.75 * b, w, lam, d, S)
    np.testing.assert_allclose(zab, 2.5 * za - 0.75 * zb, rtol=0, atol=1e-10 * np.abs(zab).max())
    t = np.arange(T) / T
    poly = 0.3 + (1.7 * t if d >= 2 else 0.0)
    np.testing.assert_allclose(solve(a + poly, w, lam, d, S), za + poly, rtol=0, atol=1e-9)


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("lam", [0.5, 10.0, 1e3])
def test_P7_first_order_dct_closed_form(lam, S):
    T = 640
    x = np.random.default_rng(7).normal(size=(3, T))
    k = np.arange(T)
    filt = 1.0 / (1.0 + 4.0 * lam * np.sin(np.pi * k / (2 * T)) ** 2)
    ref = scipy.fft.idct(scipy.fft.dct(x, type=2, norm="ortho", axis=1) * filt, type=2, norm="ortho", axis=1)
    z = solve(x, np.ones((3, T), np.uint8), np.full(3, lam), 1, S)
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("S", LAYOUTS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_P11_adjoint_dot_product_and_low_degree_gradient(d, S):
    T, P = 420, 4
    w, lam, r = case(P, T, d, 50 + d)
    x = np.where(w != 0, r.normal(size=(P, T)), 0.0)
    a = np.where(w != 0, r.normal(size=(P, T)), 0.0)     # a perturbation of x
    g = r.normal(size=(P, T))
    xt, wt, lt = to_device(x[:, :, None], w, lam, _s(S), torch.float64)
    z, _ = whs.whs_solve(xt, wt, lt, d, P, staged=_st(S))
    gt = synth.pack_series(torch.tensor(g[:, :, None]), _s(S)).cuda()
    gx, gl, _ = whs.whs_backward(wt, lt, z, gt, d, P, staged=_st(S))
    gx = from_device_series(gx, P)[:, :, 0]
    # <g, dz/dx a> = <grad_x, a>, with dz/dx a the smoother applied to a
    za = solve(a, w, lam, d, S)
    np.testing.assert_allclose((g * za).sum(1), (gx * a).sum(1), rtol=1e-10)
    # data that D annihilates: z = x is a polynomial of degree < d, D z = 0, grad_lambda = 0
    t = np.arange(T) / T
    poly = np.where(w != 0, (0.2 + 0.5 * t) if d >= 2 else 0.2 + 0 * t, 0.0)
    xp, wp, lp = to_device(poly[:, :, None], w, lam, _s(S), torch.float64)
    zp, _ = whs.whs_solve(xp, wp, lp, d, P, staged=_st(S))
    _, glp, _ = whs.whs_backward(wp, lp, zp, gt, d, P, staged=_st(S))
    glp = from_device_rows(glp, P)
    gl = from_device_rows(gl, P)
    assert np.abs(glp).max() <= 1e-8 * np.abs(gl).max()
