"""GPU parity of whs_solve / whs_factor / whs_backward against the FP64 oracle.

Every call goes through the C-ABI (ctypes binding); expected values come
from ``oracle/`` on the same seeded inputs.  Sizes span several tiles and a
ragged tail in both time and series.
"""

import numpy as np
import pytest
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import synth, whs
from tests._cases import adjoint_tol, assert_solution, from_device_rows, from_device_series, random_case, to_device

pytestmark = pytest.mark.gpu

DT = {"f32": torch.float32, "f64": torch.float64}


def _run_solve(x, w, lam, d, S, dtype):
    P = x.shape[0]
    xt, wt, lt = to_device(x, w, lam, S, dtype)
    z, info = whs.whs_solve(xt, wt, lt, d, P)
    torch.cuda.synchronize()
    return from_device_series(z, P), info.cpu().numpy()


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_small_homoscedastic_year(dt):
    """64 series, T = 365, d = 2, scalar weight, Bernoulli(0.2) mask."""
    b = synth.small_homoscedastic()
    dtype = DT[dt]
    x = b.x.to(dtype).double().numpy()
    w = b.w.numpy()
    lam = b.lam.to(dtype).double().numpy()
    z, info = _run_solve(x, w, lam, 2, 64, dtype)
    zref, iref = R.solve_band(x, w, lam, 2)
    np.testing.assert_array_equal(info, iref)
    err = assert_solution(z, zref, x, w, lam, 2, dt == "f64")
    print(f"[small year {dt}] max rel err {err.max():.3e}", flush=True)


CASES = [
    # P,   T,   d, C,  S,  per_diff
    (100, 101, 1, 1, 64, True),
    (130, 77, 2, 1, 32, True),
    (70, 53, 3, 1, 64, False),
    (64, 45, 4, 1, 64, True),
    (65, 200, 2, 3, 64, False),    # one 3-band group (16-step tiles in FP32)
    (40, 120, 2, 10, 64, True),    # solve groups 5 + 5, adjoint 3 + 3 + 3 + 1
    (33, 60, 3, 13, 16, True),     # generic groups of 2 and 1
    (5, 3, 2, 1, 64, True),        # T = d + 1
    (9, 7, 1, 2, 4, False),        # one partial tile
    (3, 16, 2, 1, 1, True),        # S = 1, exactly one tile
    (70, 150, 1, 3, 64, False),    # order 1, one 3-band group, ragged last tile
    (66, 90, 2, 2, 64, True),      # a 2-band group with a weight per difference row
    (64, 37, 1, 5, 64, False),     # solve groups 3 + 2 in FP32, 5 in FP64
]

# band groupings that depend on storage type and weight kind (the widest
# spill-free group of each variant)
GROUP_CASES = [
    (64, 50, 2, 3, 64, False),     # adjoint 2 + 1 in FP64, 3 in FP32
    (64, 80, 3, 5, 64, False),     # adjoint 2 + 2 + 1
    (64, 80, 3, 5, 64, True),      # adjoint 3 + 2 in FP32, 2 + 2 + 1 in FP64
    (64, 60, 4, 4, 64, False),     # adjoint one band at a time; solve 3 + 1
    (64, 60, 4, 4, 64, True),      # adjoint 3 + 1 in FP32, 2 + 2 in FP64
]


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("P,T,d,C,S,per_diff", CASES + GROUP_CASES)
def test_solve_parity(P, T, d, C, S, per_diff, dt):
    dtype = DT[dt]
    x, w, lam = random_case(P, T, d, C=C, per_diff=per_diff, seed=P * 7 + T, dtype=dtype,
                            lam_hi=3.0 if d >= 3 else 4.0)
    z, info = _run_solve(x, w, lam, d, S, dtype)
    zref, iref = R.solve_band(x, w, lam, d)
    np.testing.assert_array_equal(info, iref)
    assert_solution(z, zref, x, w, lam, d, dt == "f64")


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("P,T,d,C,S,per_diff", CASES[:7] + GROUP_CASES)
def test_backward_parity(P, T, d, C, S, per_diff, dt):
    dtype = DT[dt]
    x, w, lam = random_case(P, T, d, C=C, per_diff=per_diff, seed=P * 11 + T, dtype=dtype,
                            lam_hi=3.0 if d >= 3 else 4.0)
    g = np.random.default_rng(P + T).normal(size=x.shape)
    g = torch.tensor(g).to(dtype).double().numpy()
    xt, wt, lt = to_device(x, w, lam, S, dtype)
    z, info = whs.whs_solve(xt, wt, lt, d, P)
    gt = synth.pack_series(torch.tensor(g, dtype=dtype), S).cuda()
    gx, gl, info2 = whs.whs_backward(wt, lt, z, gt, d, P)
    torch.cuda.synchronize()
    zc = from_device_series(z, P)
    gx = from_device_series(gx, P)
    gl = from_device_rows(gl, P)
    # the oracle adjoint at the same (stored) z
    gx_ref, gl_ref, iref = R.vjp(x, w, lam, d, g, z=zc)
    np.testing.assert_array_equal(info2.cpu().numpy(), iref)
    # FP64: 1e-9, or twice the Oettli-Prager bound of u = Omega^{-1} g where the
    # series is conditioned so that the FP64 oracle itself may be farther off
    tol = adjoint_tol(g, w, lam, d) if dt == "f64" else np.full(P, 1e-4)
    ex = np.abs(gx - gx_ref).max(axis=(1, 2)) / np.abs(gx_ref).max(axis=(1, 2))
    assert (ex <= tol).all(), (ex.max(), ex[ex > tol], tol[ex > tol])
    if gl.ndim == 1:
        el = np.abs(gl - gl_ref) / np.maximum(np.abs(gl_ref), 1e-300)
    else:
        el = np.abs(gl - gl_ref).max(1) / np.abs(gl_ref).max(1)
    assert (el <= tol * 10).all(), (el.max(), el[el > tol * 10])
    assert (gx[w == 0] == 0).all()


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("per_diff", [True, False])
def test_factor_is_the_cholesky_band(d, per_diff):
    P, T, S = 70, 90, 64
    x, w, lam = random_case(P, T, d, per_diff=per_diff, seed=d, lam_hi=3.0)
    _, wt, lt = to_device(x, w, lam, S, torch.float64)
    F, info = whs.whs_factor(wt, lt, d, P)
    torch.cuda.synchronize()
    Fn = F.permute(0, 3, 1, 2).reshape(-1, d + 1, T)[:P].cpu().numpy()
    Lb, iref = R.cholesky_band(R.omega_band(w, lam, d), w)
    np.testing.assert_array_equal(info.cpu().numpy(), iref)
    err = np.abs(Fn - Lb).max(axis=(1, 2)) / np.abs(Lb).max(axis=(1, 2))
    # condition-aware: LAPACK's banded Cholesky is a second FP64 opinion
    import scipy.linalg
    AB = R.omega_band(w, lam, d)
    spread = np.array([np.abs(scipy.linalg.cholesky_banded(AB[p], lower=True) - Lb[p]).max() / np.abs(Lb[p]).max()
                       for p in range(P)])
    assert (err <= np.maximum(1e-11, 10 * spread)).all(), (err.max(), spread.max())
    for i in range(1, d + 1):
        assert (Fn[:, i, T - i:] == 0).all()
    # solving with the exported factor reproduces the fused solve
    xt = synth.pack_series(torch.tensor(x), S).cuda()
    z1, _ = whs.whs_solve(xt, wt, lt, d, P)
    z2, i2 = whs.whs_solve(xt, wt, None, d, P, factor=F)
    torch.cuda.synchronize()
    a, b = from_device_series(z1, P), from_device_series(z2, P)
    assert (R.rel_err(a, b) < 1e-11).all()
    # and the adjoint with the exported factor matches the fused adjoint
    g = torch.randn(xt.shape, generator=torch.Generator(device="cuda").manual_seed(11), device="cuda",
                    dtype=xt.dtype)
    gx1, gl1, _ = whs.whs_backward(wt, lt, z1, g, d, P)
    gx2, gl2, _ = whs.whs_backward(wt, lt, z1, g, d, P, factor=F)
    torch.cuda.synchronize()
    # compare the P real series only (padding slots of the last block are never written)
    np.testing.assert_allclose(from_device_series(gx2, P), from_device_series(gx1, P), rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(from_device_rows(gl2, P), from_device_rows(gl1, P), rtol=1e-8, atol=1e-12)


def test_failures_and_ignored_unobserved_values():
    P, T, d, S = 6, 40, 2, 64
    x, w, lam = random_case(P, T, d, per_diff=True, seed=3)
    w[0] = 0
    w[0, 7] = 1               # one observation < d
    w[1] = 0                  # none
    lam[2, 10] = -1e3         # indefinite
    lam[3, 5] = np.nan        # NaN weight
    x_nan = np.where(w[:, :, None] != 0, x, np.nan)  # NaN where unobserved: must be ignored
    z, info = _run_solve(x_nan, w, lam, d, S, torch.float64)
    _, iref = R.solve_band(x, w, lam, d)
    assert (info[:4] > 0).all() and (info[4:] == 0).all()
    assert info[2] == iref[2] and info[3] == iref[3]
    assert np.isnan(z[:4]).all()
    zref, _ = R.solve_band(x, w, lam, d)
    assert np.isfinite(z[4:]).all()
    assert (R.rel_err(z[4:], zref[4:]) < 1e-10).all()


@pytest.mark.parametrize("S", [64, 1])
def test_long_series(S):
    # 200,000 steps: 8,334 tiles of checkpoints per series, one full block of 64
    # series and a ragged one; the contiguous layout goes through the interleaved copies
    P, T, d = 65, 200_000, 2
    x, w, lam = random_case(P, T, d, per_diff=True, seed=200 + S, dtype=torch.float32)
    xt, wt, lt = to_device(x, w, lam, S, torch.float32)
    z, info = whs.whs_solve(xt, wt, lt, d, P)
    g = torch.tensor(np.random.default_rng(S).normal(size=x.shape), dtype=torch.float32)
    gx, gl, info2 = whs.whs_backward(wt, lt, z, synth.pack_series(g, S).cuda(), d, P)
    torch.cuda.synchronize()
    zc = from_device_series(z, P)
    zref, iref = R.solve_band(x, w, lam, d)
    np.testing.assert_array_equal(info.cpu().numpy(), iref)
    np.testing.assert_array_equal(info2.cpu().numpy(), iref)
    assert_solution(zc, zref, x, w, lam, d, False)
    gx_ref, gl_ref, _ = R.vjp(x, w, lam, d, g.double().numpy(), z=zc)
    ex = np.abs(from_device_series(gx, P) - gx_ref).max(axis=(1, 2)) / np.abs(gx_ref).max(axis=(1, 2))
    el = np.abs(from_device_rows(gl, P) - gl_ref).max(1) / np.abs(gl_ref).max(1)
    assert ex.max() <= 1e-4, ex.max()
    assert el.max() <= 1e-3, el.max()


def test_empty_batch_and_determinism_and_in_place():
    P, T, d, S = 200, 150, 2, 64
    x, w, lam = random_case(P, T, d, per_diff=True, seed=9)
    xt, wt, lt = to_device(x, w, lam, S, torch.float32)
    z1, _ = whs.whs_solve(xt, wt, lt, d, P)
    z2, _ = whs.whs_solve(xt, wt, lt, d, P)
    x3 = xt.clone()
    whs.whs_solve(x3, wt, lt, d, P, z=x3)
    torch.cuda.synchronize()
    a, b, c = (synth.unpack_series(t.cpu(), P) for t in (z1, z2, x3))
    assert torch.equal(a, b)  # run-to-run bitwise determinism
    assert torch.equal(a, c)  # in place (z aliases x) gives the same result
    e = torch.empty((0, T, 1, S), dtype=torch.float32, device="cuda")
    we = torch.empty((0, T, S), dtype=torch.uint8, device="cuda")
    z0, i0 = whs.whs_solve(e, we, torch.empty(0, device="cuda"), d, 0)
    assert z0.numel() == 0 and i0.numel() == 0


def test_autograd_function_matches_oracle():
    P, T, d, S = 64, 120, 2, 64
    x, w, lam = random_case(P, T, d, per_diff=True, seed=21)
    xt, wt, lt = to_device(x, w, lam, S, torch.float64)
    xt.requires_grad_(True)
    lt.requires_grad_(True)
    z = whs.smooth(xt, lt, wt, d, P)
    g = torch.randn(z.shape, generator=torch.Generator(device="cuda").manual_seed(21), device="cuda",
                    dtype=z.dtype)
    (z * g).sum().backward()
    gn = from_device_series(g, P)
    gx_ref, gl_ref, _ = R.vjp(x, w, lam, d, gn, z=from_device_series(z.detach(), P))
    # norm-wise per series against the oracle's adjoint at the kernel's z, within
    # max(1e-9, the error bound of u = Omega^{-1} g for a small backward error)
    # (grad_lambda 10x: single entries of -(D u)(D z) cancel)
    tol = adjoint_tol(gn, w, lam, d)
    gx = from_device_series(xt.grad, P)
    gl = from_device_rows(lt.grad, P)
    assert (np.abs(gx - gx_ref).max(axis=(1, 2)) / np.abs(gx_ref).max(axis=(1, 2)) <= tol).all()
    assert (np.abs(gl - gl_ref).max(axis=1) / np.abs(gl_ref).max(axis=1) <= 10 * tol).all()
