"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compare the oracle with itself: each checks a closed form, an
invariant, a library routine, exact rational arithmetic or a hand-derived
fixture, chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.
"""

import os
from fractions import Fraction
from math import comb

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

from oracle import whs_ref as R

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
rng0 = np.random.default_rng(12345)


def _rand_case(P, T, d, p_obs=0.5, per_diff=False, C=1, seed=0, lam_lo=0.0, lam_hi=3.0):
    r = np.random.default_rng(seed)
    x = r.normal(size=(P, T, C))
    w = (r.random((P, T)) < p_obs).astype(np.uint8)
    w[:, :d + 1] = 1  # keep Omega positive definite for any draw
    if per_diff:
        lam = 10.0 ** r.uniform(lam_lo, lam_hi, size=(P, T - d))
    else:
        lam = 10.0 ** r.uniform(lam_lo, lam_hi, size=P)
    x = np.where(w[:, :, None] != 0, x, 0.0)
    return (x[:, :, 0] if C == 1 else x), w, lam


def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *v = line.split()
            vals[k] = [float(s) for s in v]
    return vals


# --- difference operator ----------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_difference_operator_is_numpy_diff(d):
    v = rng0.normal(size=(3, 17))
    np.testing.assert_allclose(R.apply_D(v, d), np.diff(v, n=d, axis=1), rtol=0, atol=1e-12)
    D = R.diff_matrix(17, d)
    np.testing.assert_allclose(v @ D.T, np.diff(v, n=d, axis=1), rtol=0, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_difference_kills_low_degree_and_scales_top_degree(d):
    t = np.arange(12, dtype=np.float64)
    D = R.diff_matrix(12, d)
    for deg in range(d):
        assert np.abs(D @ t ** deg).max() < 1e-9
    np.testing.assert_allclose(D @ t ** d, np.full(12 - d, float(np.prod(np.arange(1, d + 1)))))


# --- band storage (Fig. 2) ---------------------------------------------------

@pytest.mark.parametrize("name", ["band_T4_d1.txt", "band_T5_d2.txt"])
def test_band_storage_hand_fixture(name):
    g = _read_golden(name)
    T, d = int(g["T"][0]), int(g["d"][0])
    w = np.array([g["w"]], dtype=np.uint8)
    lam = np.array([g["lambda"]])
    AB = R.omega_band(w, lam, d)
    for i in range(d + 1):
        np.testing.assert_array_equal(AB[0, i], np.array(g[f"AB{i}"]))
    dense = R.omega_dense(w, lam, d)[0]
    for i in range(d + 1):
        np.testing.assert_array_equal(np.diagonal(dense, -i), np.array(g[f"AB{i}"])[:T - i])


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_band_equals_dense_assembly(d):
    x, w, lam = _rand_case(3, 11, d, per_diff=True, seed=d)
    np.testing.assert_allclose(R.band_to_dense(R.omega_band(w, lam, d)), R.omega_dense(w, lam, d),
                               rtol=1e-14, atol=0)


# --- exact rational arithmetic ------------------------------------------------

def _exact_solve(T, d, w, lam, x):
    """Gauss-Jordan on Fractions: Omega z = W x with Omega from its definition."""
    c = [(-1) ** (d - j) * comb(d, j) for j in range(d + 1)]
    A = [[Fraction(0)] * T for _ in range(T)]
    for t in range(T):
        A[t][t] += Fraction(w[t])
    for k in range(T - d):
        for a in range(d + 1):
            for b in range(d + 1):
                A[k + a][k + b] += Fraction(lam[k]) * c[a] * c[b]
    rhs = [Fraction(x[t]) if w[t] else Fraction(0) for t in range(T)]
    M = [row[:] + [rhs[i]] for i, row in enumerate(A)]
    for col in range(T):
        piv = next(r for r in range(col, T) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(T):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * b for a, b in zip(M[r], M[col])]
    return [M[i][T] / M[i][i] for i in range(T)]


@pytest.mark.parametrize("d", [1, 2, 3])
def test_exact_rational_solution(d):
    T = 9
    w = [1, 0, 1, 1, 0, 0, 1, 1, 1]
    lam = [Fraction(k + 1, 3) for k in range(T - d)]
    x = [Fraction(3 * t - 4, 7) for t in range(T)]
    ex = np.array([float(v) for v in _exact_solve(T, d, w, lam, x)])
    wa = np.array([w], dtype=np.uint8)
    la = np.array([[float(v) for v in lam]])
    xa = np.array([[float(v) for v in x]])
    zb, info = R.solve_band(xa, wa, la, d)
    zd = R.solve_dense(xa, wa, la, d)
    assert info[0] == 0
    np.testing.assert_allclose(zb[0], ex, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(zd[0], ex, rtol=1e-12, atol=1e-13)


# --- invariants the paper fixes ----------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3])
def test_P1_zero_weight_full_mask_is_identity(d):
    x = rng0.normal(size=(4, 30))
    w = np.ones((4, 30), dtype=np.uint8)
    for lam in (np.zeros(4), np.zeros((4, 30 - d))):
        zb, info = R.solve_band(x, w, lam, d)
        assert (info == 0).all()
        np.testing.assert_allclose(zb, x, rtol=0, atol=1e-14)
        np.testing.assert_allclose(R.solve_dense(x, w, lam, d), x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("per_diff", [False, True])
def test_P2_polynomials_below_order_reproduced(d, per_diff):
    T = 40
    _, w, lam = _rand_case(5, T, d, p_obs=0.3, per_diff=per_diff, seed=10 + d)
    t = np.arange(T, dtype=np.float64) / T
    r = np.random.default_rng(d)
    coef = r.normal(size=(5, d))
    p = sum(coef[:, j:j + 1] * t ** j for j in range(d))
    x = np.where(w != 0, p, 0.0)
    zb, info = R.solve_band(x, w, lam, d)
    assert (info == 0).all()
    # exact in exact arithmetic; in FP64 the residue grows with cond(Omega) ~ 4^d lambda
    tol = 1e-9 if d <= 3 else 1e-7
    np.testing.assert_allclose(zb, p, rtol=0, atol=tol)
    np.testing.assert_allclose(R.solve_dense(x, w, lam, d), p, rtol=0, atol=10 * tol)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P3_large_weight_tends_to_weighted_polynomial_fit(d):
    T = 14
    r = np.random.default_rng(100 + d)
    x = r.normal(size=(1, T))
    w = (r.random((1, T)) < 0.6).astype(np.uint8)
    w[0, :d + 2] = 1
    t = np.arange(T, dtype=np.float64)
    obs = w[0] != 0
    coef = np.polyfit(t[obs], x[0, obs], d - 1)  # least-squares polynomial of degree d-1
    fit = np.polyval(coef, t)
    # smallest non-null mode of D^T D ~ (pi/T)^(2d): start where 1/lambda dominates roundoff
    lam0 = 30.0 * (T / np.pi) ** (2 * d)
    errs = []
    for lam in (lam0, 10 * lam0, 100 * lam0):
        z, info = R.solve_band(np.where(w != 0, x, 0.0), w, np.array([lam]), d)
        errs.append(np.abs(z[0] - fit).max())
    # O(1/lambda) convergence: one decade of lambda gives one decade of error
    assert errs[2] < 1e-3 * np.abs(x).max()
    for a, b in zip(errs, errs[1:]):
        assert 7.0 < a / b < 14.0, errs


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P4_symmetry_and_time_reversal(d):
    T = 50
    _, w, lam = _rand_case(3, T, d, per_diff=True, seed=20 + d)
    r = np.random.default_rng(d)
    a = r.normal(size=(3, T))
    b = r.normal(size=(3, T))
    za, _ = R.solve_band(a, w, lam, d)
    zb, _ = R.solve_band(b, w, lam, d)
    lhs = (a * w * zb).sum(1)
    rhs = (b * w * za).sum(1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11)
    zr, _ = R.solve_band(a[:, ::-1], w[:, ::-1], lam[:, ::-1], d)
    np.testing.assert_allclose(zr[:, ::-1], za, rtol=0, atol=1e-11 * np.abs(za).max())


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P5_padding_with_unobserved_samples(d):
    T, pad = 35, 9
    x, w, lam = _rand_case(4, T, d, per_diff=False, seed=30 + d)
    z, _ = R.solve_band(x, w, lam, d)
    xp = np.concatenate([x, np.zeros((4, pad))], 1)
    wp = np.concatenate([w, np.zeros((4, pad), dtype=np.uint8)], 1)
    zp, info = R.solve_band(xp, wp, lam, d)
    assert (info == 0).all()
    np.testing.assert_allclose(zp[:, :T], z, rtol=0, atol=1e-10 * np.abs(z).max())


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P6_linearity_and_polynomial_shift(d):
    T = 45
    _, w, lam = _rand_case(3, T, d, per_diff=True, seed=40 + d)
    r = np.random.default_rng(d)
    a = r.normal(size=(3, T))
    b = r.normal(size=(3, T))
    za, _ = R.solve_band(a, w, lam, d)
    zb, _ = R.solve_band(b, w, lam, d)
    zab, _ = R.solve_band(2.5 * a - 0.75 * b, w, lam, d)
    np.testing.assert_allclose(zab, 2.5 * za - 0.75 * zb, rtol=0, atol=1e-11 * np.abs(zab).max())
    t = np.arange(T) / T
    poly = 0.3 + (1.7 * t if d >= 2 else 0.0)
    zs, _ = R.solve_band(a + poly, w, lam, d)
    np.testing.assert_allclose(zs, za + poly, rtol=0, atol=1e-10)


@pytest.mark.parametrize("lam", [0.5, 10.0, 1e3])
def test_P7_first_order_full_mask_dct_closed_form(lam):
    T = 64
    x = np.random.default_rng(7).normal(size=(2, T))
    w = np.ones((2, T), dtype=np.uint8)
    k = np.arange(T)
    filt = 1.0 / (1.0 + 4.0 * lam * np.sin(np.pi * k / (2 * T)) ** 2)
    ref = scipy.fft.idct(scipy.fft.dct(x, type=2, norm="ortho", axis=1) * filt, type=2, norm="ortho", axis=1)
    z, _ = R.solve_band(x, w, np.full(2, lam), 1)
    np.testing.assert_allclose(z, ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("per_diff", [False, True])
def test_P8_lapack_banded_solver(d, per_diff):
    T = 120
    x, w, lam = _rand_case(6, T, d, per_diff=per_diff, seed=50 + d, C=3)
    z, info = R.solve_band(x, w, lam, d)
    AB = R.omega_band(w, lam, d)
    for p in range(6):
        ref = scipy.linalg.solveh_banded(AB[p], np.where(w[p][:, None] != 0, x[p], 0.0), lower=True)
        np.testing.assert_allclose(z[p], ref, rtol=0, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P9_cholesky_band_is_numpy_cholesky(d):
    T = 25
    _, w, lam = _rand_case(4, T, d, per_diff=True, seed=60 + d)
    AB = R.omega_band(w, lam, d)
    Lb, info = R.cholesky_band(AB)
    assert (info == 0).all()
    dense = R.omega_dense(w, lam, d)
    for p in range(4):
        Lc = np.linalg.cholesky(dense[p])
        for i in range(d + 1):
            ref = np.concatenate([np.diagonal(Lc, -i), np.zeros(i)])
            np.testing.assert_allclose(Lb[p, i], ref, rtol=0, atol=1e-12 * np.abs(Lc).max())
        assert np.abs(np.tril(Lc, -d - 1)).max() < 1e-12 * np.abs(Lc).max()
    # LDL^T and LL^T agree: L_chol[t+i, t] = L[t+i, t] sqrt(D_t)
    Lrow, Dp, _ = R.ldl_band(AB)
    for i in range(1, d + 1):
        np.testing.assert_allclose(Lb[:, i, :T - i], Lrow[:, i, i:] * np.sqrt(Dp[:, :T - i]), rtol=1e-10)
    np.testing.assert_allclose(Lb[:, 0], np.sqrt(Dp), rtol=1e-9)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P9_alg1_update_order_is_numpy_cholesky(d):
    # the right-looking in-place factorisation (Alg. 1's order) against LAPACK's
    # dense Cholesky and against the left-looking column definition
    T = 23
    _, w, lam = _rand_case(3, T, d, per_diff=True, seed=90 + d)
    AB = R.omega_band(w, lam, d)
    AB0 = AB.copy()
    Lb, info = R.cholesky_band_inplace(AB)
    assert (info == 0).all()
    np.testing.assert_array_equal(AB, AB0)  # the caller's array is untouched
    dense = R.omega_dense(w, lam, d)
    for p in range(3):
        Lc = np.linalg.cholesky(dense[p])
        for i in range(d + 1):
            ref = np.concatenate([np.diagonal(Lc, -i), np.zeros(i)])
            # two FP64 factorisations of a matrix with condition up to ~1e9 (d = 4)
            np.testing.assert_allclose(Lb[p, i], ref, rtol=0, atol=1e-10 * np.abs(Lc).max())
    Lb2, _ = R.cholesky_band(AB)
    np.testing.assert_allclose(Lb, Lb2, rtol=0, atol=1e-10 * np.abs(Lb2).max())


def test_P9_alg1_update_order_hand_example_and_failure():
    # T = 3, d = 1, Omega = [[4, 2, 0], [2, 5, 3], [0, 3, 10]]: L = [[2], [1, 2], [0, 1.5, sqrt(7.75)]]
    AB = np.array([[[4.0, 5.0, 10.0], [2.0, 3.0, 0.0]]])
    Lb, info = R.cholesky_band_inplace(AB)
    assert info[0] == 0
    np.testing.assert_allclose(Lb[0], [[2.0, 2.0, np.sqrt(7.75)], [1.0, 1.5, 0.0]], rtol=1e-15)
    # a zero second pivot: Omega = [[1, 1], [1, 1]]
    _, info = R.cholesky_band_inplace(np.array([[[1.0, 1.0], [1.0, 0.0]]]))
    assert info[0] == 2


def test_P10_backward_error_small():
    for d in (1, 2, 3):
        x, w, lam = _rand_case(8, 300, d, p_obs=0.1, per_diff=True, seed=70 + d)
        z, _ = R.solve_band(x, w, lam, d)
        assert R.backward_error(x, w, lam, d, z).max() < 1e-13
    # and the check itself flags a wrong answer
    z2 = z.copy()
    z2[:, 150] += 1e-6
    assert R.backward_error(x, w, lam, d, z2).max() > 1e-10


# --- failure handling ------------------------------------------------------------

def test_info_reports_first_nonpositive_pivot():
    T, d = 30, 2
    x = np.ones((4, T))
    w = np.zeros((4, T), dtype=np.uint8)
    w[1, 5] = 1           # one sample < d: singular
    w[2, [3, 17]] = 1     # two samples = d: fine
    w[3, :] = 1
    lam = np.full((4, T - d), 10.0)
    lam[3, 7] = -1e3      # strongly negative weight -> indefinite
    z, info = R.solve_band(x, w, lam, d)
    assert info[0] > 0 and info[1] > 0 and info[2] == 0 and info[3] > 0
    assert np.isnan(z[0]).all() and np.isnan(z[1]).all() and np.isfinite(z[2]).all()
    # a decisive (non-rounding) failure: LAPACK reports the same leading minor
    _, info_c = R.cholesky_band(R.omega_band(w, lam, d))
    assert info_c[3] == info[3]
    with pytest.raises(np.linalg.LinAlgError) as e:
        scipy.linalg.cholesky_banded(R.omega_band(w, lam, d)[3], lower=True)
    assert str(info[3]) in str(e.value)
    # fewer than d observations: singular for any weight, reported even when
    # rounding leaves every computed pivot positive
    np.testing.assert_array_equal(R.structural_info(w, d, np.zeros(4, dtype=np.int64)), [T, T, 0, 0])


def test_unobserved_nan_is_ignored():
    x, w, lam = _rand_case(3, 40, 2, seed=80)
    z0, _ = R.solve_band(x, w, lam, 2)
    xn = np.where(w != 0, x, np.nan)
    z1, info = R.solve_band(xn, w, lam, 2)
    assert (info == 0).all()
    np.testing.assert_array_equal(z0, z1)


# --- adjoint (eq. (4), eq. (5)) ----------------------------------------------------

def _complex_step_grad_lambda(x, w, lam, d, g, h=1e-30):
    P, T = x.shape
    out = np.zeros(lam.shape)
    for k in range(lam.shape[1]):
        lc = lam.astype(np.complex128)
        lc[:, k] += 1j * h
        z = R.solve_dense(x.astype(np.complex128), w, lc, d)
        out[:, k] = (g * (z.imag / h)).sum(1)
    return out


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P11_grad_lambda_complex_step(d):
    T = 24
    x, w, lam = _rand_case(3, T, d, per_diff=True, seed=90 + d, lam_hi=2.0)
    g = np.random.default_rng(d).normal(size=(3, T))
    _, gl, info = R.vjp(x, w, lam, d, g)
    cs = _complex_step_grad_lambda(x, w, lam, d, g)
    np.testing.assert_allclose(gl, cs, rtol=1e-9, atol=1e-11 * np.abs(cs).max())
    # the complex-step path through the band solver agrees as well
    lc = lam.astype(np.complex128)
    lc[:, 3] += 1e-30j
    zc, _ = R.solve_band(x.astype(np.complex128), w, lc, d)
    np.testing.assert_allclose((g * zc.imag / 1e-30).sum(1), cs[:, 3], rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P11_grad_x_is_W_times_inverse_times_g(d):
    T = 30
    x, w, lam = _rand_case(3, T, d, per_diff=True, seed=100 + d)
    g = np.random.default_rng(d).normal(size=(3, T))
    gx, _, _ = R.vjp(x, w, lam, d, g)
    # directional derivative of the forward map, by linearity in x
    for trial in range(3):
        v = np.random.default_rng(trial).normal(size=(3, T))
        zv, _ = R.solve_band(v, w, lam, d)
        np.testing.assert_allclose((g * zv).sum(1), (gx * v).sum(1), rtol=1e-10)
    assert (gx[w == 0] == 0).all()


@pytest.mark.parametrize("d", [1, 2])
def test_P11_dense_torch_autograd(d):
    torch = pytest.importorskip("torch")
    T = 20
    x, w, lam = _rand_case(2, T, d, per_diff=True, seed=110 + d)
    g = np.random.default_rng(d).normal(size=(2, T))
    gx, gl, _ = R.vjp(x, w, lam, d, g)
    D = torch.tensor(R.diff_matrix(T, d))
    for p in range(2):
        xt = torch.tensor(x[p], requires_grad=True)
        lt = torch.tensor(lam[p], requires_grad=True)
        W = torch.diag(torch.tensor(w[p], dtype=torch.float64))
        Om = W + D.T @ torch.diag(lt) @ D
        z = torch.linalg.solve(Om, W @ xt)
        (z * torch.tensor(g[p])).sum().backward()
        np.testing.assert_allclose(gx[p], xt.grad.numpy(), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(gl[p], lt.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_P11_central_differences_and_scalar_sum():
    d, T = 2, 60
    x, w, lam = _rand_case(2, T, d, per_diff=False, seed=120, lam_lo=1.0, lam_hi=2.0)
    g = np.random.default_rng(0).normal(size=(2, T))
    _, gl, _ = R.vjp(x, w, lam, d, g)
    h = 1e-6 * lam
    zp, _ = R.solve_band(x, w, lam + h, d)
    zm, _ = R.solve_band(x, w, lam - h, d)
    fd = (g * (zp - zm)).sum(1) / (2 * h)
    np.testing.assert_allclose(gl, fd, rtol=1e-6)
    # scalar weight: gradient is the sum of the per-row gradients
    _, glr, _ = R.vjp(x, w, np.repeat(lam[:, None], T - d, 1), d, g)
    np.testing.assert_allclose(gl, glr.sum(1), rtol=1e-12)


def test_P11_dense_adjoint_matches_band_adjoint_multiband():
    d, T = 3, 22
    x, w, lam = _rand_case(2, T, d, per_diff=True, seed=130, C=3)
    g = np.random.default_rng(1).normal(size=(2, T, 3))
    gx, gl, _ = R.vjp(x, w, lam, d, g)
    gx2, gl2 = R.vjp_dense(x, w, lam, d, g)
    np.testing.assert_allclose(gx, gx2, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gl, gl2, rtol=1e-9, atol=1e-12)


def test_P11_grad_lambda_zero_for_low_degree_input():
    d, T = 3, 40
    _, w, lam = _rand_case(2, T, d, per_diff=True, seed=140)
    t = np.arange(T) / T
    x = np.where(w != 0, 1 - 2 * t + 0.5 * t ** 2, 0.0)
    g = np.random.default_rng(2).normal(size=(2, T))
    _, gl, _ = R.vjp(x, w, lam, d, g)
    assert np.abs(gl).max() < 1e-9


# --- selected inverse and GCV ------------------------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P12_selected_inverse_is_band_of_dense_inverse(d):
    T = 30
    _, w, lam = _rand_case(3, T, d, per_diff=True, seed=150 + d)
    Lrow, Dp, _ = R.ldl_band(R.omega_band(w, lam, d))
    S = R.selinv_band(Lrow, Dp)
    inv = np.linalg.inv(R.omega_dense(w, lam, d))
    for i in range(d + 1):
        np.testing.assert_allclose(S[:, i, :T - i], np.diagonal(inv, -i, axis1=1, axis2=2), rtol=1e-9,
                                   atol=1e-12)


def test_P12_effective_dimension_is_trace_of_hat_matrix():
    d, T = 2, 40
    x, w, _ = _rand_case(2, T, d, p_obs=0.4, seed=160)
    grid = np.array([0.3, 30.0, 3e3])
    _, ed, rss = R.gcv_scores(x, w, grid, d)
    for p in range(2):
        for gi, lam in enumerate(grid):
            obs = np.nonzero(w[p])[0]
            trace = 0.0
            for t in obs:  # H[t, t] = z(e_t)_t, the smoother applied to a unit spike
                e = np.zeros((1, T))
                e[0, t] = 1.0
                zt, _ = R.solve_band(e, w[p:p + 1], np.array([lam]), d)
                trace += zt[0, t]
            np.testing.assert_allclose(ed[p, gi], trace, rtol=1e-10)
            z, _ = R.solve_band(x[p:p + 1], w[p:p + 1], np.array([lam]), d)
            np.testing.assert_allclose(rss[p, gi], (w[p] * (x[p] - z[0]) ** 2).sum(), rtol=1e-10)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P12_effective_dimension_limits(d):
    T = 30
    x, w, _ = _rand_case(3, T, d, p_obs=0.3, seed=170 + d)
    m = w.sum(1)
    lam_big = 1e4 * (T / np.pi) ** (2 * d)  # far beyond the smallest non-null mode of D^T D
    grid = np.array([1e-6, 1.0, 1e3, lam_big])
    _, ed, _ = R.gcv_scores(x, w, grid, d)
    assert (ed >= d - 1e-3).all() and (ed <= m[:, None] + 1e-9).all()
    assert (np.diff(ed, axis=1) < 0).all()                # more smoothing, fewer degrees of freedom
    np.testing.assert_allclose(ed[:, -1], d, atol=1e-2)   # lambda -> inf: polynomial of degree d-1
    np.testing.assert_allclose(ed[:, 0], m, rtol=1e-4)    # lambda -> 0: interpolation
    wf = np.ones((1, T), dtype=np.uint8)
    _, ed1, _ = R.gcv_scores(x[:1], wf, np.array([1e-9]), d)
    np.testing.assert_allclose(ed1[0, 0], T, rtol=1e-6)


@pytest.mark.parametrize("lam", [0.3, 7.0, 2e3])
def test_P12_gcv_score_first_order_full_mask_closed_form(lam):
    # d = 1, w = 1: Omega = I + lam D^T D is diagonalised by the orthonormal DCT-II
    # with eigenvalues 1 + 4 lam sin^2(pi k / 2T).  So ED = sum_k 1/(1 + mu_k),
    # RSS = sum_k (mu_k / (1 + mu_k))^2 X_k^2 with X the DCT of x, and
    # GCV = T RSS / (T - ED)^2 (m = T observed points).
    T = 48
    x = np.random.default_rng(17).normal(size=(3, T)) + np.linspace(0, 2, T)
    w = np.ones((3, T), dtype=np.uint8)
    k = np.arange(T)
    mu = 4.0 * lam * np.sin(np.pi * k / (2 * T)) ** 2
    X = scipy.fft.dct(x, type=2, norm="ortho", axis=1)
    ed = (1.0 / (1.0 + mu)).sum()
    rss = ((mu / (1.0 + mu)) ** 2 * X ** 2).sum(axis=1)
    scores, eds, rsss = R.gcv_scores(x, w, np.array([lam]), 1)
    np.testing.assert_allclose(eds[:, 0], ed, rtol=1e-12)
    np.testing.assert_allclose(rsss[:, 0], rss, rtol=1e-10)
    np.testing.assert_allclose(scores[:, 0], T * rss / (T - ed) ** 2, rtol=1e-10)


def test_P12_gcv_argmin_matches_closed_form_scan():
    # the same closed form over the whole grid picks the same weight
    T = 64
    r = np.random.default_rng(23)
    x = np.sin(np.arange(T) / 6.0)[None, :] + 0.3 * r.normal(size=(4, T))
    w = np.ones((4, T), dtype=np.uint8)
    grid = R.gcv_grid()
    k = np.arange(T)
    X = scipy.fft.dct(x, type=2, norm="ortho", axis=1)
    ref = np.zeros((4, grid.size))
    for gi, lam in enumerate(grid):
        mu = 4.0 * lam * np.sin(np.pi * k / (2 * T)) ** 2
        ed = (1.0 / (1.0 + mu)).sum()
        ref[:, gi] = T * ((mu / (1.0 + mu)) ** 2 * X ** 2).sum(axis=1) / (T - ed) ** 2
    lam_best, idx, scores = R.gcv_select(x, w, grid, 1)
    np.testing.assert_allclose(scores, ref, rtol=1e-9)
    np.testing.assert_array_equal(idx, np.argmin(ref, axis=1))


@pytest.mark.parametrize("d,lam", [(1, 5.0), (2, 40.0), (3, 900.0)])
def test_gcv_sums_are_derivatives_along_the_weights(d, lam):
    # ED = tr(Omega^{-1} W) = d/deps log det(Omega + eps W) (Jacobi's formula) and
    # RSS = d/deps min_z [(1+eps) |x - z|_W^2 + lam |D z|^2] (envelope theorem), the
    # minimum being (1+eps) x'Wx - b'(Omega + eps W)^{-1} b with b = (1+eps) W x.
    # Central differences of dense LAPACK quantities against the oracle's plain sums.
    T = 60
    r = np.random.default_rng(31 + d)
    w = (r.random((1, T)) < 0.5).astype(np.uint8)
    w[0, ::7] = 1
    x = np.where(w != 0, 3.0 + np.sin(np.arange(T) / 5.0) + 0.2 * r.normal(size=(1, T)), 0.0)
    _, ed, rss = R.gcv_scores(x, w, np.array([lam]), d)
    Om = R.omega_dense(w, np.array([lam]), d)[0]
    W = np.diag(w[0].astype(np.float64))

    def logdet(eps):
        sgn, v = np.linalg.slogdet(Om + eps * W)
        assert sgn > 0
        return v

    # x relative to its first observed value: the smoother keeps constants, so RSS is
    # unchanged, and the two terms of the minimum cancel less
    xs = np.where(w[0] != 0, x[0] - x[0][np.argmax(w[0] != 0)], 0.0)

    def fmin(eps):
        b = (1.0 + eps) * (W @ xs)
        return (1.0 + eps) * xs @ W @ xs - b @ np.linalg.solve(Om + eps * W, b)

    h = 1e-4
    np.testing.assert_allclose((logdet(h) - logdet(-h)) / (2 * h), ed[0, 0], rtol=1e-7)
    np.testing.assert_allclose((fmin(h) - fmin(-h)) / (2 * h), rss[0, 0], rtol=1e-6)


def test_gcv_grid_and_tie_rule():
    grid = R.gcv_grid()
    assert grid.size == 21
    np.testing.assert_allclose(grid[[0, 10, 20]], [0.1, 100.0, 1e5], rtol=1e-12)
    # polynomial data: RSS = 0 for every lambda -> all scores tie at 0 -> smallest lambda
    T, d = 40, 2
    w = np.ones((1, T), dtype=np.uint8)
    x = (0.5 + 0.01 * np.arange(T))[None, :]
    lam_best, idx, scores = R.gcv_select(x, w, grid, d)
    assert idx[0] == 0 and lam_best[0] == grid[0]


def test_gcv_prefers_heavy_smoothing_on_noise_around_a_line():
    T, d = 200, 2
    r = np.random.default_rng(5)
    w = (r.random((4, T)) < 0.5).astype(np.uint8)
    x = np.where(w != 0, 0.1 + 0.001 * np.arange(T) + 0.05 * r.normal(size=(4, T)), 0.0)
    lam_best, idx, _ = R.gcv_select(x, w, R.gcv_grid(), d)
    assert (lam_best >= 1e3).all()


# --- posterior variance (diagonal of Omega^{-1}) ------------------------------------

@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("per_diff", [False, True])
def test_P13_posterior_variance_is_diagonal_of_dense_inverse(d, per_diff):
    T = 30
    _, w, lam = _rand_case(3, T, d, per_diff=per_diff, seed=170 + d)
    var, info = R.posterior_variance(w, lam, d)
    assert (info == 0).all()
    inv = np.linalg.inv(R.omega_dense(w, lam, d))
    np.testing.assert_allclose(var, np.diagonal(inv, axis1=1, axis2=2), rtol=1e-9)


def test_P13_posterior_variance_two_point_closed_form():
    # d = 1, T = 2, both observed: Omega = [[1+l, -l], [-l, 1+l]], diag of the
    # inverse = (1+l) / (1+2l)
    lam = np.array([0.0, 0.5, 3.0, 1e4])
    w = np.ones((4, 2), np.uint8)
    var, _ = R.posterior_variance(w, lam, 1)
    expect = (1 + lam) / (1 + 2 * lam)
    # the second pivot (1+l) - l^2/(1+l) cancels: relative rounding about l * eps
    np.testing.assert_allclose(var, np.stack([expect, expect], 1), rtol=4 * (1 + lam.max()) * 2.2e-16)


def test_P13_posterior_variance_identity_and_time_reversal():
    T, d = 25, 3
    var, _ = R.posterior_variance(np.ones((1, T), np.uint8), np.zeros(1), d)
    np.testing.assert_array_equal(var, np.ones((1, T)))
    _, w, lam = _rand_case(2, T, d, per_diff=True, seed=181)
    w[:, -d - 1:] = 1
    v, _ = R.posterior_variance(w, lam, d)
    vr, _ = R.posterior_variance(w[:, ::-1].copy(), lam[:, ::-1].copy(), d)
    np.testing.assert_allclose(vr[:, ::-1], v, rtol=1e-10)


def test_P13_posterior_variance_decreases_with_each_new_observation():
    T, d = 40, 2
    _, w, lam = _rand_case(1, T, d, per_diff=True, p_obs=0.2, seed=190)
    v0, _ = R.posterior_variance(w, lam, d)
    t = int(np.nonzero(w[0] == 0)[0][len(np.nonzero(w[0] == 0)[0]) // 2])
    w1 = w.copy()
    w1[0, t] = 1
    v1, _ = R.posterior_variance(w1, lam, d)
    assert (v1 <= v0 * (1 + 1e-12)).all()
    assert v1[0, t] < v0[0, t] * (1 - 1e-6)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P13_posterior_variance_heavy_smoothing_is_polynomial_fit_variance(d):
    # lambda -> inf: z is the least-squares polynomial of degree d-1 through the
    # observed samples, whose variance at t is phi(t)^T (V^T W V)^{-1} phi(t)
    T = 24
    r = np.random.default_rng(200 + d)
    w = (r.random((1, T)) < 0.5).astype(np.uint8)
    w[0, :d + 1] = 1
    var, _ = R.posterior_variance(w, np.array([1e9]), d)
    tt = (np.arange(T) - T / 2) / T
    V = np.stack([tt ** k for k in range(d)], 1)
    G = V.T @ (V * w[0][:, None])
    expect = np.einsum("tk,kl,tl->t", V, np.linalg.inv(G), V)
    np.testing.assert_allclose(var[0], expect, rtol=2e-4)
    assert abs((var[0] * w[0]).sum() - d) < 1e-3


# --- uneven sample times (Sec. II: divided-difference operator) ----------------------

def _uneven_times(T, seed, step=5.0):
    """Revisit every ``step`` days with random skipped passes (strictly increasing)."""
    r = np.random.default_rng(seed)
    gaps = step * r.integers(1, 4, size=T)
    return 7.0 + np.cumsum(gaps)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P14_unit_and_constant_spacing_give_binomial_rows(d):
    T = 12
    c1 = R.diff_coeffs_times(np.arange(T) + 40.0, d)
    np.testing.assert_array_equal(c1, np.tile(R.diff_coeffs(d), (T - d, 1)))
    c5 = R.diff_coeffs_times(5.0 * np.arange(T), d)
    np.testing.assert_allclose(c5, np.tile(R.diff_coeffs(d), (T - d, 1)) / 5.0 ** d, rtol=1e-14)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P14_closed_form_matches_the_recursive_definition(d):
    # order-k operator = diag(k / (t_{i+k} - t_i)) times the first difference of
    # the order-(k-1) operator, starting from diag(1 / (t_{i+1} - t_i)) times
    # the first difference
    T = 15
    t = _uneven_times(T, seed=d)

    def first_diff(n):
        F = np.zeros((n - 1, n))
        for i in range(n - 1):
            F[i, i], F[i, i + 1] = -1.0, 1.0
        return F

    Dk = np.diag(1.0 / (t[1:] - t[:-1])) @ first_diff(T)
    for k in range(2, d + 1):
        Dk = np.diag(k / (t[k:] - t[:-k])) @ first_diff(T - k + 1) @ Dk
    D = R.diff_matrix(T, d, R.diff_coeffs_times(t, d))
    np.testing.assert_allclose(D, Dk, rtol=1e-10, atol=1e-12 * np.abs(Dk).max())


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P14_kills_low_degree_polynomials_and_maps_t_to_the_d_to_d_factorial(d):
    T = 20
    t = _uneven_times(T, seed=10 + d) / 100.0
    D = R.diff_matrix(T, d, R.diff_coeffs_times(t, d))
    for q in range(d):
        assert np.abs(D @ t ** q).max() < 1e-9 * np.abs(D).max()
    np.testing.assert_allclose(D @ t ** d, np.full(T - d, float(np.prod(np.arange(1, d + 1)))), rtol=1e-8)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_P14_uneven_smoother_reproduces_low_degree_polynomials(d):
    T = 40
    t = _uneven_times(T, seed=20 + d) / 50.0
    coef = R.diff_coeffs_times(t, d)
    r = np.random.default_rng(d)
    w = (r.random((2, T)) < 0.4).astype(np.uint8)
    w[:, :d + 1] = 1
    poly = np.polyval(r.normal(size=d), t)            # degree d-1
    x = np.where(w != 0, poly[None, :], 0.0)
    z, info = R.solve_band(x, w, np.array([3.0, 300.0]), d, coef)
    assert (info == 0).all()
    # exact in exact arithmetic; the bound only absorbs rounding amplified by the
    # conditioning of Omega (close times give large coefficients)
    np.testing.assert_allclose(z, np.tile(poly, (2, 1)), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_P14_uneven_band_solve_and_adjoint_match_dense(d):
    T = 30
    t = _uneven_times(T, seed=30 + d)
    coef = R.diff_coeffs_times(t, d) * 5.0 ** d       # order-one entries
    x, w, lam = _rand_case(3, T, d, per_diff=True, seed=300 + d)
    zb, _ = R.solve_band(x, w, lam, d, coef)
    np.testing.assert_allclose(zb, R.solve_dense(x, w, lam, d, coef), rtol=1e-8, atol=1e-10)
    g = np.random.default_rng(d).normal(size=x.shape)
    gx, gl, _ = R.vjp(x, w, lam, d, g, coef=coef)
    gxd, gld = R.vjp_dense(x, w, lam, d, g, coef=coef)
    np.testing.assert_allclose(gx, gxd, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(gl, gld, rtol=1e-7, atol=1e-10 * np.abs(gld).max())


def test_P14_uneven_time_rescaling_is_absorbed_by_the_weights():
    # times * s scales row coefficients by s^-d, so lambda * s^(2d) gives the same z
    T, d, s = 35, 2, 3.7
    t = _uneven_times(T, seed=41)
    x, w, lam = _rand_case(2, T, d, per_diff=True, seed=410)
    z1, _ = R.solve_band(x, w, lam, d, R.diff_coeffs_times(t, d))
    z2, _ = R.solve_band(x, w, lam * s ** (2 * d), d, R.diff_coeffs_times(s * t, d))
    np.testing.assert_allclose(z2, z1, rtol=1e-9, atol=1e-12)


def test_P14_uneven_grad_lambda_by_finite_differences():
    T, d = 25, 2
    t = _uneven_times(T, seed=51)
    coef = R.diff_coeffs_times(t, d) * 25.0
    x, w, lam = _rand_case(1, T, d, per_diff=True, seed=510)
    g = np.random.default_rng(5).normal(size=x.shape)
    _, gl, _ = R.vjp(x, w, lam, d, g, coef=coef)
    for k in (0, 7, T - d - 1):
        h = 1e-6 * lam[0, k]
        lp, lm = lam.copy(), lam.copy()
        lp[0, k] += h
        lm[0, k] -= h
        fd = (np.sum(g * R.solve_band(x, w, lp, d, coef)[0]) - np.sum(g * R.solve_band(x, w, lm, d, coef)[0])) / (2 * h)
        assert abs(fd - gl[0, k]) <= 1e-5 * abs(fd) + 1e-6 * np.abs(gl).max(), (k, fd, gl[0, k])


# --- accuracy metrics used by the FP64 parity bars ------------------------------


def _ill_case(d):
    """An ill-conditioned series with exactly representable inputs: a long gap,
    large integer weights, dyadic values."""
    T = 16
    w = [1, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 1, 1, 1]
    lam = [Fraction(10 ** (3 + (k % 3))) for k in range(T - d)]
    x = [Fraction((5 * t * t - 3 * t + 1) % 17, 8) for t in range(T)]
    return T, w, lam, x


@pytest.mark.parametrize("d", [2, 3])
def test_refined_solution_matches_exact_rational_solution(d):
    T, w, lam, x = _ill_case(d)
    ex = np.array([float(v) for v in _exact_solve(T, d, w, lam, x)])
    wa = np.array([w], dtype=np.uint8)
    la = np.array([[float(v) for v in lam]])
    b = np.array([[float(v) if w[t] else 0.0 for t, v in enumerate(x)]])
    plain, _ = R.solve_band(b, wa, la, d)
    ref = R.solve_band_refined(b, wa, la, d).astype(np.float64)
    e_plain = np.abs(plain[0] - ex).max() / np.abs(ex).max()
    e_ref = np.abs(ref[0] - ex).max() / np.abs(ex).max()
    kappa = np.linalg.cond(R.omega_dense(wa, la, d)[0])
    assert e_plain > 1e-12  # the case is ill-conditioned enough to matter
    # limiting accuracy of refinement with a 64-bit-significand residual
    assert e_ref <= 4 * kappa * 2.0 ** -64 and e_ref <= e_plain / 100, (e_ref, e_plain, kappa)


@pytest.mark.parametrize("d", [2, 3])
def test_solution_error_bound_covers_the_true_error(d):
    T, w, lam, x = _ill_case(d)
    ex = np.array([float(v) for v in _exact_solve(T, d, w, lam, x)])
    wa = np.array([w], dtype=np.uint8)
    la = np.array([[float(v) for v in lam]])
    b = np.array([[float(v) if w[t] else 0.0 for t, v in enumerate(x)]])
    plain, _ = R.solve_band(b, wa, la, d)
    rng = np.random.default_rng(d)
    for z in (plain[0], plain[0] * (1 + 1e-9 * rng.standard_normal(T)), ex + 1e-6 * np.abs(ex).max() * np.eye(T)[5]):
        err = np.abs(z - ex).max() / np.abs(z).max()
        bound = R.solution_error_bound(b, wa, la, d, z[None])[0]
        assert err <= bound * (1 + 1e-6), (err, bound)
        assert bound <= 1e4 * max(err, 1e-16) * np.linalg.cond(R.omega_dense(wa, la, d)[0]), (err, bound)


def test_solution_error_bound_with_a_given_backward_error_scales_linearly():
    x, w, lam = _rand_case(3, 40, 2, per_diff=True, seed=4)
    b = np.where(w != 0, x, 0.0)
    z, _ = R.solve_band(b, w, lam, 2)
    b1 = R.solution_error_bound(b, w, lam, 2, z, beta=1e-15)
    b2 = R.solution_error_bound(b, w, lam, 2, z, beta=2e-15)
    np.testing.assert_allclose(b2, 2 * b1, rtol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_refined_inverse_diagonal_matches_exact_rational_inverse(d):
    T, w, lam, _ = _ill_case(d)
    wa = np.array([w], dtype=np.uint8)
    la = np.array([[float(v) for v in lam]])
    # exact inverse by Gauss-Jordan on Fractions against the identity
    c = [(-1) ** (d - j) * comb(d, j) for j in range(d + 1)]
    A = [[Fraction(0)] * T for _ in range(T)]
    for t in range(T):
        A[t][t] += Fraction(w[t])
    for k in range(T - d):
        for a in range(d + 1):
            for bb in range(d + 1):
                A[k + a][k + bb] += lam[k] * c[a] * c[bb]
    M = [row[:] + [Fraction(int(i == j)) for j in range(T)] for i, row in enumerate(A)]
    for col in range(T):
        piv = next(r for r in range(col, T) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(T):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * q for a, q in zip(M[r], M[col])]
    ex = np.array([float(M[i][T + i] / M[i][i]) for i in range(T)])
    ref = R.inverse_diag_refined(wa, la, d)[0]
    kappa = np.linalg.cond(R.omega_dense(wa, la, d)[0])
    assert np.abs(ref - ex).max() / np.abs(ex).max() <= 4 * kappa * 2.0 ** -64
    var, _ = R.posterior_variance(wa, la, d)
    err = np.abs(var[0] - ex).max() / np.abs(ex).max()
    bound = R.inverse_diag_error_bound(wa, la, d, 1e-15)[0]
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("d,per_diff,C", [(1, True, 1), (2, True, 1), (2, False, 3), (3, True, 2), (4, False, 1)])
def test_whole_batch_backward_error_helper_matches_the_oracle(d, per_diff, C):
    # the device-side helper the full-size GPU tests use, run here on the CPU
    import torch
    from paper_2604_00048_amd import synth
    from tests._cases import backward_error_interleaved
    P, T = 150, 61
    x, w, lam = _rand_case(P, T, d, p_obs=0.4, per_diff=per_diff, C=C, seed=d)
    z, _ = R.solve_band(x, w, lam, d)
    z = z.reshape(P, T, C) * (1 + 1e-9 * np.random.default_rng(0).standard_normal((P, T, C)))
    ref = R.backward_error(x.reshape(P, T, C), w, lam, d, z)
    xt = synth.pack_series(torch.tensor(x.reshape(P, T, C)), 64)
    zt = synth.pack_series(torch.tensor(z), 64)
    wt = synth.pack_rows(torch.tensor(w), 64)
    lt = synth.pack_rows(torch.tensor(lam), 64) if per_diff else torch.tensor(lam)
    got = backward_error_interleaved(xt, wt, lt, zt, d, chunk_blocks=2)[:P]
    np.testing.assert_allclose(got, ref, rtol=1e-6, atol=1e-18)
    assert got.max() > 1e-12  # the perturbation is seen
