"""FP64 reference of the Whittaker-Henderson smoother, its adjoint and GCV.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and ``bench.py``'s ``cpu_baseline`` leg, never by the GPU library.

Everything here is written from the paper's definitions, slowly and plainly:

* Sec. II: ``x`` in R^T, ``W = diag(w)`` with ``w_t`` in {0, 1}, ``D`` the
  difference operator of order ``d`` (the paper's ``k+1``), one smoothing
  weight per row of ``D``.  On a daily grid the divided difference of
  Sec. II reduces to binomial differences ``c_j = (-1)^(d-j) C(d, j)``.
* eq. (2) / eq. (3): ``z = (W + D^T Lambda D)^{-1} W x``; ``Omega`` is the
  matrix in brackets (Sec. III), symmetric positive definite with ``d``
  sub-diagonals.
* Sec. II, uneven sample times: ``D`` is the discrete derivative of the
  cited monograph (``d!`` times the divided difference over ``d+1``
  consecutive times), passed as a ``(T-d, d+1)`` table ``coef`` of row
  coefficients; every function taking ``coef=None`` uses the daily grid.
* Fig. 2: lower band storage ``AB[i, t] = Omega[t+i, t]`` with a zero tail.
* Sec. III-A: Cholesky factorisation, then forward and back substitution.
* eq. (4) / eq. (5): derivatives w.r.t. the per-row weights and w.r.t. ``x``;
  contracted with an upstream gradient ``g`` they give the adjoint
  ``grad_x = W Omega^{-1} g`` and ``grad_lambda_k = -(D u)_k (D z)_k`` with
  ``u = Omega^{-1} g``.

Array conventions (natural layout, one row per series):

* ``x``: ``(P, T)`` or ``(P, T, C)`` -- ``C`` bands share one ``Omega``
  (Sec. II: the batched multivariate extension);
* ``w``: ``(P, T)`` of 0/1;
* ``lam``: ``(P,)`` (one scalar per series, eq. (2)) or ``(P, T-d)`` (one
  weight per row of ``D``, eq. (3)).

Readings where the paper is silent or loose (each is also listed in the
design notes): the weights have length ``T-d`` (one per row of ``D``); ``x``
at ``w_t = 0`` is ignored, not multiplied (so NaN there is harmless); a
series whose ``Omega`` is not positive definite (fewer than ``d`` observed
samples, a non-positive or NaN weight) reports ``info = t+1`` for the first
failing pivot ``t`` and gets NaN outputs.
"""

from __future__ import annotations

from math import comb

import numpy as np

# ---------------------------------------------------------------------------
# operator and matrix assembly
# ---------------------------------------------------------------------------


def diff_coeffs(d: int) -> np.ndarray:
    """Coefficients of the order-``d`` forward difference on unit spacing.

    ``(D v)_k = sum_j c_j v_{k+j}``, ``c_j = (-1)^(d-j) C(d, j)`` (Sec. II, the
    divided difference on a daily grid).
    """
    return np.array([(-1) ** (d - j) * comb(d, j) for j in range(d + 1)], dtype=np.float64)


def diff_coeffs_times(times, d: int) -> np.ndarray:
    """Row coefficients of the order-``d`` discrete derivative on sample times
    ``t_0 < ... < t_{T-1}`` (Sec. II: the difference operator for unevenly
    spaced samples of the cited monograph on divided differences, Sec. 6
    there).  Row ``k`` is ``d!`` times the divided difference over
    ``t_k..t_{k+d}``:
    ``c[k, j] = d! / prod_{m != j} (t_{k+j} - t_{k+m})``, ``j = 0..d``.
    On unit spacing this is ``(-1)^(d-j) C(d, j)``.  Returns ``(T-d, d+1)``.
    """
    t = np.asarray(times, dtype=np.float64)
    T = t.shape[0]
    fact = float(np.prod(np.arange(1, d + 1)))
    c = np.zeros((T - d, d + 1))
    for k in range(T - d):
        for j in range(d + 1):
            den = 1.0
            for m in range(d + 1):
                if m != j:
                    den *= t[k + j] - t[k + m]
            c[k, j] = fact / den
    return c


def diff_matrix(T: int, d: int, coef=None) -> np.ndarray:
    """Dense ``(T-d) x T`` difference operator ``D`` (Sec. II); ``coef`` is an
    optional ``(T-d, d+1)`` table of row coefficients (uneven sample times),
    the daily-grid binomial row otherwise."""
    c = diff_coeffs(d)
    D = np.zeros((T - d, T))
    for k in range(T - d):
        D[k, k:k + d + 1] = c if coef is None else coef[k]
    return D


def _as3(x: np.ndarray) -> tuple[np.ndarray, bool]:
    x = np.asarray(x)
    if x.ndim == 2:
        return x[:, :, None], True
    return x, False


def lam_rows(lam, P: int, T: int, d: int) -> np.ndarray:
    """One weight per row of ``D``: a scalar per series is broadcast (eq. (2))."""
    lam = np.asarray(lam)
    if lam.ndim == 0:
        return np.full((P, T - d), lam[()], dtype=lam.dtype if lam.dtype.kind == "c" else np.float64)
    if lam.ndim == 1:
        assert lam.shape[0] == P
        return np.repeat(lam[:, None], T - d, axis=1)
    assert lam.shape == (P, T - d), (lam.shape, (P, T - d))
    return lam


def omega_dense(w: np.ndarray, lam, d: int, coef=None) -> np.ndarray:
    """``Omega = W + D^T Lambda D`` as dense ``(P, T, T)`` (eq. (3))."""
    w = np.asarray(w)
    P, T = w.shape
    L = lam_rows(lam, P, T, d)
    D = diff_matrix(T, d, coef)
    dt = np.result_type(L.dtype, np.float64)
    out = np.zeros((P, T, T), dtype=dt)
    for p in range(P):
        out[p] = np.diag(w[p].astype(np.float64)) + D.T @ (L[p][:, None] * D)
    return out


def omega_band(w: np.ndarray, lam, d: int, coef=None) -> np.ndarray:
    """Lower band storage of ``Omega``: ``AB[p, i, t] = Omega[p, t+i, t]`` (Fig. 2).

    Built from ``D^T Lambda D = sum_k lambda_k d_k d_k^T`` (``d_k`` the k-th row
    of ``D``): row ``k`` adds ``lambda_k c_a c_b`` to ``Omega[k+a, k+b]``
    (``c`` the row's coefficients: ``coef[k]`` if given, else the binomial row).
    Entries with ``t+i >= T`` stay zero (the padded tail of Fig. 2).
    """
    w = np.asarray(w)
    P, T = w.shape
    L = lam_rows(lam, P, T, d)
    c = np.tile(diff_coeffs(d), (T - d, 1)) if coef is None else np.asarray(coef, dtype=np.float64)
    dt = np.result_type(L.dtype, np.float64)
    AB = np.zeros((P, d + 1, T), dtype=dt)
    AB[:, 0, :] += w
    k = np.arange(T - d)
    for a in range(d + 1):
        for b in range(a + 1):
            # Omega[k+a, k+b] with a >= b  ->  AB[a-b, k+b]
            AB[:, a - b, k + b] += L * (c[:, a] * c[:, b])
    return AB


def band_to_dense(AB: np.ndarray) -> np.ndarray:
    """Symmetric dense matrix from lower band storage (inverse of Fig. 2)."""
    P, dp1, T = AB.shape
    M = np.zeros((P, T, T), dtype=AB.dtype)
    for i in range(dp1):
        for t in range(T - i):
            M[:, t + i, t] = AB[:, i, t]
            M[:, t, t + i] = AB[:, i, t]
    return M


# ---------------------------------------------------------------------------
# O-dense: the closed form by LU (tiny T)
# ---------------------------------------------------------------------------


def solve_dense(x: np.ndarray, w: np.ndarray, lam, d: int, coef=None) -> np.ndarray:
    """``z = Omega^{-1} W x`` with a dense LU solve (eq. (2) / eq. (3))."""
    x3, squeeze = _as3(x)
    w = np.asarray(w)
    Om = omega_dense(w, lam, d, coef)
    rhs = np.where(w[:, :, None] != 0, x3, 0.0)
    z = np.linalg.solve(Om, rhs)
    return z[:, :, 0] if squeeze else z


def solve_dense_rhs(b: np.ndarray, w: np.ndarray, lam, d: int, coef=None) -> np.ndarray:
    """``v = Omega^{-1} b`` (dense LU), any right-hand side ``b``."""
    b3, squeeze = _as3(b)
    v = np.linalg.solve(omega_dense(w, lam, d, coef), b3)
    return v[:, :, 0] if squeeze else v


# ---------------------------------------------------------------------------
# O-band: banded LDL^T with a loop over time, vectorised over series
# ---------------------------------------------------------------------------


def ldl_band(AB: np.ndarray):
    """Banded ``Omega = L diag(Dp) L^T`` with unit lower ``L`` (Sec. III-A).

    Returns ``Lrow`` with ``Lrow[p, j, t] = L[t, t-j]`` (``j = 1..d``; row 0 is
    1), the pivots ``Dp`` and ``info`` (0, or ``t+1`` for the first pivot that
    is not positive and finite).  From ``Omega = L D L^T`` entrywise:
    ``L[t, t-j] = (Omega[t, t-j] - sum_{m>j} L[t, t-m] Dp[t-m] L[t-j, t-m]) / Dp[t-j]``
    and ``Dp[t] = Omega[t, t] - sum_j L[t, t-j]^2 Dp[t-j]``.
    """
    P, dp1, T = AB.shape
    d = dp1 - 1
    Lrow = np.zeros_like(AB)
    Lrow[:, 0, :] = 1.0
    Dp = np.zeros((P, T), dtype=AB.dtype)
    info = np.zeros(P, dtype=np.int64)
    for t in range(T):
        for j in range(min(d, t), 0, -1):
            acc = AB[:, j, t - j].copy()  # Omega[t, t-j]
            for m in range(j + 1, min(d, t) + 1):
                acc -= Lrow[:, m, t] * Dp[:, t - m] * Lrow[:, m - j, t - j]
            Lrow[:, j, t] = acc / Dp[:, t - j]
        acc = AB[:, 0, t].copy()
        for j in range(1, min(d, t) + 1):
            acc -= Lrow[:, j, t] ** 2 * Dp[:, t - j]
        Dp[:, t] = acc
        bad = (info == 0) & ~(np.isfinite(acc) & (np.real(acc) > 0))
        info[bad] = t + 1
    return Lrow, Dp, info


def _subst(Lrow: np.ndarray, Dp: np.ndarray, b3: np.ndarray) -> np.ndarray:
    """Forward ``L y = b`` then back ``D L^T z = y`` (Sec. III-A)."""
    P, dp1, T = Lrow.shape
    d = dp1 - 1
    y = np.zeros_like(b3, dtype=np.result_type(b3.dtype, Lrow.dtype))
    for t in range(T):
        acc = b3[:, t, :].astype(y.dtype)
        for j in range(1, min(d, t) + 1):
            acc = acc - Lrow[:, j, t, None] * y[:, t - j, :]
        y[:, t, :] = acc
    z = np.zeros_like(y)
    for t in range(T - 1, -1, -1):
        acc = y[:, t, :] / Dp[:, t, None]
        for j in range(1, min(d, T - 1 - t) + 1):
            acc = acc - Lrow[:, j, t + j, None] * z[:, t + j, :]
        z[:, t, :] = acc
    return z


def structural_info(w: np.ndarray, d: int, info: np.ndarray) -> np.ndarray:
    """Fewer than ``d`` observed samples make ``Omega`` singular for every weight
    (polynomials of degree < d are in the null space of ``D``).  Rounding decides
    the sign of the last pivots then, so such a series is reported as failed
    with ``info = T`` when no pivot failed before."""
    w = np.asarray(w)
    T = w.shape[1]
    m = (w != 0).sum(axis=1)
    out = info.copy()
    out[(out == 0) & (m < d)] = T
    return out


def solve_band_rhs(b: np.ndarray, w: np.ndarray, lam, d: int, coef=None):
    """``v = Omega^{-1} b`` by banded LDL^T; returns ``(v, info)``; failed series are NaN."""
    b3, squeeze = _as3(b)
    AB = omega_band(w, lam, d, coef)
    Lrow, Dp, info = ldl_band(AB)
    info = structural_info(w, d, info)
    v = _subst(Lrow, Dp, b3)
    v[info != 0] = np.nan
    return (v[:, :, 0] if squeeze else v), info


def solve_band(x: np.ndarray, w: np.ndarray, lam, d: int, coef=None):
    """``z = Omega^{-1} W x`` by banded LDL^T (eq. (3), Sec. III-A); returns ``(z, info)``.

    ``x`` is selected where ``w_t = 1``, never multiplied, so its value at
    unobserved times does not matter.
    """
    x3, squeeze = _as3(x)
    w = np.asarray(w)
    rhs = np.where(w[:, :, None] != 0, x3, 0.0)
    z, info = solve_band_rhs(rhs, w, lam, d, coef)
    return (z[:, :, 0] if squeeze else z), info


def cholesky_band(AB: np.ndarray, w: np.ndarray | None = None):
    """Cholesky factor ``Omega = L L^T`` in lower band storage (Sec. III-A, Alg. 1 output).

    ``Lb[p, i, t] = L[t+i, t]`` (Fig. 2 layout, zero tail).  Written from the
    definition column by column: ``L[t, t] = sqrt(Omega[t, t] - sum_m L[t, t-m]^2)``
    and ``L[t+i, t] = (Omega[t+i, t] - sum_m L[t+i, t-m] L[t, t-m]) / L[t, t]``.
    Returns ``(Lb, info)``; with the mask ``w`` the singular-series rule of
    ``structural_info`` is applied as well.
    """
    P, dp1, T = AB.shape
    d = dp1 - 1
    Lb = np.zeros_like(AB)
    info = np.zeros(P, dtype=np.int64)
    for t in range(T):
        acc = AB[:, 0, t].copy()
        for m in range(1, min(d, t) + 1):
            acc -= Lb[:, m, t - m] ** 2  # L[t, t-m]
        bad = (info == 0) & ~(np.isfinite(acc) & (acc > 0))
        info[bad] = t + 1
        piv = np.sqrt(np.where(acc > 0, acc, np.nan))
        Lb[:, 0, t] = piv
        for i in range(1, min(d, T - 1 - t) + 1):
            acc = AB[:, i, t].copy()  # Omega[t+i, t]
            for m in range(1, d - i + 1):
                if t - m < 0:
                    break
                acc -= Lb[:, i + m, t - m] * Lb[:, m, t - m]  # L[t+i, t-m] L[t, t-m]
            Lb[:, i, t] = acc / piv
    if w is not None:
        info = structural_info(w, d, info)
    return Lb, info


def cholesky_band_inplace(AB: np.ndarray):
    """Cholesky factor in lower band storage by Alg. 1's update order (Sec. III-A).

    A second, independently organised factorisation next to ``cholesky_band``:
    Alg. 1 works in place on the band array and is right-looking.  For each
    column ``t``: the pivot ``omega = AB[0, t]`` becomes ``sqrt(omega)``, the
    column's sub-diagonal entries ``v = AB[1:, t]`` are divided by
    ``sqrt(omega)``, and every later column ``t+1+u`` that ``v`` reaches
    (``u < d`` and ``t+1+u < T``) loses the outer-product term: its band
    entries ``AB[i, t+1+u] = Omega[t+1+u+i, t+1+u]`` for ``i = 0..d-1-u``
    decrease by ``v[u+i] v[u] / omega`` (``v`` is the column before scaling).
    ``AB[p, i, t]`` is ``Omega[t+i, t]`` with a zero tail (Fig. 2).  Returns
    ``(Lb, info)`` like ``cholesky_band``; the input is not modified.
    """
    A = np.array(AB, dtype=np.float64, copy=True)
    P, dp1, T = A.shape
    d = dp1 - 1
    info = np.zeros(P, dtype=np.int64)
    for t in range(T):
        omega = A[:, 0, t].copy()
        bad = (info == 0) & ~(np.isfinite(omega) & (omega > 0))
        info[bad] = t + 1
        omega = np.where(omega > 0, omega, np.nan)
        v = A[:, 1:, t].copy()          # Omega[t+1.., t] after the earlier updates
        root = np.sqrt(omega)
        A[:, 0, t] = root
        A[:, 1:, t] = v / root[:, None]
        for u in range(min(d, T - t - 1)):
            col = t + 1 + u
            n = d - u                   # entries of column col still inside v's reach
            A[:, :n, col] -= v[:, u:u + n] * (v[:, u] / omega)[:, None]
    return A, info


# ---------------------------------------------------------------------------
# adjoint (eq. (4), eq. (5))
# ---------------------------------------------------------------------------


def apply_D(v: np.ndarray, d: int, coef=None) -> np.ndarray:
    """``(D v)_k`` along axis 1 for ``k = 0..T-d-1``."""
    T = v.shape[1]
    c = np.tile(diff_coeffs(d), (T - d, 1)) if coef is None else np.asarray(coef, dtype=np.float64)
    out = np.zeros((v.shape[0], T - d) + v.shape[2:], dtype=v.dtype)
    for j in range(d + 1):
        cj = c[:, j].reshape((1, T - d) + (1,) * (v.ndim - 2))
        out = out + cj * v[:, j:T - d + j]
    return out


def vjp(x: np.ndarray, w: np.ndarray, lam, d: int, g: np.ndarray, z: np.ndarray | None = None, coef=None):
    """Adjoint of ``z = Omega^{-1} W x`` against upstream gradient ``g``.

    ``u = Omega^{-1} g``; ``grad_x = W u`` (eq. (5) as a vector-Jacobian
    product); ``grad_lambda_k = -sum_c (D u_c)_k (D z_c)_k`` (eq. (4)
    contracted with ``g``: ``g^T dz/dlambda_k = -u^T d_k d_k^T z``).  For a
    scalar weight per series the per-row gradients are summed.
    Returns ``(grad_x, grad_lambda, info)``.
    """
    x3, squeeze = _as3(x)
    g3, _ = _as3(g)
    w = np.asarray(w)
    if z is None:
        z3, info = solve_band(x3, w, lam, d, coef)
    else:
        z3, _ = _as3(z)
        info = None
    u, info_u = solve_band_rhs(g3, w, lam, d, coef)
    if info is None:
        info = info_u
    gx = np.where(w[:, :, None] != 0, u, 0.0)
    gl = -(apply_D(u, d, coef) * apply_D(z3, d, coef)).sum(axis=2)
    lam = np.asarray(lam)
    if lam.ndim <= 1:
        gl = gl.sum(axis=1)
    bad = info != 0
    gx[bad] = np.nan
    gl[bad] = np.nan
    return (gx[:, :, 0] if squeeze else gx), gl, info


def vjp_dense(x: np.ndarray, w: np.ndarray, lam, d: int, g: np.ndarray, coef=None):
    """Same adjoint through explicit dense inverses (tiny T): ``grad_x = W Omega^{-1} g``,
    ``grad_lambda_k = -g^T Omega^{-1} d_k d_k^T z`` (eq. (4), eq. (5))."""
    x3, squeeze = _as3(x)
    g3, _ = _as3(g)
    w = np.asarray(w)
    P, T, C = x3.shape
    Om = omega_dense(w, lam, d, coef)
    Oi = np.linalg.inv(Om)
    z = np.einsum("pts,psc->ptc", Oi, np.where(w[:, :, None] != 0, x3, 0.0))
    gx = np.einsum("pts,psc->ptc", Oi, g3) * (w[:, :, None] != 0)
    D = diff_matrix(T, d, coef)
    gl = np.zeros((P, T - d))
    for p in range(P):
        for k in range(T - d):
            dk = D[k]
            dz = -Oi[p] @ (np.outer(dk, dk) @ z[p])  # eq. (4), (T, C)
            gl[p, k] = np.sum(g3[p] * dz)
    lam = np.asarray(lam)
    if lam.ndim <= 1:
        gl = gl.sum(axis=1)
    return (gx[:, :, 0] if squeeze else gx), gl


# ---------------------------------------------------------------------------
# selected inverse and GCV (lambda selection for the plain form)
# ---------------------------------------------------------------------------


def selinv_band(Lrow: np.ndarray, Dp: np.ndarray) -> np.ndarray:
    """Band of ``Sigma = Omega^{-1}`` from the LDL^T factor.

    ``Sigma = D^{-1} L^{-1} + (I - L^T) Sigma``; for ``s >= t`` (``L^{-1}`` is
    lower triangular) this gives, running ``t`` downwards,
    ``Sigma[t, t+j] = -sum_i L[t+i, t] Sigma[t+i, t+j]`` (``j >= 1``) and
    ``Sigma[t, t] = 1/Dp[t] - sum_i L[t+i, t] Sigma[t+i, t]``.
    Returns ``S[p, i, t] = Sigma[t+i, t]`` (``i = 0..d``).
    """
    P, dp1, T = Lrow.shape
    d = dp1 - 1
    S = np.zeros_like(Lrow)

    def sig(r, s):  # Sigma[r, s] for |r-s| <= d, both already known
        hi, lo = (r, s) if r >= s else (s, r)
        return S[:, hi - lo, lo]

    for t in range(T - 1, -1, -1):
        n = min(d, T - 1 - t)
        for j in range(n, 0, -1):
            acc = np.zeros(P, dtype=Lrow.dtype)
            for i in range(1, n + 1):
                acc -= Lrow[:, i, t + i] * sig(t + i, t + j)
            S[:, j, t] = acc
        acc = 1.0 / Dp[:, t]
        for i in range(1, n + 1):
            acc = acc - Lrow[:, i, t + i] * S[:, i, t]
        S[:, 0, t] = acc
    return S


def posterior_variance(w: np.ndarray, lam, d: int, coef=None):
    """Diagonal of ``Omega^{-1}`` for every series: the pointwise posterior
    variance of ``z`` in units of the observation noise variance (the
    credibility band of Sec. IV-D, Fig. 4, is ``z`` plus or minus a multiple of
    its square root times the noise level).  Taken from the selected inverse of
    the banded LDL^T factor.  Returns ``(var, info)`` with ``var`` of shape
    ``(P, T)``; failed series are NaN.
    """
    w = np.asarray(w)
    AB = omega_band(w, lam, d, coef)
    Lrow, Dp, info = ldl_band(AB)
    info = structural_info(w, d, info)
    var = selinv_band(Lrow, Dp)[:, 0, :].copy()
    var[info != 0] = np.nan
    return var, info


def gcv_scores(x: np.ndarray, w: np.ndarray, grid, d: int):
    """Generalised cross-validation for each scalar weight in ``grid``.

    ``m = sum w``, ``RSS = sum_t w_t (x_t - z_t)^2``, effective dimension
    ``ED = sum_t w_t Sigma[t, t]`` (trace of the hat matrix), and
    ``GCV = m RSS / (m - ED)^2``.  ``x``: ``(P, T)``.  Returns
    ``(scores, ed, rss)`` each of shape ``(P, n_grid)``.
    """
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w)
    P, T = x.shape
    wf = (w != 0).astype(np.float64)
    m = wf.sum(axis=1)
    grid = np.asarray(grid, dtype=np.float64)
    scores = np.zeros((P, grid.size))
    eds = np.zeros((P, grid.size))
    rsss = np.zeros((P, grid.size))
    for gi, lam in enumerate(grid):
        lamv = np.full(P, lam)
        AB = omega_band(w, lamv, d)
        Lrow, Dp, info = ldl_band(AB)
        info = structural_info(w, d, info)
        z = _subst(Lrow, Dp, np.where(wf[:, :, None] != 0, x[:, :, None], 0.0))[:, :, 0]
        S = selinv_band(Lrow, Dp)
        ed = (wf * S[:, 0, :]).sum(axis=1)
        rss = (wf * (x - z) ** 2).sum(axis=1)
        scores[:, gi] = m * rss / (m - ed) ** 2
        eds[:, gi] = ed
        rsss[:, gi] = rss
        scores[info != 0, gi] = np.nan
    return scores, eds, rsss


def gcv_grid(n: int = 21, lo: float = -1.0, step: float = 0.3) -> np.ndarray:
    """The 21-point grid ``10^(-1 + 0.3 i)`` over [1e-1, 1e5]."""
    return 10.0 ** (lo + step * np.arange(n))


def gcv_select(x: np.ndarray, w: np.ndarray, grid, d: int):
    """Per-series argmin of GCV over ``grid``; ties go to the smallest weight.

    Returns ``(lam_best, index, scores)``.
    """
    scores, _, _ = gcv_scores(x, w, grid, d)
    s = np.where(np.isnan(scores), np.inf, scores)
    idx = np.argmin(s, axis=1)  # first minimum = smallest lambda on an ascending grid
    grid = np.asarray(grid, dtype=np.float64)
    return grid[idx], idx, scores


# ---------------------------------------------------------------------------
# checks and metrics
# ---------------------------------------------------------------------------


def backward_error(x: np.ndarray, w: np.ndarray, lam, d: int, z: np.ndarray, coef=None) -> np.ndarray:
    """Componentwise backward error ``max_t |Omega z - W x|_t / (|Omega||z| + |W x|)_t`` per series."""
    x3, _ = _as3(np.asarray(x, dtype=np.float64))
    z3, _ = _as3(np.asarray(z, dtype=np.float64))
    w = np.asarray(w)
    AB = omega_band(w, lam, d, coef)
    P, dp1, T = AB.shape
    b = np.where(w[:, :, None] != 0, x3, 0.0)
    r = -b.copy()
    den = np.abs(b).copy()
    for i in range(dp1):
        a = AB[:, i, :T - i, None]
        # lower part: row t+i, column t
        r[:, i:, :] += a * z3[:, :T - i, :]
        den[:, i:, :] += np.abs(a) * np.abs(z3[:, :T - i, :])
        if i > 0:  # symmetric upper part: row t, column t+i
            r[:, :T - i, :] += a * z3[:, i:, :]
            den[:, :T - i, :] += np.abs(a) * np.abs(z3[:, i:, :])
    with np.errstate(invalid="ignore", divide="ignore"):
        q = np.where(den > 0, np.abs(r) / den, 0.0)
    return q.max(axis=(1, 2))


def rel_err(z: np.ndarray, zref: np.ndarray) -> np.ndarray:
    """Norm-wise error per series ``max_t |z - zref| / max_t |zref|``."""
    z3, _ = _as3(np.asarray(z, dtype=np.float64))
    r3, _ = _as3(np.asarray(zref, dtype=np.float64))
    num = np.abs(z3 - r3).max(axis=(1, 2))
    den = np.abs(r3).max(axis=(1, 2))
    return num / np.where(den > 0, den, 1.0)


# ---------------------------------------------------------------------------
# accuracy of an FP64 result (test metrics, not steps of the method)
# ---------------------------------------------------------------------------


def _band_matvec(AB: np.ndarray, v3: np.ndarray) -> np.ndarray:
    """``Omega v`` per series from lower band storage (symmetric), in the dtype of
    the operands: ``(Omega v)_t = sum_i AB[i, t] v_{t+i} + sum_{i>0} AB[i, t-i] v_{t-i}``."""
    P, dp1, T = AB.shape
    out = AB[:, 0, :, None] * v3
    for i in range(1, dp1):
        a = AB[:, i, :T - i, None]
        out[:, i:, :] += a * v3[:, :T - i, :]
        out[:, :T - i, :] += a * v3[:, i:, :]
    return out


def solve_band_refined(b: np.ndarray, w: np.ndarray, lam, d: int, coef=None, steps: int = 3) -> np.ndarray:
    """``Omega^{-1} b`` close to exact: the banded LDL^T solve (Sec. III-A), then
    iterative refinement (Wilkinson's method: ``v <- v + Omega^{-1}(b - Omega v)``)
    with ``Omega`` assembled and the residual evaluated in numpy's extended
    precision (64-bit significand) and each correction an FP64 LDL^T solve.
    The result (``longdouble``) is accurate to about ``cond(Omega) * 2^-64``,
    far below the error of any FP64 solver on the same system."""
    b3, squeeze = _as3(np.asarray(b, dtype=np.float64))
    w = np.asarray(w)
    AB = omega_band(w, lam, d, coef)
    Lrow, Dp, _ = ldl_band(AB)
    lam_x = np.asarray(lam, dtype=np.longdouble)
    ABx = omega_band(w, lam_x, d, None if coef is None else np.asarray(coef, dtype=np.longdouble))
    v = _subst(Lrow, Dp, b3).astype(np.longdouble)
    bx = b3.astype(np.longdouble)
    for _ in range(steps):
        r = bx - _band_matvec(ABx, v)
        v = v + _subst(Lrow, Dp, r.astype(np.float64)).astype(np.longdouble)
    return v[:, :, 0] if squeeze else v


def solution_error_bound(b: np.ndarray, w: np.ndarray, lam, d: int, v: np.ndarray, coef=None,
                         beta: float | None = None) -> np.ndarray:
    """Per series, the largest norm-wise error ``max_t |v - v*| / max_t |v|`` that
    the componentwise backward error of ``v`` allows, ``v*`` the exact solution of
    ``Omega v* = b``.  With ``beta = max_t |b - Omega v|_t / (|Omega||v| + |b|)_t``
    (residual in extended precision) there are perturbations ``|dOmega| <= beta
    |Omega|``, ``|db| <= beta |b|`` with ``(Omega + dOmega) v = b + db`` (Oettli and
    Prager), hence ``|v - v*| <= beta |Omega^{-1}| (|Omega||v| + |b|)`` exactly.
    A given ``beta`` replaces the measured one (for a ``v`` known only in part,
    the bound is then evaluated at a reference solution).
    ``|Omega^{-1}|`` is formed densely up to T = 4096; beyond, the max-norm of
    ``Omega^{-1} diag(s)`` is estimated by Higham's 1-norm estimator on LAPACK
    banded solves (a lower estimate, so the bound can only come out tighter)."""
    import scipy.linalg
    import scipy.sparse.linalg as spla

    b3, _ = _as3(np.asarray(b, dtype=np.float64))
    v3, _ = _as3(np.asarray(v, dtype=np.float64))
    w = np.asarray(w)
    ABx = omega_band(w, np.asarray(lam, dtype=np.longdouble), d,
                     None if coef is None else np.asarray(coef, dtype=np.longdouble))
    AB = omega_band(w, lam, d, coef)
    P, dp1, T = AB.shape
    r = np.abs(b3.astype(np.longdouble) - _band_matvec(ABx, v3.astype(np.longdouble)))
    s = (_band_matvec(np.abs(ABx), np.abs(v3).astype(np.longdouble)) + np.abs(b3)).astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        be = np.where(s > 0, r.astype(np.float64) / s, 0.0).max(axis=(1, 2))
    if beta is not None:
        be = np.full(P, float(beta))
    out = np.zeros(P)
    for p in range(P):
        sp = s[p].max(axis=1)  # one scale per time step covers every band
        if T <= 4096:
            inv = np.linalg.inv(band_to_dense(AB[p:p + 1])[0])
            g = (np.abs(inv) @ sp).max()
        else:
            def mv(y, p=p, sp=sp):
                return scipy.linalg.solveh_banded(AB[p], sp * np.ravel(y), lower=True)

            def rmv(y, p=p, sp=sp):
                return sp * scipy.linalg.solveh_banded(AB[p], np.ravel(y), lower=True)

            op = spla.LinearOperator((T, T), matvec=mv, rmatvec=rmv, dtype=np.float64)
            g = spla.onenormest(op.H)  # ||M||_inf = ||M^T||_1
        out[p] = be[p] * g / max(np.abs(v3[p]).max(), 1e-300)
    return out


def inverse_diag_refined(w: np.ndarray, lam, d: int, coef=None) -> np.ndarray:
    """``diag(Omega^{-1})`` close to exact: the columns of ``Omega^{-1}`` by
    ``solve_band_refined`` against the identity (small T only)."""
    w = np.asarray(w)
    P, T = w.shape
    eye = np.broadcast_to(np.eye(T), (P, T, T)).copy()
    inv = solve_band_refined(eye, w, lam, d, coef)
    return np.diagonal(inv, axis1=1, axis2=2).astype(np.float64)


def inverse_diag_error_bound(w: np.ndarray, lam, d: int, beta: float, coef=None) -> np.ndarray:
    """Per series, the first-order norm-wise error of ``diag(Omega^{-1})`` under a
    componentwise perturbation ``|dOmega| <= beta |Omega|``: from
    ``d(Omega^{-1}) = -Omega^{-1} dOmega Omega^{-1}``,
    ``|d Sigma_tt| <= beta (|Omega^{-1}| |Omega| |Omega^{-1}|)_tt``, divided by
    ``max_t Sigma_tt`` (dense, small T only)."""
    A = omega_dense(w, lam, d, coef)
    out = np.zeros(A.shape[0])
    for p in range(A.shape[0]):
        inv = np.linalg.inv(A[p])
        ai = np.abs(inv)
        g = np.einsum("ij,jk,ki->i", ai, np.abs(A[p]), ai)
        out[p] = beta * g.max() / np.abs(np.diagonal(inv)).max()
    return out
