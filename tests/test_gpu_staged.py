"""Series-contiguous calls (interleave 1) given the workspace of
whs_interleave_workspace_bytes run the interleaved kernels on copies.  Their
results must be bit-identical to the same call on interleaved tensors (the same
kernels on the same values), which the oracle parity of the interleaved path
then covers: every order, several bands (beyond the partition kernel's one),
both weight kinds, both storage types, the adjoint, a series count that is not
a multiple of 64, the uneven-date calls, which take the contiguous layout
only this way, GCV and the posterior variance, and arrays and workspaces whose
addresses make the copies take their narrower accesses."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2604_00048_amd import synth, whs
from tests._cases import from_device_rows, from_device_series, random_case, to_device

pytestmark = pytest.mark.gpu
DT = {"f64": torch.float64, "f32": torch.float32}
CASES = [  # P, T, d, C, per_diff
    (70, 300, 1, 1, True), (65, 500, 2, 3, False), (33, 350, 3, 1, True), (64, 260, 4, 2, True),
    (130, 3288, 2, 1, True), (5, 40, 2, 10, False),
]


def both_layouts(x, w, lam, dtype):
    return to_device(x, w, lam, 64, dtype), to_device(x, w, lam, 1, dtype)


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("P,T,d,C,per_diff", CASES)
def test_contiguous_calls_match_interleaved_bit_for_bit(P, T, d, C, per_diff, dt):
    dtype = DT[dt]
    x, w, lam = random_case(P, T, d, C=C, per_diff=per_diff, seed=P + T + d + C, dtype=dtype)
    (x64, w64, l64), (x1, w1, l1) = both_layouts(x, w, lam, dtype)
    z64, i64 = whs.whs_solve(x64, w64, l64, d, P)
    z1, i1 = whs.whs_solve(x1, w1, l1, d, P)
    g = torch.tensor(np.random.default_rng(P * 3 + C).normal(size=x.shape), dtype=dtype)
    gx64, gl64, _ = whs.whs_backward(w64, l64, z64, synth.pack_series(g, 64).cuda(), d, P)
    gx1, gl1, _ = whs.whs_backward(w1, l1, z1, synth.pack_series(g, 1).cuda(), d, P)
    _, gl1n, _ = whs.whs_backward(w1, l1, z1, synth.pack_series(g, 1).cuda(), d, P, need_x=False)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(from_device_rows(gl1n, P), from_device_rows(gl64, P))   # grad_x not requested
    np.testing.assert_array_equal(i1.cpu().numpy(), i64.cpu().numpy())
    np.testing.assert_array_equal(from_device_series(z1, P), from_device_series(z64, P))
    np.testing.assert_array_equal(from_device_series(gx1, P), from_device_series(gx64, P))
    np.testing.assert_array_equal(from_device_rows(gl1, P), from_device_rows(gl64, P))


@pytest.mark.parametrize("d,C", [(1, 1), (2, 4), (3, 1)])
def test_uneven_dates_contiguous_match_interleaved(d, C):
    P, T, dtype = 77, 300, torch.float32
    x, w, lam = random_case(P, T, d, C=C, per_diff=True, seed=31 * d + C, dtype=dtype)
    times = 3.0 + np.cumsum(np.random.default_rng(d).integers(1, 4, size=T)).astype(np.float64)
    coef = whs.whs_diff_coef(torch.tensor(times, device="cuda"), d)
    (x64, w64, l64), (x1, w1, l1) = both_layouts(x, w, lam, dtype)
    z64, _ = whs.whs_solve(x64, w64, l64, d, P, coef=coef)
    z1, _ = whs.whs_solve(x1, w1, l1, d, P, coef=coef)
    g = torch.tensor(np.random.default_rng(5).normal(size=x.shape), dtype=dtype)
    gx64, gl64, _ = whs.whs_backward(w64, l64, z64, synth.pack_series(g, 64).cuda(), d, P, coef=coef)
    gx1, gl1, _ = whs.whs_backward(w1, l1, z1, synth.pack_series(g, 1).cuda(), d, P, coef=coef)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(from_device_series(z1, P), from_device_series(z64, P))
    np.testing.assert_array_equal(from_device_series(gx1, P), from_device_series(gx64, P))
    np.testing.assert_array_equal(from_device_rows(gl1, P), from_device_rows(gl64, P))
    # without the larger workspace the uneven-date calls refuse the contiguous layout
    with pytest.raises(RuntimeError):
        whs.whs_solve(x1, w1, l1, d, P, coef=coef, staged=False)


def _at_offset(t, k):
    """The values of t at a storage offset of k elements (the data pointer then
    loses its 16-byte alignment unless k elements make 16 bytes)."""
    buf = torch.zeros(t.numel() + k, dtype=t.dtype, device=t.device)
    v = buf[k:].view(t.shape)
    v.copy_(t)
    return v


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("k_x,k_w,ws_off", [(1, 1, 0), (2, 4, 0), (0, 0, 8), (1, 3, 8)])
def test_contiguous_calls_at_unaligned_addresses(dt, k_x, k_w, ws_off):
    # where a contiguous array does not start 16-byte aligned the copies take
    # narrower accesses, and where the workspace (8-byte aligned is allowed)
    # puts the interleaved copies off 16 bytes they take one element per
    # access: the same results, bit for bit
    dtype = DT[dt]
    P, T, d = 70, 300, 2
    x, w, lam = random_case(P, T, d, per_diff=True, seed=9 + k_x, dtype=dtype)
    (x64, w64, l64), (x1, w1, l1) = both_layouts(x, w, lam, dtype)
    xo, wo, lo = _at_offset(x1, k_x), _at_offset(w1, k_w), _at_offset(l1, k_x)
    desc = whs.make_desc(P, T, d, 1, 1, whs.WHS_F64 if dt == "f64" else whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    n = int(whs.lib().whs_interleave_workspace_bytes(ctypes.byref(desc)))
    assert n > 0
    ws = torch.empty(n + 256, dtype=torch.uint8, device="cuda")[ws_off:ws_off + n]
    z64, i64 = whs.whs_solve(x64, w64, l64, d, P)
    zo, io = whs.whs_solve(xo, wo, lo, d, P, z=_at_offset(torch.zeros_like(x1), k_x), workspace=ws)
    g = torch.tensor(np.random.default_rng(3).normal(size=x.shape), dtype=dtype)
    g64, g1 = synth.pack_series(g, 64).cuda(), _at_offset(synth.pack_series(g, 1).cuda(), k_x)
    gx64, gl64, _ = whs.whs_backward(w64, l64, z64, g64, d, P)
    gxo, glo = _at_offset(torch.zeros_like(x1), k_x), _at_offset(torch.zeros_like(l1), k_x)
    whs.whs_backward(wo, lo, zo, g1, d, P, grad_x=gxo, grad_lambda=glo, workspace=ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(io.cpu().numpy(), i64.cpu().numpy())
    np.testing.assert_array_equal(from_device_series(zo, P), from_device_series(z64, P))
    np.testing.assert_array_equal(from_device_series(gxo, P), from_device_series(gx64, P))
    np.testing.assert_array_equal(from_device_rows(glo, P), from_device_rows(gl64, P))


GCV_GRID = 10.0 ** (-1 + 0.3 * np.arange(21))


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("P,T,d", [(70, 300, 2), (33, 350, 1), (130, 97, 3), (5, 40, 4)])
def test_gcv_contiguous_matches_interleaved(P, T, d, dt):
    dtype = DT[dt]
    x, w, _ = random_case(P, T, d, per_diff=False, seed=P + T, dtype=dtype)
    (x64, w64, _), (x1, w1, _) = both_layouts(x, w, np.ones(P), dtype)
    grid = torch.tensor(GCV_GRID, device="cuda")
    lb64, sc64, i64 = whs.whs_gcv(x64, w64, grid, d, P, want_scores=True)
    lb1, sc1, i1 = whs.whs_gcv(x1, w1, grid, d, P, want_scores=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(i1.cpu().numpy(), i64.cpu().numpy())
    np.testing.assert_array_equal(lb1.cpu().numpy(), lb64.cpu().numpy())
    np.testing.assert_array_equal(sc1.cpu().numpy(), sc64.cpu().numpy())


@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("per_diff", [True, False])
@pytest.mark.parametrize("P,T,d", [(70, 300, 2), (33, 350, 1), (130, 97, 3), (5, 40, 4)])
def test_variance_contiguous_matches_interleaved(P, T, d, per_diff, dt):
    dtype = DT[dt]
    x, w, lam = random_case(P, T, d, per_diff=per_diff, seed=2 * P + T, dtype=dtype)
    (_, w64, l64), (_, w1, l1) = both_layouts(x, w, lam, dtype)
    v64, i64 = whs.whs_variance(w64, l64, d, P)
    v1, i1 = whs.whs_variance(w1, l1, d, P)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(i1.cpu().numpy(), i64.cpu().numpy())
    np.testing.assert_array_equal(from_device_series(v1, P), from_device_series(v64, P))
