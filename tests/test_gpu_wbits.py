"""Weights packed eight to a byte (WHS_W_BITS) give the results of the same calls
with one byte per weight, bit for bit: the same kernels on the same values, so
the oracle parity of the byte calls covers them.  Every order, both storage
types, both weight kinds, series counts that are not a multiple of 64, an
interleave of 128, series whose factorisation fails (the rescan that finds the
failing pivot reads the weights again), and the headline size."""

import numpy as np
import pytest
import torch

from paper_2604_00048_amd import synth, whs
from tests._cases import from_device_rows, from_device_series, random_case, to_device

pytestmark = pytest.mark.gpu
DT = {"f64": torch.float64, "f32": torch.float32}
CASES = [  # P, T, d, S, per_diff, dtype
    (200, 150, 1, 64, True, "f32"), (200, 300, 2, 64, True, "f32"), (131, 500, 3, 128, False, "f64"),
    (70, 260, 4, 64, True, "f64"), (65, 3288, 2, 64, True, "f32"), (300, 1000, 2, 64, False, "f32"),
    (64, 77, 3, 64, True, "f32"), (1, 40, 2, 64, False, "f64"),
]


def both(x, w, lam, S, dtype):
    xt, wt, lt = to_device(x, w, lam, S, dtype)
    return xt, wt, synth.pack_bits(wt), lt


@pytest.mark.parametrize("P,T,d,S,per_diff,dt", CASES)
def test_bits_match_bytes_bit_for_bit(P, T, d, S, per_diff, dt):
    dtype = DT[dt]
    x, w, lam = random_case(P, T, d, per_diff=per_diff, seed=P + 7 * T + d, dtype=dtype)
    if P >= 3:
        w[1] = 0          # no observation: every pivot of the weights' part is 0
        w[2, 1:] = 0      # one observation
    xt, wt, wb, lt = both(x, w, lam, S, dtype)
    z1, i1 = whs.whs_solve(xt, wt, lt, d, P)
    z2, i2 = whs.whs_solve(xt, wb, lt, d, P)
    g = synth.pack_series(torch.tensor(np.random.default_rng(P).normal(size=x.shape), dtype=dtype), S).cuda()
    gx1, gl1, j1 = whs.whs_backward(wt, lt, z1, g, d, P)
    gx2, gl2, j2 = whs.whs_backward(wb, lt, z1, g, d, P)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2) and torch.equal(j1, j2)
    if P >= 3:
        assert int(i1[1].item()) != 0 or int(i1[2].item()) != 0 or d == 1
    # the P series (slots of the last block past P are not written)
    for a, b in [(from_device_series(z1, P), from_device_series(z2, P)),
                 (from_device_series(gx1, P), from_device_series(gx2, P)),
                 (from_device_rows(gl1, P), from_device_rows(gl2, P))]:
        # NaN where a series failed, in both
        np.testing.assert_array_equal(np.isnan(a), np.isnan(b))
        np.testing.assert_array_equal(np.nan_to_num(a), np.nan_to_num(b))


def test_bits_at_the_headline_size():
    # 65,536 series of 3288 days, per-difference weights, FP32 storage: the
    # launch configuration of the benchmark
    P, T, d, S = 65536, 3288, 2, 64
    pk = synth.generate_packed("heteroscedastic", P, S=S, dtype=torch.float32, device="cuda", chunk=8192, T=T, d=d)
    wb = synth.pack_bits(pk.w)
    z1, i1 = whs.whs_solve(pk.x, pk.w, pk.lam, d, P)
    z2, i2 = whs.whs_solve(pk.x, wb, pk.lam, d, P)
    g = torch.randn(pk.x.shape, generator=torch.Generator(device="cuda").manual_seed(3), device="cuda")
    gx1, gl1, _ = whs.whs_backward(pk.w, pk.lam, z1, g, d, P)
    gx2, gl2, _ = whs.whs_backward(wb, pk.lam, z1, g, d, P)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2) and int((i1 != 0).sum().item()) == 0
    assert torch.equal(z1, z2) and torch.equal(gx1, gx2) and torch.equal(gl1, gl2)


def test_bits_through_the_entry_point_that_allocates_nothing():
    P, T, d, S = 300, 700, 2, 64
    x, w, lam = random_case(P, T, d, per_diff=True, seed=11, dtype=torch.float32)
    xt, wt, wb, lt = both(x, w, lam, S, torch.float32)
    z1, i1 = whs.whs_solve(xt, wt, lt, d, P)
    z2, i2 = whs.whs_solve_noalloc(xt, wb, lt, d, P)
    torch.cuda.synchronize()
    assert torch.equal(i1, i2)
    np.testing.assert_array_equal(from_device_series(z1, P), from_device_series(z2, P))
