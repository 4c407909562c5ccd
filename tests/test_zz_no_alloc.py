"""GPU check of whs_solve_noalloc (the entry point that allocates nothing):
through the C ABI it must give what whs_solve gives on the same inputs --
the same kernels run, so bit for bit -- and pass the oracle's bar, on two
calls in a row, the second with a smaller input (the library's scratch array
keeps the first call's contents), in the interleaved and the contiguous
layout."""

import numpy as np
import pytest
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import whs
from tests._cases import assert_solution, from_device_series, random_case, to_device

pytestmark = pytest.mark.gpu


def _pair(P, T, d, per_diff, dtype, S, seed):
    x, w, lam = random_case(P, T, d, per_diff=per_diff, seed=seed, p_obs=0.1, dtype=dtype)
    xt, wt, lt = to_device(x, w, lam, S, dtype)
    print(f"noalloc case P={P} T={T} d={d} per_diff={per_diff} {dtype} S={S}", flush=True)
    z0, i0 = whs.whs_solve(xt, wt, lt, d, P)
    z1 = torch.full_like(xt, float("nan"))
    i1 = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    whs.whs_solve_noalloc(xt, wt, lt, d, P, z=z1, info=i1)
    torch.cuda.synchronize()
    assert torch.equal(i0, i1)
    # live series only: slots of the last block beyond P are never written
    a, b = from_device_series(z0, P), from_device_series(z1, P)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    zref, iref = R.solve_band(x, w, lam, d)
    np.testing.assert_array_equal(i1.cpu().numpy(), iref)
    assert_solution(from_device_series(z1, P), zref, x, w, lam, d, dtype == torch.float64, info=iref)


@pytest.mark.parametrize("S", [64, 1])
def test_noalloc_matches_whs_solve_on_two_calls(S):
    _pair(1000, 1461, 2, True, torch.float32, S, seed=5)     # ragged last block, several tiles
    _pair(130, 365, 3, False, torch.float64, S, seed=6)      # smaller, another order and storage type


def test_noalloc_refuses_more_than_its_scratch():
    P, T, d = 65536, 3288, 2
    x = torch.empty((P // 64, T, 1, 64), dtype=torch.float32, device="cuda")
    w = torch.empty((P // 64, T, 64), dtype=torch.uint8, device="cuda")
    lam = torch.empty((P // 64, T - d, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="unsupported"):
        whs.whs_solve_noalloc(x, w, lam, d, P)
