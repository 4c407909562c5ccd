"""GPU parity of whs_gcv (grid search of a scalar weight by GCV) against the oracle."""

import numpy as np
import pytest
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import synth, whs
from tests._cases import random_case, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("P,T,d", [(100, 365, 2), (70, 120, 1), (64, 97, 3), (65, 60, 4)])
def test_gcv_scores_and_choice(P, T, d, dt):
    x, w, _ = random_case(P, T, d, per_diff=False, seed=P + T + d, p_obs=0.25, dtype=dt)
    # smooth signal plus noise so the criterion has an interior minimum
    t = np.arange(T) / T
    x = np.where(w != 0, (0.3 + 0.2 * np.sin(6 * t))[None, :] + 0.05 * x[:, :, 0], 0.0)
    x = torch.tensor(x).to(dt).double().numpy()
    grid = R.gcv_grid()
    xt, wt, _ = to_device(x[:, :, None], w, np.ones(P), 64, dt)
    gt = torch.tensor(grid, device="cuda")
    lb, sc, info = whs.whs_gcv(xt, wt, gt, d, P, want_scores=True)
    torch.cuda.synchronize()
    sc = sc.cpu().numpy()
    ref, ed, rss = R.gcv_scores(x, w, grid, d)
    ok = np.isfinite(ref)
    rel = np.abs(sc[ok] - ref[ok]) / np.abs(ref[ok])
    assert rel.max() < 1e-7, rel.max()
    # the chosen weight attains the minimum (first one on ties)
    idx = np.array([np.argmin(np.where(np.isnan(r), np.inf, r)) for r in sc])
    np.testing.assert_array_equal(lb.cpu().double().numpy(), torch.tensor(grid[idx]).to(dt).double().numpy())
    ref_best = np.nanmin(ref, axis=1)
    assert (ref[np.arange(P), idx] <= ref_best * (1 + 1e-9)).all()
    assert (info.cpu().numpy() == 0).all()


def test_gcv_failed_series_and_ties():
    P, T, d = 64, 50, 2
    x, w, _ = random_case(P, T, d, per_diff=False, seed=5)
    w[3] = 0
    w[3, 10] = 1                      # one observation: singular for every weight
    x[7, :, 0] = 0.0                  # z = 0 exactly: every score is exactly 0, a true tie
    grid = R.gcv_grid()
    xt, wt, _ = to_device(x, w, np.ones(P), 64, torch.float64)
    lb, sc, info = whs.whs_gcv(xt, wt, torch.tensor(grid, device="cuda"), d, P, want_scores=True)
    torch.cuda.synchronize()
    lb = lb.cpu().numpy()
    assert np.isnan(lb[3]) and info.cpu().numpy()[3] > 0
    assert (sc.cpu().numpy()[7] == 0).all() and lb[7] == grid[0]
    ref_l, ref_i, ref_s = R.gcv_select(x[:, :, 0], w, grid, d)
    keep = np.arange(P) != 3
    np.testing.assert_array_equal(lb[keep], ref_l[keep])
