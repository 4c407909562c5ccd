"""GPU parity of the uneven-batch plan: one persistent launch over groups of
different length and order, its HIP graph replay, and its autotuner."""

import os

import numpy as np
import pytest
import torch

from oracle import whs_ref as R
from paper_2604_00048_amd import synth, whs
from tests._cases import assert_solution

pytestmark = pytest.mark.gpu

SHAPES = [(37, 1, 5), (37, 3, 64), (100, 2, 150), (100, 4, 70), (365, 1, 129), (365, 2, 1), (365, 3, 65)]


def _groups(dtype):
    r = np.random.default_rng(11)
    out = []
    for T, d, n in SHAPES:
        x = r.normal(size=(n, T, 1)) * 0.1 + 0.3
        p = r.uniform(0.05, 0.3, size=(n, 1))
        w = (r.random((n, T)) < p).astype(np.uint8)
        w[:, ::max(T // (d + 2), 1)] = 1
        lam = 10.0 ** r.uniform(-1, 5 if d <= 2 else 3, size=n)
        x = np.where(w[:, :, None] != 0, x, 0.0)
        b = synth.Batch(torch.tensor(x).to(dtype).double(), torch.tensor(w), torch.tensor(lam).to(dtype).double(), d)
        out.append(((T, d), b))
    return out


@pytest.fixture(scope="module")
def f32_case():
    g = _groups(torch.float32)
    x, w, lam, descs = synth.pack_groups(g, dtype=torch.float32, device="cuda")
    return g, x, w, lam, descs


def test_plan_matches_oracle_per_group(f32_case):
    g, x, w, lam, descs = f32_case
    plan = whs.Plan(descs, torch.float32)
    z = torch.zeros_like(x)
    info = torch.full((sum(d["n_series"] for d in descs),), -1, dtype=torch.int32, device="cuda")
    plan.solve(w, lam, x, z, info)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    for ((T, d), b), desc in zip(g, descs):
        zn = synth.unpack_group(z, desc).cpu().double().numpy()
        xn = b.x.numpy()
        zref, _ = R.solve_band(xn, b.w.numpy(), b.lam.numpy(), d)
        assert_solution(zn, zref, xn, b.w.numpy(), b.lam.numpy(), d, f64=False)
    # the plan equals one whs_solve per group, bit for bit
    for ((T, d), b), desc in zip(g, descs):
        xi = synth.pack_series(b.x.to(torch.float32), 64).cuda()
        wi = synth.pack_rows(b.w, 64).cuda()
        zi, _ = whs.whs_solve(xi, wi, b.lam.to(torch.float32).cuda(), d, b.P)
        assert torch.equal(synth.unpack_series(zi, b.P), synth.unpack_group(z, desc))


def test_graph_replay_matches_eager(f32_case):
    g, x, w, lam, descs = f32_case
    plan = whs.Plan(descs, torch.float32)
    z0 = torch.zeros_like(x)
    plan.solve(w, lam, x, z0)
    for k in range(3):
        z = torch.full_like(x, float("nan"))
        plan.graph_launch(w, lam, x, z)
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda", generator=torch.Generator(device="cuda").manual_seed(k)).sum()
        torch.cuda.synchronize()
        for desc in descs:
            assert torch.equal(synth.unpack_group(z, desc), synth.unpack_group(z0, desc)), k
        del junk


def test_autotuner_choices_give_identical_results(f32_case, tmp_path):
    # configurations with the same lanes per series give bitwise-identical z;
    # the tuned one (which may split long series) passes the oracle's bar
    g, x, w, lam, descs = f32_case
    os.environ["WHS_TUNE_CACHE"] = str(tmp_path / "tune.txt")
    try:
        plan = whs.Plan(descs, torch.float32)
        z0 = torch.zeros_like(x)
        plan.solve(w, lam, x, z0)
        for prof, wpb, wps in [(0, 1, 2), (2, 4, 1), (1, 2, 2)]:
            plan.set_config(prof, wpb, wps, 0)
            z = torch.zeros_like(x)
            plan.solve(w, lam, x, z)
            torch.cuda.synchronize()
            for desc in descs:
                assert torch.equal(synth.unpack_group(z, desc), synth.unpack_group(z0, desc)), (prof, wpb, wps)
        cfg = plan.autotune(w, lam, x, torch.zeros_like(x), force=True)
        assert cfg["tile_profile"] in (0, 1, 2) and cfg["waves_per_block"] in (1, 2, 4)
        assert set(cfg["lanes_per_series"]) <= {1, 2}
        z1 = torch.zeros_like(x)
        plan.solve(w, lam, x, z1)
        torch.cuda.synchronize()
        for ((T, d), b), desc in zip(g, descs):
            zn = synth.unpack_group(z1, desc).cpu().double().numpy()
            zref, _ = R.solve_band(b.x.numpy(), b.w.numpy(), b.lam.numpy(), d)
            assert_solution(zn, zref, b.x.numpy(), b.w.numpy(), b.lam.numpy(), d, f64=False)
        assert (tmp_path / "tune.txt").exists()
        plan2 = whs.Plan(descs, torch.float32)      # picks the cached choice at creation
        assert plan2.config() == cfg
    finally:
        os.environ.pop("WHS_TUNE_CACHE", None)


# lengths around tile multiples and both parities, every order
SPLIT_SHAPES = [(64, 1, 70), (65, 2, 64), (77, 3, 10), (100, 4, 65), (129, 2, 128), (200, 3, 63), (257, 1, 64),
                (365, 2, 130), (366, 4, 64)]


def _split_groups(dtype, per_diff, seed):
    r = np.random.default_rng(seed)
    out = []
    for T, d, n in SPLIT_SHAPES:
        x = r.normal(size=(n, T, 1)) * 0.1 + 0.3
        p = r.uniform(0.05, 0.3, size=(n, 1))
        w = (r.random((n, T)) < p).astype(np.uint8)
        w[:, ::max(T // (d + 2), 1)] = 1
        hi = 4 if d <= 2 else 3
        lam = 10.0 ** r.uniform(-1, hi, size=(n, T - d) if per_diff else n)
        x = np.where(w[:, :, None] != 0, x, 0.0)
        b = synth.Batch(torch.tensor(x).to(dtype).double(), torch.tensor(w), torch.tensor(lam).to(dtype).double(), d)
        out.append(((T, d), b))
    return out


def _check_groups(groups, descs, z, info, f64):
    info = info.cpu().numpy()
    for ((T, d), b), desc in zip(groups, descs):
        xn, wn, ln = b.x.numpy(), b.w.numpy(), b.lam.numpy()
        zref, iref = R.solve_band(xn, wn, ln, d)
        got = info[desc["info_off"]:desc["info_off"] + b.P]
        np.testing.assert_array_equal(got, iref)
        zn = synth.unpack_group(z, desc).cpu().double().numpy()
        assert_solution(zn, zref, xn, wn, ln, d, f64=f64, info=iref)


@pytest.mark.parametrize("prof", [0, 2])
@pytest.mark.parametrize("dt,per_diff", [(torch.float32, False), (torch.float32, True), (torch.float64, False),
                                         (torch.float64, True)])
def test_two_lanes_per_series_match_oracle(dt, per_diff, prof):
    groups = _split_groups(dt, per_diff, seed=5 + prof)
    x, w, lam, descs = synth.pack_groups(groups, dtype=dt, device="cuda")
    plan = whs.Plan(descs, dt, per_diff=per_diff)
    for split_T in (64, 200):              # every group split; long ones split, short ones whole in one launch
        plan.set_config(prof, 2, 1, split_T)
        lanes = plan.config()["lanes_per_series"]
        assert lanes == [2 if T >= split_T else 1 for (T, d), _ in groups]
        z = torch.full_like(x, float("nan"))
        info = torch.full((sum(dd["n_series"] for dd in descs),), -1, dtype=torch.int32, device="cuda")
        print(f"two-lane plan: {dt} per_diff={per_diff} profile {prof} split_T {split_T}", flush=True)
        plan.solve(w, lam, x, z, info)
        torch.cuda.synchronize()
        _check_groups(groups, descs, z, info, dt == torch.float64)
    plan.close()


def test_two_lanes_failures_are_reported_in_time_order():
    dt = torch.float64
    groups = _split_groups(dt, True, seed=9)
    (T, d), b = groups[7]                                   # T = 365, d = 2
    b.w[3] = 0
    b.w[3, 200] = 1                                         # one observation: singular
    b.x[3] = 0
    b.lam[5, 40] = -1e6                                     # indefinite early (top part)
    b.lam[6, 300] = -1e6                                    # indefinite late (bottom part)
    b.lam[7, 181] = float("nan")                            # at the separator
    x, w, lam, descs = synth.pack_groups(groups, dtype=dt, device="cuda")
    plan = whs.Plan(descs, dt, per_diff=True)
    plan.set_config(1, 2, 2, 64)
    z = torch.zeros_like(x)
    info = torch.full((sum(dd["n_series"] for dd in descs),), -1, dtype=torch.int32, device="cuda")
    plan.solve(w, lam, x, z, info)
    torch.cuda.synchronize()
    _check_groups(groups, descs, z, info, True)
    zg = synth.unpack_group(z, descs[7]).cpu().numpy()
    ig = info.cpu().numpy()[descs[7]["info_off"]:descs[7]["info_off"] + b.P]
    assert ig[3] == T and (ig[[5, 6, 7]] > 0).all()
    assert np.isnan(zg[[3, 5, 6, 7]]).all()
    plan.close()


def test_two_lane_graph_replay_matches_eager():
    groups = _split_groups(torch.float32, False, seed=12)
    x, w, lam, descs = synth.pack_groups(groups, dtype=torch.float32, device="cuda")
    plan = whs.Plan(descs, torch.float32)
    plan.set_config(2, 2, 1, 100)
    z0 = torch.zeros_like(x)
    plan.solve(w, lam, x, z0)
    for k in range(3):
        z = torch.full_like(x, float("nan"))
        plan.graph_launch(w, lam, x, z)
        junk = torch.randn(1 << 20, device="cuda", generator=torch.Generator(device="cuda").manual_seed(k)).sum()
        torch.cuda.synchronize()
        for desc in descs:
            assert torch.equal(synth.unpack_group(z, desc), synth.unpack_group(z0, desc)), k
        del junk
    plan.close()


def test_set_config_rejects_bad_choices():
    groups = _split_groups(torch.float32, False, seed=1)[:2]
    _, _, _, descs = synth.pack_groups(groups, dtype=torch.float32, device="cuda")
    plan = whs.Plan(descs, torch.float32)
    for bad in [(3, 1, 1, 0), (0, 3, 1, 0), (0, 1, 3, 0), (0, 4, 1, 64), (0, 2, 1, -1)]:
        with pytest.raises(RuntimeError, match="invalid argument"):
            plan.set_config(*bad)
    plan.close()


def test_plan_f64_per_difference():
    r = np.random.default_rng(3)
    groups = []
    for T, d, n in [(80, 2, 70), (50, 1, 10), (120, 3, 64)]:
        x = r.normal(size=(n, T, 1))
        w = (r.random((n, T)) < 0.3).astype(np.uint8)
        w[:, ::max(T // (d + 2), 1)] = 1
        lam = 10.0 ** r.uniform(0, 3, size=(n, T - d))
        x = np.where(w[:, :, None] != 0, x, 0.0)
        groups.append(((T, d), synth.Batch(torch.tensor(x), torch.tensor(w), torch.tensor(lam), d)))
    x, w, lam, descs = synth.pack_groups(groups, dtype=torch.float64, device="cuda")
    plan = whs.Plan(descs, torch.float64, per_diff=True)
    z = plan.solve(w, lam, x, torch.zeros_like(x))
    torch.cuda.synchronize()
    for ((T, d), b), desc in zip(groups, descs):
        zn = synth.unpack_group(z, desc).cpu().numpy()
        zref, _ = R.solve_band(b.x.numpy(), b.w.numpy(), b.lam.numpy(), d)
        assert_solution(zn, zref, b.x.numpy(), b.w.numpy(), b.lam.numpy(), d, f64=True)
