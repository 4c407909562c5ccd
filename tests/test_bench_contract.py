"""The measurement script's contract, checked without a GPU: one GPU only (a
larger --gpus exits with a message and status 2), the algorithmic bytes behind
``roofline.achieved`` (every API tensor once per pass at its storage type), and
the traffic figures keyed to the sources of the kernels they were measured on."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_bytes_per_series():
    # headline: T = 3288, d = 2, one band, FP32, one weight per difference row
    fwd, bwd = bench.alg_bytes(3288, 2, 1, 4, True)
    assert fwd == 4 * 3288 + 3288 + 4 * 3286 + 4 * 3288 == 42736
    assert bwd == 3 * 4 * 3288 + 3288 + 2 * 4 * 3286 == 69032          # g, z, grad_x; w; lambda, grad_lambda
    # scalar weight: one value per series in and out
    fwd, bwd = bench.alg_bytes(365, 2, 10, 8, False)
    assert fwd == 2 * 8 * 365 * 10 + 365 + 8
    assert bwd == 3 * 8 * 365 * 10 + 365 + 2 * 8


def test_traffic_is_keyed_to_the_kernel_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    h = bench.kernel_source_hash()
    assert len(h) == 16
    for key, v in rec.items():
        assert v["bytes_per_launch"] > 0 and v["read_bytes"] + v["write_bytes"] == v["bytes_per_launch"]
    # a figure is reported only while it describes the current sources
    for kernel in ("whs_solve", "whs_backward"):
        t = bench.measured_traffic(kernel, "heteroscedastic P=65536 T=3288 d=2 C=1")
        stored = rec[f"{kernel}|heteroscedastic P=65536 T=3288 d=2 C=1"]
        assert (t is not None) == (stored["source_hash"] == h)


def _fake_rocprof(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "1234_counter_collection.csv"), "w") as f:
        f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},"{k}",{c},{v}\n')


def test_counter_ingest_scales_by_the_copy_calibration(tmp_path, monkeypatch, capsys):
    solve = "void whs::k_fast<2, 1, 24, float, false, true, false, false>(whs::FastArgs)"
    back = "void whs::k_fast<2, 1, 24, float, true, true, false, false>(whs::FastArgs)"
    _fake_rocprof(tmp_path / "f", [(solve, "FETCH_SIZE", 1000.0), (solve, "FETCH_SIZE", 3000.0),
                                   (back, "FETCH_SIZE", 4000.0)])
    _fake_rocprof(tmp_path / "w", [(solve, "WRITE_SIZE", 500.0), (back, "WRITE_SIZE", 700.0)])
    _fake_rocprof(tmp_path / "cf", [("void copy_kernel<float>", "FETCH_SIZE", 131072.0)])  # half of 256 MiB
    _fake_rocprof(tmp_path / "cw", [("void copy_kernel<float>", "WRITE_SIZE", 262144.0)])
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0123456789abcdef")
    bench.ingest_counters(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                          P=65536, T=3288, d=2)
    rec = json.load(open(tmp_path / "profiles" / "traffic.json"))
    s = rec["whs_solve|heteroscedastic P=65536 T=3288 d=2 C=1"]
    assert s["fetch_scale"] == 2.0 and s["write_scale"] == 1.0
    assert s["read_bytes"] == 2.0 * 2000.0 * 1024 and s["write_bytes"] == 500.0 * 1024
    b = rec["whs_backward|heteroscedastic P=65536 T=3288 d=2 C=1"]
    assert b["bytes_per_launch"] == 2.0 * 4000.0 * 1024 + 700.0 * 1024
    assert s["source_hash"] == "0123456789abcdef"


def test_holdout_split_is_a_seeded_subset_of_the_observed_points():
    import torch
    from paper_2604_00048_amd import synth
    g = torch.Generator().manual_seed(3)
    w = (torch.rand((64, 3288), generator=g) < 0.08).to(torch.uint8)
    a = synth.holdout_split(w, 0.1, torch.Generator().manual_seed(9))
    b = synth.holdout_split(w, 0.1, torch.Generator().manual_seed(9))
    assert torch.equal(a, b)
    assert ((a != 0) <= (w != 0)).all()
    frac = a.sum().item() / w.sum().item()
    assert abs(frac - 0.1) < 0.015, frac          # about 16,800 observed points


def test_learned_batches_take_the_layout_of_their_size():
    # training batches (a few thousand series) are series-contiguous, evaluation
    # chunks interleaved; the same seed gives the same series in either layout
    import torch
    from paper_2604_00048_amd import learned, synth
    assert learned.layout_for(4096) == 1 and learned.layout_for(learned.SMALL_BATCH) == 1
    assert learned.layout_for(learned.SMALL_BATCH + 1) == 64 and learned.layout_for(65536) == 64
    a = learned.make_batch(70, 5, 0, "cpu", T=120)
    b = learned.make_batch(70, 5, 0, "cpu", T=120, S=64)
    assert a.S == 1 and b.S == 64 and tuple(a.x_train.shape) == (70, 120, 1, 1)
    assert torch.equal(synth.unpack_series(a.x_train, 70), synth.unpack_series(b.x_train, 70))
    assert torch.equal(synth.unpack_rows(a.w_train, 70), synth.unpack_rows(b.w_train, 70))
    assert torch.equal(synth.unpack_rows(a.hold, 70), synth.unpack_rows(b.hold, 70))
    assert a.n_hold == b.n_hold > 0
