"""The C-ABI library loads and exports every declared symbol; host-side
argument checks reject bad calls before anything is launched (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_2604_00048_amd import whs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(whs_[a-z_0-9]+)\s*\(", src)))


def test_library_built():
    assert os.path.exists(whs.LIB_PATH), "run __graft_entry__.build() first"


def test_library_matches_the_sources():
    # the binding refuses a library built from other sources; the id is the source hash
    from paper_2604_00048_amd.build import source_hash
    assert whs.build_id() == source_hash()
    assert len(whs.build_id()) == 16


def test_every_declared_symbol_is_exported():
    from paper_2604_00048_amd import net
    L = whs.lib()
    names = _declared("whs.h")
    assert {"whs_solve", "whs_backward", "whs_factor", "whs_status_str", "whs_gcv", "whs_plan_create"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
        assert n in whs.SIGNATURES, f"binding lacks {n}"
    for n in _declared("whs_net.h"):
        assert hasattr(L, n), n
        assert n in net.NET_SIGNATURES, f"binding lacks {n}"
    net.lib()  # every signature binds
    from paper_2604_00048_amd import tf
    for n in _declared("whs_tf.h"):
        assert hasattr(L, n), n
        assert n in tf.TF_SIGNATURES, f"binding lacks {n}"
    assert set(tf.TF_SIGNATURES) == set(_declared("whs_tf.h"))
    tf.lib()


def test_status_strings_and_version():
    assert whs.lib().whs_version() >= 100
    for code in (0, -1, -2, -3, -4):
        assert whs.status_str(code) != "unknown status"
    assert whs.status_str(-99) == "unknown status"


def _solve_raw(desc, w=None, lam=None, x=None, z=None, ws=None, nws=0):
    L = whs.lib()
    return L.whs_solve(ctypes.byref(desc), w, lam, None, x, z, None, ws, nws, None)


FAKE = ctypes.c_void_p(1 << 20)          # never dereferenced: checks fail first
FAKE_ODD = ctypes.c_void_p((1 << 20) + 2)


@pytest.mark.parametrize("bad", [
    dict(T=2, d=2),          # T <= d
    dict(d=0),
    dict(n_rhs=0),
    dict(interleave=0),
    dict(dtype=7),
    dict(lambda_kind=3),
    dict(n_series=-1),
])
def test_descriptor_validation(bad):
    kw = dict(n_series=10, T=50, d=2, n_rhs=1, interleave=64, dtype=0, lambda_kind=0)
    kw.update(bad)
    desc = whs.make_desc(kw["n_series"], kw["T"], kw["d"], kw["n_rhs"], kw["interleave"], kw["dtype"],
                         kw["lambda_kind"])
    assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30) == -1


def test_order_above_four_is_unsupported():
    desc = whs.make_desc(10, 50, 5, 1, 64, 0, 0)
    assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30) == -2


@pytest.mark.parametrize("P,T,d,C,S,dt", [
    (262144, 3288, 2, 10, 262144, 0),    # the ten-band batch as one block: 34 GB of x per block
    (262144, 3288, 2, 1, 262144, 0),     # one band: 3.4 GB of x, 2.9 GB of checkpoints per block
    (1048576, 3288, 2, 1, 1048576, 0),
    (640, 100000, 4, 5, 640, 1),         # long many-band series: x and checkpoints past 2 GiB per block
])
def test_blocks_past_32_bit_ranges_are_unsupported(P, T, d, C, S, dt):
    # the fast kernels address one block through 32-bit buffer ranges, with byte
    # offset 2^31 marking padding lanes: such descriptors are refused, never run
    L = whs.lib()
    desc = whs.make_desc(P, T, d, C, S, dt, 1)
    assert whs.workspace_bytes(desc) == 0
    assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 40) == -2
    assert L.whs_backward(ctypes.byref(desc), FAKE, FAKE, None, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 40,
                          None) == -2
    assert L.whs_solve_coef(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 40, None) == -2
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, FAKE, 1 << 40, None) == -2
    # the same batch in blocks of 64 series is accepted
    ok = whs.make_desc(P, T, d, C, 64, dt, 1)
    assert whs.workspace_bytes(ok) > 0


def test_block_range_limit_edges():
    # one block of S = 2^16 series at T = 8192 in FP32: x is exactly 2^31 bytes (refused);
    # at T = 4000 every per-block array is below 2^31 bytes, checkpoints included (accepted)
    assert whs.workspace_bytes(whs.make_desc(65536, 8192, 1, 1, 65536, 0, 0)) == 0
    assert whs.workspace_bytes(whs.make_desc(65536, 4000, 1, 1, 65536, 0, 0)) > 0
    # plan groups: 64-series blocks of very long series are refused as well
    h = ctypes.c_void_p()
    g = (whs.WhsGroup * 1)(whs.WhsGroup(64, 1 << 21, 2, 0, 0, 0, 0))
    assert whs.lib().whs_plan_create(ctypes.byref(h), g, 1, 1, 0, 0, 64) == -2


def test_null_and_misaligned_pointers():
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 0)
    assert _solve_raw(desc, None, FAKE, FAKE, FAKE, FAKE, 1 << 30) == -1
    assert _solve_raw(desc, FAKE, None, FAKE, FAKE, FAKE, 1 << 30) == -1   # no lambda and no factor
    assert _solve_raw(desc, FAKE, FAKE, FAKE_ODD, FAKE, FAKE, 1 << 30) == -1
    assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, None, 0) == -4          # workspace missing
    need = whs.workspace_bytes(desc)
    assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, FAKE, need - 8) == -4


def test_empty_batch_is_a_noop():
    desc = whs.make_desc(0, 50, 2, 1, 64, 0, 0)
    assert whs.workspace_bytes(desc) == 0
    assert _solve_raw(desc) == 0
    L = whs.lib()
    assert L.whs_backward(ctypes.byref(desc), None, None, None, None, None, None, None, None, None, 0, None) == 0
    assert L.whs_factor(ctypes.byref(desc), None, None, None, None, None) == 0
    # every entry point, both layouts it accepts: no pointer is read and no launch made
    for S in (64, 1):
        e = whs.make_desc(0, 50, 2, 1, S, 0, 0)
        assert L.whs_solve_coef(ctypes.byref(e), None, None, None, None, None, None, None, 0, None) == 0
        assert L.whs_backward_coef(ctypes.byref(e), None, None, None, None, None, None, None, None, None, 0,
                                   None) == 0
        assert L.whs_interleave_workspace_bytes(ctypes.byref(e)) == 0
        assert L.whs_gcv(ctypes.byref(e), None, None, None, 21, None, None, None, None, 0, None) == 0
        assert L.whs_variance(ctypes.byref(e), None, None, None, None, None, 0, None) == 0
        assert L.whs_gcv_workspace_bytes(ctypes.byref(e)) == 0
        assert L.whs_variance_workspace_bytes(ctypes.byref(e)) == 0
    assert L.whs_solve_coef(ctypes.byref(whs.make_desc(0, 50, 2, 1, 32, 0, 0)), None, None, None, None, None,
                            None, None, 0, None) == -2                                  # layout still checked
    assert L.whs_gcv(ctypes.byref(desc), None, None, None, 21, None, None, None, None, 0, None) == 0
    assert L.whs_variance(ctypes.byref(desc), None, None, None, None, None, 0, None) == 0
    assert L.whs_gcv_workspace_bytes(ctypes.byref(desc)) == 0
    assert L.whs_variance_workspace_bytes(ctypes.byref(desc)) == 0


def test_workspace_and_factor_sizes():
    # order 2, one band: 2 + 1 + 2 = 5 doubles per tile per series; the largest
    # user is the uneven-time adjoint with a weight per difference row, whose
    # tiles are 12 steps
    desc = whs.make_desc(100, 365, 2, 1, 64, 0, 1)
    tiles = (365 + 11) // 12
    assert whs.workspace_bytes(desc) == 2 * tiles * 5 * 64 * 8
    assert whs.lib().whs_factor_bytes(ctypes.byref(desc)) == 128 * 3 * 365 * 8


def test_interleave_workspace_size():
    # series-contiguous calls: slots for x/g, z, grad_x (3 x), w, lambda and
    # grad_lambda (per difference row), each rounded up to 256 bytes, then the
    # checkpoints of the same call on interleave 64
    L = whs.lib()
    up = lambda n: (n + 255) // 256 * 256   # noqa: E731
    for P, T, d, C, dt, kind in [(100, 365, 2, 1, 0, 1), (65, 3288, 3, 4, 1, 0), (1, 10, 1, 2, 0, 1)]:
        desc = whs.make_desc(P, T, d, C, 1, dt, kind)
        e = 8 if dt == 1 else 4
        nb = (P + 63) // 64
        x = up(nb * 64 * T * C * e)
        lam = up(nb * 64 * (T - d) * e) if kind == 1 else 0
        ck = whs.workspace_bytes(whs.make_desc(P, T, d, C, 64, dt, kind))
        n = L.whs_interleave_workspace_bytes(ctypes.byref(desc))
        assert n == 3 * x + up(nb * 64 * T) + 2 * lam + ck
        assert n >= whs.workspace_bytes(desc)
    assert L.whs_interleave_workspace_bytes(ctypes.byref(whs.make_desc(100, 365, 2, 1, 64, 0, 1))) == 0
    assert L.whs_interleave_workspace_bytes(ctypes.byref(whs.make_desc(0, 365, 2, 1, 1, 0, 1))) == 0
    # the copies' grids count at most 2^32 - 1 work-items of 256 per workgroup, one
    # workgroup per 64 series and 256 bytes of their rows: beyond that the
    # contiguous layout is refused this way (0), not launched
    big = lambda P, T, dt: L.whs_interleave_workspace_bytes(ctypes.byref(whs.make_desc(P, T, 2, 1, 1, dt, 1)))  # noqa: E731
    assert big(2 ** 30, 365, 0) == 0                    # 2^24 series blocks
    assert big(2 ** 24, 3288, 1) == 0 and big(2 ** 24, 3288, 0) > 0   # FP64 rows take twice the tiles
    assert big(64 * (2 ** 24 - 1), 31, 0) == 0 and big(64 * (2 ** 24 - 8), 31, 0) > 0


def test_backward_validation():
    L = whs.lib()
    desc = whs.make_desc(10, 50, 2, 1, 64, 1, 1)
    ws = 1 << 30
    assert L.whs_backward(ctypes.byref(desc), FAKE, FAKE, None, None, FAKE, FAKE, FAKE, None, FAKE, ws, None) == -1
    assert L.whs_backward(ctypes.byref(desc), FAKE, FAKE, None, FAKE, FAKE, FAKE_ODD, None, None, FAKE, ws,
                          None) == -1


def test_binding_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    x = torch.zeros((1, 10, 1, 64))
    w = torch.zeros((1, 10, 64), dtype=torch.uint8)
    with pytest.raises(ValueError):
        whs.whs_solve(x, w, torch.ones(64), 2)


def test_gcv_validation():
    L = whs.lib()
    g = ctypes.c_void_p(1 << 20)
    desc = whs.make_desc(10, 50, 2, 2, 64, 0, 0)        # two bands: unsupported
    assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 21, FAKE, None, None, FAKE, 1 << 30, None) == -2
    desc = whs.make_desc(10, 50, 2, 1, 32, 0, 0)        # interleave not a multiple of 64
    assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 21, FAKE, None, None, FAKE, 1 << 30, None) == -2
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 1)        # lambda_best is scalar per series
    assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 21, FAKE, None, None, FAKE, 1 << 30, None) == -2
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 0)
    assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 0, FAKE, None, None, FAKE, 1 << 30, None) == -1
    assert L.whs_gcv_workspace_bytes(ctypes.byref(desc)) == 0    # one forward sweep, no workspace
    # interleave 1: copies of x and w; a smaller workspace is refused before any launch
    up = lambda n: (n + 255) // 256 * 256   # noqa: E731
    for dt, e in [(0, 4), (1, 8)]:
        desc = whs.make_desc(70, 50, 2, 1, 1, dt, 0)
        n = L.whs_gcv_workspace_bytes(ctypes.byref(desc))
        assert n == up(128 * 50 * e) + up(128 * 50)
        assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 21, FAKE, None, None, FAKE, n - 8, None) == -4
        assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, g, 21, FAKE, None, None, None, 0, None) == -4
    huge = whs.make_desc(2 ** 30, 365, 2, 1, 1, 0, 0)
    assert L.whs_gcv_workspace_bytes(ctypes.byref(huge)) == 0
    assert L.whs_gcv(ctypes.byref(huge), FAKE, FAKE, g, 21, FAKE, None, None, FAKE, 1 << 40, None) == -2


def test_plan_validation():
    L = whs.lib()
    h = ctypes.c_void_p()
    g = (whs.WhsGroup * 1)(whs.WhsGroup(10, 50, 2, 0, 0, 0, 0))
    assert L.whs_plan_create(ctypes.byref(h), g, 1, 2, 0, 0, 64) == -2      # several bands
    assert L.whs_plan_create(ctypes.byref(h), g, 1, 1, 0, 0, 32) == -2      # interleave != 64
    assert L.whs_plan_create(ctypes.byref(h), g, 0, 1, 0, 0, 64) == -1      # no groups
    bad = (whs.WhsGroup * 1)(whs.WhsGroup(10, 2, 2, 0, 0, 0, 0))            # T <= d
    assert L.whs_plan_create(ctypes.byref(h), bad, 1, 1, 0, 0, 64) == -1
    bad = (whs.WhsGroup * 1)(whs.WhsGroup(10, 50, 5, 0, 0, 0, 0))           # order 5
    assert L.whs_plan_create(ctypes.byref(h), bad, 1, 1, 0, 0, 64) == -2
    assert L.whs_plan_solve(None, FAKE, FAKE, FAKE, FAKE, None, None) == -1
    assert L.whs_plan_config(None, None, None, None, None) == -1


def test_variance_validation():
    L = whs.lib()
    desc = whs.make_desc(10, 50, 2, 2, 64, 0, 1)        # one output channel only
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -1
    desc = whs.make_desc(10, 50, 2, 1, 32, 0, 1)        # interleave neither 1 nor a multiple of 64
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -2
    # interleave 1: copies of w, lambda (per difference row) and var, then the
    # checkpoints of interleave 64; a smaller workspace is refused before any launch
    up = lambda n: (n + 255) // 256 * 256   # noqa: E731
    for kind, dt in [(1, 0), (0, 1)]:
        desc = whs.make_desc(10, 50, 2, 1, 1, dt, kind)
        e = 8 if dt else 4
        n = L.whs_variance_workspace_bytes(ctypes.byref(desc))
        assert n == up(64 * 50) + (up(64 * 48 * e) if kind else 0) + up(64 * 50 * e) + ((50 + 15) // 16) * 5 * 64 * 8
        assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, FAKE, n - 8, None) == -4
        assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, None, 0, None) == -4
    huge = whs.make_desc(2 ** 30, 365, 2, 1, 1, 0, 1)   # the copies' grid does not fit a launch
    assert L.whs_variance_workspace_bytes(ctypes.byref(huge)) == 0
    assert L.whs_variance(ctypes.byref(huge), FAKE, FAKE, FAKE, None, FAKE, 1 << 40, None) == -2
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 1)
    assert L.whs_variance(ctypes.byref(desc), FAKE, None, FAKE, None, FAKE, 1 << 30, None) == -1
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE_ODD, None, FAKE, 1 << 30, None) == -1
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, None, 0, None) == -4
    # order 2: 2 + 1 + 2 = 5 doubles per tile of 16 steps per series
    assert L.whs_variance_workspace_bytes(ctypes.byref(desc)) == ((50 + 15) // 16) * 5 * 64 * 8
    empty = whs.make_desc(0, 50, 2, 1, 64, 0, 1)
    assert L.whs_variance(ctypes.byref(empty), None, None, None, None, None, 0, None) == 0


def test_uneven_time_validation():
    L = whs.lib()
    assert L.whs_diff_coef(FAKE, 10, 0, FAKE, None) == -1
    assert L.whs_diff_coef(FAKE, 2, 2, FAKE, None) == -1          # T <= d
    assert L.whs_diff_coef(FAKE, 10, 5, FAKE, None) == -2
    assert L.whs_diff_coef(None, 10, 2, FAKE, None) == -1
    assert L.whs_diff_coef(FAKE, 10, 2, FAKE_ODD, None) == -1
    desc = whs.make_desc(10, 50, 2, 1, 32, 0, 1)        # interleave not a multiple of 64
    assert L.whs_solve_coef(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -2
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 1)
    assert L.whs_solve_coef(ctypes.byref(desc), None, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -1
    assert L.whs_solve_coef(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE, None, None, 0, None) == -4
    assert L.whs_backward_coef(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE_ODD, None, None, None, FAKE,
                               1 << 30, None) == -1
    empty = whs.make_desc(0, 50, 2, 1, 64, 0, 1)
    assert L.whs_solve_coef(ctypes.byref(empty), None, None, None, None, None, None, None, 0, None) == 0


def test_network_entry_points_validate_arguments():
    from paper_2604_00048_amd import net
    L = net.lib()
    # unsupported channel pairs and modes, null pointers, negative sizes
    assert L.whs_net_conv_fwd(FAKE, 32, FAKE, FAKE, 64, 0, None, FAKE, None, 4, 100, None) == -1
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 2, None, FAKE, None, 4, 100, None) == -1  # mode 2 needs a mask
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 3, None, FAKE, None, 4, 100, None) == -1  # so does mode 3
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 4, FAKE, FAKE, None, 4, 100, None) == -1  # no mode 4
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 2, FAKE, FAKE, FAKE, 4, 100, None) == -1  # bits: mode 0 only
    assert L.whs_net_conv_fwd(FAKE, 8, FAKE, FAKE, 16, 1, None, FAKE, None, 4, 100, None) == -2   # no such layer
    assert L.whs_net_conv_fwd(FAKE, 8, FAKE, FAKE, 64, 3, FAKE, FAKE, None, 4, 100, None) == -2   # nor this one
    assert L.whs_net_conv_fwd(None, 64, FAKE, FAKE, 64, 0, None, FAKE, None, 4, 100, None) == -1
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 0, None, FAKE, FAKE, 0, 100, None) == 0    # empty batch
    assert L.whs_net_conv_fwd(FAKE, 64, FAKE, FAKE, 64, 0, None, FAKE, None, 4, 1 << 24, None) == -2  # 32-bit range
    # the last layer's one-channel backward
    n = L.whs_net_last_bwd_workspace_bytes(8)
    assert n == 8 * (9 * 64 + 1) * 4 and L.whs_net_last_bwd_workspace_bytes(0) == 0
    assert L.whs_net_last_bwd(FAKE, FAKE, FAKE, None, FAKE, FAKE, FAKE, n, 8, 4, 100, None) == -1   # no bits
    assert L.whs_net_last_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, n, 8, 0, 100, None) == -1   # P < 1
    assert L.whs_net_last_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, n - 4, 8, 4, 100, None) == -4
    assert L.whs_net_head_bwd1(None, FAKE, 4, 100, 64, 2, 0.0, 1.0, FAKE, None) == -1
    n = L.whs_net_wgrad_workspace_bytes(64, 64, 7)
    assert n == 7 * (64 * 9 * 64 + 64) * 4
    assert L.whs_net_conv_wgrad(FAKE, 64, FAKE, 64, FAKE, FAKE, n - 1, 7, 4, 100, None) == -4
    assert L.whs_net_conv_wgrad(FAKE, 64, FAKE, 32, FAKE, FAKE, n, 7, 4, 100, None) == -1
    assert L.whs_net_head_fwd(FAKE, 4, 2, 64, 2, -1.0, 5.0, FAKE, None) == -1                # T <= d
    assert L.whs_net_mse(None, FAKE, FAKE, 10, 1.0, FAKE, None, None) == -1
    assert L.whs_net_adam(FAKE, FAKE, FAKE, FAKE, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None) == -1   # step >= 1
    assert L.whs_net_scalar_head_fwd(FAKE, 10, 5.0, -1.0, FAKE, None) == -1                    # hi > lo
    assert L.whs_net_scalar_head_bwd(FAKE, FAKE, 0, -1.0, 5.0, FAKE, None) == -1               # P >= 1


def test_transformer_entry_points_validate_arguments():
    from paper_2604_00048_amd import tf
    L = tf.lib()
    # unsupported widths and modes, missing operands, empty inputs, small workspaces
    assert L.whs_tf_linear(FAKE, 0, 96, FAKE, None, 64, 0, None, None, FAKE, 100, None) == -1     # K
    assert L.whs_tf_linear(FAKE, 0, 64, FAKE, None, 64, 5, None, None, FAKE, 100, None) == -1     # mode
    assert L.whs_tf_linear(FAKE, 1, 64, FAKE, None, 64, 4, None, None, FAKE, 100, None) == -1     # mask
    assert L.whs_tf_linear(FAKE, 0, 64, FAKE, None, 64, 2, None, None, FAKE, 100, None) == -1     # residual
    assert L.whs_tf_linear(FAKE, 1, 192, FAKE, None, 64, 3, None, None, FAKE, 100, None) == -2    # no such product
    assert L.whs_tf_linear(FAKE, 0, 64, FAKE, None, 64, 0, None, None, FAKE, 0, None) == 0        # empty
    n = L.whs_tf_wgrad_workspace_bytes(192, 64, 5)
    assert n == 5 * (192 * 64 + 192) * 4
    assert L.whs_tf_wgrad(FAKE, 0, 192, FAKE, 64, 100, FAKE, FAKE, n - 1, 5, None) == -4
    assert L.whs_tf_wgrad(FAKE, 0, 192, FAKE, 192, 100, FAKE, FAKE, n, 5, None) == -1              # K
    assert L.whs_tf_attn_fwd(FAKE, 4, 0, FAKE, FAKE, None) == -1                                   # T >= 1
    assert L.whs_tf_attn_fwd(FAKE, 4, 4097, FAKE, FAKE, None) == -1
    assert L.whs_tf_attn_bwd(FAKE, FAKE, None, FAKE, 4, 10, FAKE, None) == -1
    assert L.whs_tf_head_fwd(FAKE, 4, 2, FAKE, 64, 2, -6.0, 10.0, FAKE, FAKE, FAKE, FAKE, None) == -1   # T <= d
    assert L.whs_tf_head_fwd(FAKE, 4, 9, FAKE, 64, 2, 10.0, -6.0, FAKE, FAKE, FAKE, FAKE, None) == -1   # hi > lo
    assert L.whs_tf_embed(FAKE, FAKE, 4, 9, 16, 64, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == -1    # C <= 15
    assert L.whs_tf_embed_bwd(FAKE, FAKE, 10, 17, FAKE, FAKE, 1 << 20, 4, None) == -1                  # F <= 16
    assert L.whs_tf_ln_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, 10, FAKE, FAKE, FAKE, 0, 4, None) == -4
    assert L.whs_tf_head_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 4, 9, 64, 2, -6.0, 10.0, FAKE, FAKE, FAKE, 0, 4,
                             None) == -4
    assert L.whs_tf_cast(FAKE, 0, 64, FAKE, None, None) == -1
    # empty inputs: per-token calls return 0 without launching, reductions refuse
    assert L.whs_tf_embed(FAKE, FAKE, 0, 9, 4, 64, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, None) == 0
    assert L.whs_tf_ln_fwd(FAKE, 0, FAKE, FAKE, FAKE, FAKE, None) == 0
    assert L.whs_tf_attn_fwd(FAKE, 0, 9, FAKE, FAKE, None) == 0
    assert L.whs_tf_head_fwd(FAKE, 0, 9, FAKE, 64, 2, -6.0, 10.0, FAKE, FAKE, FAKE, FAKE, None) == 0
    big = 1 << 30
    assert L.whs_tf_ln_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, big, 4, None) == -1
    assert L.whs_tf_wgrad(FAKE, 0, 192, FAKE, 64, 0, FAKE, FAKE, big, 5, None) == -1
    assert L.whs_tf_embed_bwd(FAKE, FAKE, 0, 5, FAKE, FAKE, big, 4, None) == -1
    assert L.whs_tf_head_bwd(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 0, 9, 64, 2, -6.0, 10.0, FAKE, FAKE, FAKE, big, 4,
                             None) == -1


def test_noalloc_entry_point_checks_sizes_before_touching_the_device():
    L = whs.lib()
    assert L.whs_solve_noalloc_max_bytes() == 64 << 20
    big = whs.make_desc(65536, 3288, 2, 1, 64, whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    assert L.whs_workspace_bytes(ctypes.byref(big)) > L.whs_solve_noalloc_max_bytes()
    assert L.whs_solve_noalloc(ctypes.byref(big), FAKE, FAKE, FAKE, FAKE, None, None) == whs.WHS_ERR_UNSUPPORTED
    small = whs.make_desc(100, 365, 2, 1, 64, whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    assert L.whs_solve_noalloc(ctypes.byref(small), None, FAKE, FAKE, FAKE, None, None) == whs.WHS_ERR_ARG
    assert L.whs_solve_noalloc(ctypes.byref(small), FAKE, FAKE, FAKE, None, None, None) == whs.WHS_ERR_ARG
    empty = whs.make_desc(0, 365, 2, 1, 64, whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)
    assert L.whs_solve_noalloc(ctypes.byref(empty), None, None, None, None, None, None) == whs.WHS_OK
    bad = whs.make_desc(100, 2, 2, 1, 64, whs.WHS_F32, whs.WHS_LAMBDA_PER_DIFF)  # T <= d
    assert L.whs_solve_noalloc(ctypes.byref(bad), FAKE, FAKE, FAKE, FAKE, None, None) == whs.WHS_ERR_ARG


def test_weights_as_bits_are_taken_where_built():
    # fused one-band solve and adjoint on the daily grid with an interleave that is
    # a multiple of 64; everything else refuses the bit format without launching
    L = whs.lib()
    bad = whs.make_desc(10, 50, 2, 1, 64, 0, 0, 2)
    assert _solve_raw(bad, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30) == -1          # no such format
    for P, C, S in [(10, 1, 1), (10, 2, 64), (10, 1, 32)]:
        desc = whs.make_desc(P, 50, 2, C, S, 0, 0, whs.WHS_W_BITS)
        assert _solve_raw(desc, FAKE, FAKE, FAKE, FAKE, FAKE, 1 << 30) == -2
    desc = whs.make_desc(10, 50, 2, 1, 64, 0, 0, whs.WHS_W_BITS)
    # a given factor, the factor export, GCV, the variance and uneven dates
    assert L.whs_solve(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -2
    assert L.whs_factor(ctypes.byref(desc), FAKE, FAKE, FAKE, None, None) == -2
    assert L.whs_gcv(ctypes.byref(desc), FAKE, FAKE, FAKE, 3, FAKE, None, None, FAKE, 0, None) == -2
    assert L.whs_variance(ctypes.byref(desc), FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -2
    assert L.whs_solve_coef(ctypes.byref(desc), FAKE, FAKE, FAKE, FAKE, FAKE, None, FAKE, 1 << 30, None) == -2
    # and the empty batch of a supported call is a no-op
    empty = whs.make_desc(0, 50, 2, 1, 64, 0, 0, whs.WHS_W_BITS)
    assert _solve_raw(empty, None, None, None, None, None, 0) == 0


def test_bit_packing_round_trip():
    import torch
    from paper_2604_00048_amd import synth
    g = torch.Generator().manual_seed(4)
    w = (torch.rand((3, 17, 128), generator=g) < 0.3).to(torch.uint8)
    b = synth.pack_bits(w)
    assert tuple(b.shape) == (3, 17, 16) and b.dtype == torch.uint8
    assert torch.equal(synth.unpack_bits(b), w)
    # bit s % 8 of byte s / 8
    s = 77
    assert torch.equal((b[:, :, s // 8] >> (s % 8)) & 1, w[:, :, s])
    # the binding tells the formats apart by shape
    assert whs._w_format(w, 3, 17, 128) == whs.WHS_W_BYTES
    assert whs._w_format(b, 3, 17, 128) == whs.WHS_W_BITS
    with pytest.raises(ValueError):
        whs._w_format(b[:, :, :8], 3, 17, 128)
