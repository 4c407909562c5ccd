"""Python binding of libwhs (ctypes).  Argument marshalling only.

Every computation runs in the HIP kernels of ``libwhs.so``; this module
checks tensor shapes, dtypes and devices, fills the descriptor, and passes
device pointers and the current HIP stream.  It raises if the library is not
built -- there is no CPU fallback.

Layouts are the interleaved ones of the C header (``S`` series per block):

* ``x``, ``z``, ``g``, ``grad_x``: ``(nb, T, C, S)``
* ``w``: ``(nb, T, S)`` uint8
* ``lam``, ``grad_lambda``: ``(P,)`` (one scalar per series) or
  ``(nb, T-d, S)`` (one weight per difference row)
* ``factor``: ``(nb, d+1, T, S)`` float64
"""

from __future__ import annotations

import ctypes
import os

import torch

from .build import source_hash

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwhs.so")

WHS_F32, WHS_F64 = 0, 1
WHS_LAMBDA_SCALAR, WHS_LAMBDA_PER_DIFF = 0, 1
WHS_W_BYTES, WHS_W_BITS = 0, 1
WHS_OK, WHS_ERR_ARG, WHS_ERR_UNSUPPORTED, WHS_ERR_HIP, WHS_ERR_WORKSPACE = 0, -1, -2, -3, -4


class WhsDesc(ctypes.Structure):
    _fields_ = [
        ("n_series", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("n_rhs", ctypes.c_int32),
        ("interleave", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("lambda_kind", ctypes.c_int32),
        ("w_format", ctypes.c_int32),
    ]


class WhsGroup(ctypes.Structure):
    _fields_ = [
        ("n_series", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("x_off", ctypes.c_int64),
        ("w_off", ctypes.c_int64),
        ("lam_off", ctypes.c_int64),
        ("info_off", ctypes.c_int64),
    ]


_lib = None

_VP = ctypes.c_void_p
_SZ = ctypes.c_size_t
_DP = ctypes.POINTER(WhsDesc)

# symbol -> (restype, argtypes); the same names as include/whs.h
SIGNATURES = {
    "whs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "whs_version": (ctypes.c_int, []),
    "whs_build_id": (ctypes.c_char_p, []),
    "whs_workspace_bytes": (_SZ, [_DP]),
    "whs_interleave_workspace_bytes": (_SZ, [_DP]),
    "whs_factor_bytes": (_SZ, [_DP]),
    "whs_factor": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP]),
    "whs_solve": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_backward": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_solve_noalloc_max_bytes": (_SZ, []),
    "whs_solve_noalloc": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "whs_gcv_workspace_bytes": (_SZ, [_DP]),
    "whs_gcv": (ctypes.c_int, [_DP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_diff_coef": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, _VP, _VP]),
    "whs_solve_coef": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_backward_coef": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_variance_workspace_bytes": (_SZ, [_DP]),
    "whs_variance": (ctypes.c_int, [_DP, _VP, _VP, _VP, _VP, _VP, _SZ, _VP]),
    "whs_plan_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(WhsGroup), ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "whs_plan_solve": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "whs_plan_graph_launch": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "whs_plan_autotune": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, _VP]),
    "whs_plan_config": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "whs_plan_set_config": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "whs_plan_lanes": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "whs_plan_destroy": (None, [_VP]),
}


def lib() -> ctypes.CDLL:
    """Load ``libwhs.so`` (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or `python -m paper_2604_00048_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        built = L.whs_build_id().decode()
        want = source_hash()
        if built != want:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (build id {built}, sources {want}): "
                               "rebuild it with __graft_entry__.build()")
        _lib = L
    return _lib


def build_id() -> str:
    """Build id of the loaded library (hash of the sources it was compiled from)."""
    return lib().whs_build_id().decode()


def status_str(code: int) -> str:
    return lib().whs_status_str(int(code)).decode()


def _check(code: int, what: str):
    if code != 0:
        raise RuntimeError(f"{what} failed: {status_str(code)} (status {code})")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return WHS_F32
    if t.dtype == torch.float64:
        return WHS_F64
    raise TypeError(f"storage dtype must be float32 or float64, got {t.dtype}")


def _need_gpu(*ts):
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("libwhs works on device tensors only (got a CPU tensor)")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous in the interleaved layout")


def make_desc(P: int, T: int, d: int, C: int, S: int, dtype: int, lambda_kind: int, w_format: int = 0) -> WhsDesc:
    return WhsDesc(int(P), int(T), int(d), int(C), int(S), int(dtype), int(lambda_kind), int(w_format))


def _w_format(w: torch.Tensor, nb: int, T: int, S: int) -> int:
    """WHS_W_BYTES for uint8 weights of shape (nb, T, S), WHS_W_BITS for the
    packed form (nb, T, S / 8) of an interleave that is a multiple of 64
    (``synth.pack_bits``)."""
    if w.dtype != torch.uint8:
        raise ValueError("w must be uint8")
    if tuple(w.shape) == (nb, T, S):
        return WHS_W_BYTES
    if S % 64 == 0 and tuple(w.shape) == (nb, T, S // 8):
        return WHS_W_BITS
    raise ValueError(f"w must be uint8 of shape {(nb, T, S)}" + (f" or {(nb, T, S // 8)} (bits)" if S % 64 == 0 else ""))


def _lambda_kind(lam: torch.Tensor | None, P: int, nb: int, T: int, d: int, S: int) -> int:
    if lam is None:
        return WHS_LAMBDA_SCALAR
    if lam.dim() == 1:
        if lam.shape[0] != P:
            raise ValueError(f"scalar weights need shape ({P},), got {tuple(lam.shape)}")
        return WHS_LAMBDA_SCALAR
    if tuple(lam.shape) != (nb, T - d, S):
        raise ValueError(f"per-difference weights need shape {(nb, T - d, S)}, got {tuple(lam.shape)}")
    return WHS_LAMBDA_PER_DIFF


def workspace_bytes(desc: WhsDesc) -> int:
    return int(lib().whs_workspace_bytes(ctypes.byref(desc)))


def _workspace(desc: WhsDesc, device, workspace, staged: bool = False):
    """The caller's workspace (checked), or a new one; ``staged``: large enough for
    series-contiguous calls to run the interleaved kernels on copies."""
    n = workspace_bytes(desc)
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < n:
            raise ValueError(f"workspace has {workspace.numel() * workspace.element_size()} bytes, needs {n}")
        return workspace, n
    if staged:
        n = max(n, int(lib().whs_interleave_workspace_bytes(ctypes.byref(desc))))
    return torch.empty(max(n, 8), dtype=torch.uint8, device=device), n


def _geometry(x: torch.Tensor, P: int | None):
    if x.dim() != 4:
        raise ValueError(f"series need the interleaved shape (nb, T, C, S), got {tuple(x.shape)}")
    nb, T, C, S = x.shape
    if P is None:
        P = nb * S
    if not (nb - 1) * S < P <= nb * S and not (P == 0 and nb == 0):
        raise ValueError(f"P={P} does not fit {nb} blocks of {S}")
    return int(nb), int(T), int(C), int(S), int(P)


def whs_factor(w: torch.Tensor, lam: torch.Tensor, d: int, P: int | None = None, factor=None, info=None):
    """Cholesky factor of Omega in lower band storage (Alg. 1 output, Fig. 2 layout).

    Returns ``(factor (nb, d+1, T, S) float64, info (P,) int32)``.
    """
    _need_gpu(w, lam, factor, info)
    nb, T, S = w.shape
    P = nb * S if P is None else int(P)
    kind = _lambda_kind(lam, P, nb, T, d, S)
    desc = make_desc(P, T, d, 1, S, _dtype_code(lam), kind)
    if factor is None:
        factor = torch.empty((nb, d + 1, T, S), dtype=torch.float64, device=w.device)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=w.device)
    _check(lib().whs_factor(ctypes.byref(desc), _ptr(w), _ptr(lam), _ptr(factor), _ptr(info), _stream(w.device)),
           "whs_factor")
    return factor, info


def whs_diff_coef(times: torch.Tensor, d: int, coef=None) -> torch.Tensor:
    """Rows of the order-``d`` difference operator on the sample times ``times``
    (1-D float64 device tensor, strictly increasing): ``(T-d, d+1)`` float64."""
    _need_gpu(times, coef)
    if times.dtype != torch.float64 or times.dim() != 1 or not times.is_contiguous():
        raise TypeError("times must be a contiguous 1-D float64 device tensor")
    T = times.numel()
    if coef is None:
        coef = torch.empty((max(T - d, 0), d + 1), dtype=torch.float64, device=times.device)
    _check(lib().whs_diff_coef(_ptr(times), T, d, _ptr(coef), _stream(times.device)), "whs_diff_coef")
    return coef


def _check_coef(coef, T, d):
    if coef.dtype != torch.float64 or tuple(coef.shape) != (T - d, d + 1) or not coef.is_contiguous():
        raise ValueError(f"coef must be a contiguous float64 ({T - d}, {d + 1}) device tensor")


def whs_solve(x: torch.Tensor, w: torch.Tensor, lam: torch.Tensor | None, d: int, P: int | None = None,
              factor=None, z=None, info=None, workspace=None, coef=None, staged: bool = True):
    """``z = Omega^{-1} W x`` per series and band.  Returns ``(z, info)``.

    ``staged``: with interleave 1 and no workspace given, allocate the larger
    workspace that lets the call run the interleaved kernels on copies
    (``whs_interleave_workspace_bytes``); ``False`` keeps the kernels that read
    the contiguous layout in place.

    ``coef``: rows of ``D`` on uneven sample times (``whs_diff_coef``); the
    daily grid when ``None``.
    """
    _need_gpu(x, w, lam, factor, z, info, workspace, coef)
    nb, T, C, S, P = _geometry(x, P)
    wf = _w_format(w, nb, T, S)
    if lam is not None and lam.dtype != x.dtype:
        raise TypeError("lambda must have the storage dtype of x")
    kind = _lambda_kind(lam, P, nb, T, d, S)
    desc = make_desc(P, T, d, C, S, _dtype_code(x), kind, wf)
    if z is None:
        z = torch.empty_like(x)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=x.device)
    ws, n = _workspace(desc, x.device, workspace, staged and factor is None)
    if coef is not None:
        if factor is not None:
            raise ValueError("uneven sample times use the fused path (no factor)")
        _check_coef(coef, T, d)
        _check(lib().whs_solve_coef(ctypes.byref(desc), _ptr(coef), _ptr(w), _ptr(lam), _ptr(x), _ptr(z),
                                    _ptr(info), _ptr(ws), ws.numel() * ws.element_size(), _stream(x.device)),
               "whs_solve_coef")
        return z, info
    _check(lib().whs_solve(ctypes.byref(desc), _ptr(w), _ptr(lam), _ptr(factor), _ptr(x), _ptr(z), _ptr(info),
                           _ptr(ws), ws.numel() * ws.element_size(), _stream(x.device)), "whs_solve")
    return z, info


def whs_solve_noalloc(x: torch.Tensor, w: torch.Tensor, lam: torch.Tensor, d: int, P: int | None = None,
                      z: torch.Tensor | None = None, info: torch.Tensor | None = None):
    """``whs_solve`` through the entry point that allocates nothing (its
    checkpoints use the library's own device array).  Returns ``(z, info)``;
    pass ``z`` and ``info`` to keep this call free of allocations too."""
    _need_gpu(x, w, lam, z, info)
    nb, T, C, S, P = _geometry(x, P)
    wf = _w_format(w, nb, T, S)
    if lam.dtype != x.dtype:
        raise TypeError("lambda must have the storage dtype of x")
    desc = make_desc(P, T, d, C, S, _dtype_code(x), _lambda_kind(lam, P, nb, T, d, S), wf)
    if z is None:
        z = torch.empty_like(x)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=x.device)
    _check(lib().whs_solve_noalloc(ctypes.byref(desc), _ptr(w), _ptr(lam), _ptr(x), _ptr(z), _ptr(info),
                                   _stream(x.device)), "whs_solve_noalloc")
    return z, info


def whs_backward(w: torch.Tensor, lam: torch.Tensor | None, z: torch.Tensor, g: torch.Tensor, d: int,
                 P: int | None = None, factor=None, need_x: bool = True, need_lambda: bool = True,
                 grad_x=None, grad_lambda=None, info=None, workspace=None, lambda_kind: int | None = None,
                 coef=None, staged: bool = True):
    """Adjoint against ``g``: ``grad_x = W Omega^{-1} g``, ``grad_lambda_k = -(D u)_k (D z)_k``.

    Returns ``(grad_x or None, grad_lambda or None, info)``.  ``coef`` and ``staged`` as in ``whs_solve``.
    """
    _need_gpu(w, lam, z, g, factor, grad_x, grad_lambda, info, workspace, coef)
    nb, T, C, S, P = _geometry(z, P)
    if tuple(g.shape) != tuple(z.shape) or g.dtype != z.dtype:
        raise ValueError("g must match z in shape and dtype")
    kind = _lambda_kind(lam, P, nb, T, d, S) if lambda_kind is None else int(lambda_kind)
    desc = make_desc(P, T, d, C, S, _dtype_code(z), kind, _w_format(w, nb, T, S))
    if need_x and grad_x is None:
        grad_x = torch.empty_like(g)
    if need_lambda and grad_lambda is None:
        shape = (P,) if kind == WHS_LAMBDA_SCALAR else (nb, T - d, S)
        grad_lambda = torch.empty(shape, dtype=z.dtype, device=z.device)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=z.device)
    ws, n = _workspace(desc, z.device, workspace, staged and factor is None)
    if coef is not None:
        if factor is not None:
            raise ValueError("uneven sample times use the fused path (no factor)")
        _check_coef(coef, T, d)
        _check(lib().whs_backward_coef(ctypes.byref(desc), _ptr(coef), _ptr(w), _ptr(lam), _ptr(z), _ptr(g),
                                       _ptr(grad_x if need_x else None), _ptr(grad_lambda if need_lambda else None),
                                       _ptr(info), _ptr(ws), ws.numel() * ws.element_size(), _stream(z.device)),
               "whs_backward_coef")
        return (grad_x if need_x else None), (grad_lambda if need_lambda else None), info
    _check(lib().whs_backward(ctypes.byref(desc), _ptr(w), _ptr(lam), _ptr(factor), _ptr(z), _ptr(g),
                              _ptr(grad_x if need_x else None), _ptr(grad_lambda if need_lambda else None),
                              _ptr(info), _ptr(ws), ws.numel() * ws.element_size(), _stream(z.device)),
           "whs_backward")
    return (grad_x if need_x else None), (grad_lambda if need_lambda else None), info


def whs_gcv(x: torch.Tensor, w: torch.Tensor, grid: torch.Tensor, d: int, P: int | None = None,
            lambda_best=None, scores=None, info=None, want_scores: bool = False, workspace=None):
    """Per-series scalar weight by GCV over ``grid`` (float64 device tensor).

    ``x``: ``(nb, T, 1, S)``.  Returns ``(lambda_best (P,), scores (P, n_grid) or None, info)``.
    """
    _need_gpu(x, w, grid, lambda_best, scores, info, workspace)
    nb, T, C, S, P = _geometry(x, P)
    if C != 1:
        raise ValueError("GCV works on one band")
    if grid.dtype != torch.float64 or grid.dim() != 1:
        raise TypeError("grid must be a 1-D float64 device tensor")
    desc = make_desc(P, T, d, 1, S, _dtype_code(x), WHS_LAMBDA_SCALAR)
    if lambda_best is None:
        lambda_best = torch.empty(P, dtype=x.dtype, device=x.device)
    if want_scores and scores is None:
        scores = torch.empty((P, grid.numel()), dtype=torch.float64, device=x.device)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=x.device)
    n = int(lib().whs_gcv_workspace_bytes(ctypes.byref(desc)))
    ws = workspace if workspace is not None or n == 0 else torch.empty(n, dtype=torch.uint8, device=x.device)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().whs_gcv(ctypes.byref(desc), _ptr(w), _ptr(x), _ptr(grid), int(grid.numel()), _ptr(lambda_best),
                         _ptr(scores), _ptr(info), _ptr(ws), nbytes, _stream(x.device)),
           "whs_gcv")
    return lambda_best, scores, info


def whs_variance(w: torch.Tensor, lam: torch.Tensor, d: int, P: int | None = None, var=None, info=None,
                 workspace=None):
    """Posterior variance ``diag(Omega^{-1})`` per series, in the series layout ``(nb, T, 1, S)``.

    Returns ``(var, info)``; ``var`` has the storage dtype of ``lam``.
    """
    _need_gpu(w, lam, var, info, workspace)
    if w.dim() != 3 or w.dtype != torch.uint8:
        raise ValueError("w must be uint8 of shape (nb, T, S)")
    nb, T, S = w.shape
    P = nb * S if P is None else int(P)
    kind = _lambda_kind(lam, P, nb, T, d, S)
    desc = make_desc(P, T, d, 1, S, _dtype_code(lam), kind)
    if var is None:
        var = torch.empty((nb, T, 1, S), dtype=lam.dtype, device=w.device)
    if info is None:
        info = torch.empty(P, dtype=torch.int32, device=w.device)
    n = int(lib().whs_variance_workspace_bytes(ctypes.byref(desc)))
    ws = workspace if workspace is not None else torch.empty(max(n, 8), dtype=torch.uint8, device=w.device)
    _check(lib().whs_variance(ctypes.byref(desc), _ptr(w), _ptr(lam), _ptr(var), _ptr(info), _ptr(ws),
                              ws.numel() * ws.element_size(), _stream(w.device)), "whs_variance")
    return var, info


class Plan:
    """Uneven batch (groups of equal length and order) solved in one persistent launch.

    ``groups``: list of dicts with keys ``n_series, T, d, x_off, w_off,
    lam_off, info_off`` (element offsets into flat buffers, interleave 64).
    """

    def __init__(self, groups, dtype=torch.float32, per_diff: bool = False):
        n = len(groups)
        arr = (WhsGroup * n)(*[WhsGroup(int(g["n_series"]), int(g["T"]), int(g["d"]), int(g["x_off"]),
                                        int(g["w_off"]), int(g["lam_off"]), int(g["info_off"])) for g in groups])
        self.groups = [dict(g) for g in groups]
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        code = WHS_F64 if dtype == torch.float64 else WHS_F32
        kind = WHS_LAMBDA_PER_DIFF if per_diff else WHS_LAMBDA_SCALAR
        _check(lib().whs_plan_create(ctypes.byref(self._h), arr, n, 1, code, kind, 64), "whs_plan_create")

    def _args(self, w, lam, x, z):
        _need_gpu(w, lam, x, z)
        for t in (lam, x, z):
            if t.dtype != self.dtype:
                raise TypeError("plan buffers must have the plan's storage dtype")
        return _ptr(w), _ptr(lam), _ptr(x), _ptr(z)

    def solve(self, w, lam, x, z, info=None):
        a = self._args(w, lam, x, z)
        _check(lib().whs_plan_solve(self._h, *a, _ptr(info), _stream(x.device)), "whs_plan_solve")
        return z

    def graph_launch(self, w, lam, x, z, info=None):
        a = self._args(w, lam, x, z)
        _check(lib().whs_plan_graph_launch(self._h, *a, _ptr(info), _stream(x.device)), "whs_plan_graph_launch")
        return z

    def autotune(self, w, lam, x, z, force: bool = False):
        a = self._args(w, lam, x, z)
        _check(lib().whs_plan_autotune(self._h, *a, int(bool(force)), _stream(x.device)), "whs_plan_autotune")
        return self.config()

    def config(self) -> dict:
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().whs_plan_config(self._h, *[ctypes.byref(t) for t in v]), "whs_plan_config")
        lanes = []
        for g in range(len(self.groups)):
            n = ctypes.c_int32()
            _check(lib().whs_plan_lanes(self._h, g, ctypes.byref(n)), "whs_plan_lanes")
            lanes.append(n.value)
        return {"tile_profile": v[0].value, "waves_per_block": v[1].value, "waves_per_simd": v[2].value,
                "n_items": v[3].value, "lanes_per_series": lanes}

    def set_config(self, tile_profile: int, waves_per_block: int, waves_per_simd: int, split_T: int = 0):
        """Choose the configuration instead of tuning it (``split_T > 0``: groups of at
        least that length take two lanes per series, two wavefronts per workgroup)."""
        _check(lib().whs_plan_set_config(self._h, tile_profile, waves_per_block, waves_per_simd, split_T),
               "whs_plan_set_config")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().whs_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class WhittakerFn(torch.autograd.Function):
    """``z = (W + D^T Lambda D)^{-1} W x`` as a differentiable layer (Sec. II-C).

    ``apply(x, lam, w, d, P)`` on interleaved tensors; gradients flow to ``x``
    and ``lam`` through the adjoint kernel (one extra banded solve).
    """

    @staticmethod
    def forward(ctx, x, lam, w, d, P=None):
        z, info = whs_solve(x, w, lam, d, P)
        ctx.save_for_backward(w, lam, z)
        ctx.d = d
        ctx.P = P
        ctx.mark_non_differentiable(info)
        return z, info

    @staticmethod
    def backward(ctx, gz, ginfo):
        w, lam, z = ctx.saved_tensors
        need_x, need_l = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_x or need_l):
            return None, None, None, None, None
        gx, gl, _ = whs_backward(w, lam, z, gz.contiguous(), ctx.d, ctx.P, need_x=need_x, need_lambda=need_l)
        return gx, gl, None, None, None


def smooth(x, lam, w, d, P=None):
    """Differentiable smoother; returns ``z`` only."""
    z, _ = WhittakerFn.apply(x, lam, w, d, P)
    return z
