"""Transformer weight network g_theta (Sec. IV-B) on the library's kernels.

Bindings of ``include/whs_tf.h`` and the parameter, activation and gradient
bookkeeping of one network.  Tokens are the acquisitions of a series (row
``p*T + t``); the network reads the standardised bands where an acquisition
is used and the use flag, adds a sinusoidal encoding of the acquisition day,
runs pre-norm encoder layers (width 64, 2 heads, feed-forward 128, ReLU) and
maps each token through a final layer norm and a linear head to a weight
``10^(lo + (hi - lo) sigmoid(s))`` (Sec. IV-B bounds it with a sigmoid; the
paper's typical bounds are 1e-6 and 1e10).  Difference row k takes the weight
of acquisition ``k + d // 2``.

Every numerical step runs in HIP kernels; this module only allocates tensors
and orders the calls.
"""

from __future__ import annotations

import ctypes
import math

import torch

from . import whs

_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int
_F = ctypes.c_float
_SZ = ctypes.c_size_t

TF_SIGNATURES = {
    "whs_tf_pe": (_I32, [_VP, _I32, _VP, _VP]),
    "whs_tf_embed": (_I32, [_VP, _VP, _I64, _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "whs_tf_ln_fwd": (_I32, [_VP, _I64, _VP, _VP, _VP, _VP, _VP]),
    "whs_tf_ln_bwd_workspace_bytes": (_SZ, [_I32]),
    "whs_tf_ln_bwd": (_I32, [_VP, _VP, _VP, _VP, _VP, _I64, _VP, _VP, _VP, _SZ, _I32, _VP]),
    "whs_tf_linear": (_I32, [_VP, _I32, _I32, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _I64, _VP]),
    "whs_tf_wgrad_workspace_bytes": (_SZ, [_I32, _I32, _I32]),
    "whs_tf_wgrad": (_I32, [_VP, _I32, _I32, _VP, _I32, _I64, _VP, _VP, _SZ, _I32, _VP]),
    "whs_tf_attn_fwd": (_I32, [_VP, _I64, _I32, _VP, _VP, _VP]),
    "whs_tf_attn_bwd": (_I32, [_VP, _VP, _VP, _VP, _I64, _I32, _VP, _VP]),
    "whs_tf_head_fwd": (_I32, [_VP, _I64, _I32, _VP, _I32, _I32, _F, _F, _VP, _VP, _VP, _VP, _VP]),
    "whs_tf_head_bwd_workspace_bytes": (_SZ, [_I32]),
    "whs_tf_head_bwd": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _I64, _I32, _I32, _I32, _F, _F, _VP, _VP, _VP, _SZ,
                               _I32, _VP]),
    "whs_tf_embed_bwd_workspace_bytes": (_SZ, [_I32, _I32]),
    "whs_tf_embed_bwd": (_I32, [_VP, _VP, _I64, _I32, _VP, _VP, _SZ, _I32, _VP]),
    "whs_tf_cast": (_I32, [_VP, _I32, _I32, _VP, _VP, _VP]),
}

E, H, DH, FF, NL = 64, 2, 32, 128, 2
LO, HI = -6.0, 10.0
BF16 = torch.int16   # bfloat16 bits travel as int16 tensors
PARTS = 512           # workgroups of the weight-gradient and layer-norm reductions
PARTS_TOKEN = 2048    # workgroups of the per-token reductions (head, embedding): more in flight

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = whs.lib()
        for name, (res, args) in TF_SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _chk(code, what):
    if code != 0:
        raise RuntimeError(f"{what} failed with status {code}")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


# ---------------------------------------------------------------------------
# thin wrappers (same names as the C entry points, without the prefix)
# ---------------------------------------------------------------------------
def pe(times: torch.Tensor, out=None):
    T = times.numel()
    out = torch.empty((T, E), dtype=torch.float32, device=times.device) if out is None else out
    _chk(lib().whs_tf_pe(_p(times), T, _p(out), _s(times.device)), "whs_tf_pe")
    return out


def embed(x, w, P, T, C, S, mean, inv_sd, pe_t, web, feats, h):
    _chk(lib().whs_tf_embed(_p(x), _p(w), P, T, C, S, _p(mean), _p(inv_sd), _p(pe_t), _p(web), _p(feats), _p(h),
                            _s(h.device)), "whs_tf_embed")


def ln_fwd(h, M, gb, out, mean, rstd):
    _chk(lib().whs_tf_ln_fwd(_p(h), M, _p(gb), _p(out), _p(mean), _p(rstd), _s(h.device)), "whs_tf_ln_fwd")


def ln_bwd(ga, h, mean, rstd, gb, M, gh, dgb, ws, parts=PARTS):
    _chk(lib().whs_tf_ln_bwd(_p(ga), _p(h), _p(mean), _p(rstd), _p(gb), M, _p(gh), _p(dgb), _p(ws),
                             ws.numel() * ws.element_size(), parts, _s(h.device)), "whs_tf_ln_bwd")


def linear(x, x_f32, K, w, bias, N, mode, mask, res, out, M):
    _chk(lib().whs_tf_linear(_p(x), int(x_f32), K, _p(w), _p(bias), N, mode, _p(mask), _p(res), _p(out), M,
                             _s(out.device)), "whs_tf_linear")


def wgrad(dy, dy_f32, N, x, K, M, dwb, ws, parts=PARTS):
    _chk(lib().whs_tf_wgrad(_p(dy), int(dy_f32), N, _p(x), K, M, _p(dwb), _p(ws), ws.numel() * ws.element_size(),
                            parts, _s(x.device)), "whs_tf_wgrad")


def attn_fwd(qkv, P, T, o, lse):
    _chk(lib().whs_tf_attn_fwd(_p(qkv), P, T, _p(o), _p(lse), _s(qkv.device)), "whs_tf_attn_fwd")


def attn_bwd(qkv, o, go, lse, P, T, dqkv):
    _chk(lib().whs_tf_attn_bwd(_p(qkv), _p(o), _p(go), _p(lse), P, T, _p(dqkv), _s(qkv.device)), "whs_tf_attn_bwd")


def head_fwd(h, P, T, hp, S, d, lo, hi, s, mean, rstd, lam):
    _chk(lib().whs_tf_head_fwd(_p(h), P, T, _p(hp), S, d, lo, hi, _p(s), _p(mean), _p(rstd), _p(lam),
                               _s(h.device)), "whs_tf_head_fwd")


def head_bwd(h, s, mean, rstd, hp, glam, P, T, S, d, lo, hi, gh, dhp, ws, parts=PARTS_TOKEN):
    _chk(lib().whs_tf_head_bwd(_p(h), _p(s), _p(mean), _p(rstd), _p(hp), _p(glam), P, T, S, d, lo, hi, _p(gh),
                               _p(dhp), _p(ws), ws.numel() * ws.element_size(), parts, _s(h.device)),
         "whs_tf_head_bwd")


def embed_bwd(gh, feats, M, F, dweb, ws, parts=PARTS_TOKEN):
    _chk(lib().whs_tf_embed_bwd(_p(gh), _p(feats), M, F, _p(dweb), _p(ws), ws.numel() * ws.element_size(), parts,
                                _s(gh.device)), "whs_tf_embed_bwd")


def cast(w, N, K, out, out_t=None):
    _chk(lib().whs_tf_cast(_p(w), N, K, _p(out), _p(out_t), _s(w.device)), "whs_tf_cast")


def workspace_bytes(F: int) -> int:
    L = lib()
    return max(int(L.whs_tf_wgrad_workspace_bytes(3 * E, E, PARTS)), int(L.whs_tf_wgrad_workspace_bytes(E, FF, PARTS)),
               int(L.whs_tf_ln_bwd_workspace_bytes(PARTS)), int(L.whs_tf_head_bwd_workspace_bytes(PARTS_TOKEN)),
               int(L.whs_tf_embed_bwd_workspace_bytes(F, PARTS_TOKEN)))


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------
LAYER_KEYS = [("g1", (E,)), ("b1", (E,)), ("Wqkv", (3 * E, E)), ("bqkv", (3 * E,)), ("Wo", (E, E)), ("bo", (E,)),
              ("g2", (E,)), ("b2", (E,)), ("W1", (FF, E)), ("bf1", (FF,)), ("W2", (E, FF)), ("bf2", (E,))]


def layout(F: int, nl: int = NL):
    """Offsets of every parameter in the flat FP32 buffer: ``{name: (offset, shape)}``
    with per-layer names ``"<i>.<key>"``."""
    out, off = {}, 0

    def put(name, shape):
        nonlocal off
        out[name] = (off, shape)
        off += math.prod(shape)
    put("We", (E, F))
    put("be", (E,))
    for i in range(nl):
        for k, shp in LAYER_KEYS:
            put(f"{i}.{k}", shp)
    put("gf", (E,))
    put("bf", (E,))
    put("wh", (E,))
    put("bh", (1,))
    return out, off


class TransformerNet:
    """FP32 master parameters, Adam state, bfloat16 copies and saved activations."""

    def __init__(self, device, C: int, seed: int = 0, nl: int = NL, lo: float = LO, hi: float = HI):
        self.device = torch.device(device)
        self.C, self.F, self.nl, self.lo, self.hi = C, C + 1, nl, lo, hi
        self.lay, n = layout(self.F, nl)
        g = torch.Generator().manual_seed(seed)
        theta = torch.zeros(n, dtype=torch.float64)
        for name, (off, shp) in self.lay.items():
            key = name.split(".")[-1]
            if key.startswith("W") or key == "wh":
                fan_in = shp[-1]
                theta[off:off + math.prod(shp)] = (torch.rand(math.prod(shp), generator=g, dtype=torch.float64) * 2
                                                   - 1) / math.sqrt(fan_in)
            elif key in ("g1", "g2", "gf"):
                theta[off:off + math.prod(shp)] = 1.0
        self.theta = theta.float().to(self.device)
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        self.wbf = {}
        for i in range(nl):
            for k, (N, K) in (("Wqkv", (3 * E, E)), ("Wo", (E, E)), ("W1", (FF, E)), ("W2", (E, FF))):
                self.wbf[f"{i}.{k}"] = (torch.empty((N, K), dtype=BF16, device=self.device),
                                        torch.empty((K, N), dtype=BF16, device=self.device))
        self.ws = torch.empty(workspace_bytes(self.F) // 4 + 1, dtype=torch.float32, device=self.device)
        self.cast()

    def view(self, name, t=None):
        off, shp = self.lay[name]
        return (self.theta if t is None else t)[off:off + math.prod(shp)].view(shp)

    def run(self, name, length, t=None):
        """A run of the flat buffer starting at ``name`` (parameters stored together)."""
        off, _ = self.lay[name]
        return (self.theta if t is None else t)[off:off + length]

    def cast(self):
        for name, (wf, wt) in self.wbf.items():
            N, K = wf.shape
            cast(self.view(name), N, K, wf, wt)

    def forward(self, x, w, P: int, T: int, S: int, mean, inv_sd, pe_t, d: int, keep: bool = True):
        """Weights of the difference rows, interleaved ``(nb, T - d, S)`` FP32, for
        bands ``x`` (the smoother's layout) and use flags ``w``."""
        dev = self.device
        M = P * T
        feats = torch.empty((M, self.F), dtype=torch.float32, device=dev)
        h = torch.empty((M, E), dtype=torch.float32, device=dev)
        embed(x, w, P, T, self.C, S, mean, inv_sd, pe_t, self.run("We", E * self.F + E), feats, h)
        acts = []
        for i in range(self.nl):
            c = {"h_in": h}
            c["a"] = torch.empty((M, E), dtype=BF16, device=dev)
            c["mu1"] = torch.empty(M, dtype=torch.float32, device=dev)
            c["rs1"] = torch.empty(M, dtype=torch.float32, device=dev)
            ln_fwd(h, M, self.run(f"{i}.g1", 2 * E), c["a"], c["mu1"], c["rs1"])
            c["qkv"] = torch.empty((M, 3 * E), dtype=BF16, device=dev)
            linear(c["a"], 0, E, self.wbf[f"{i}.Wqkv"][0], self.view(f"{i}.bqkv"), 3 * E, 0, None, None, c["qkv"], M)
            c["o"] = torch.empty((M, E), dtype=BF16, device=dev)
            c["lse"] = torch.empty((P, H, T), dtype=torch.float32, device=dev)
            attn_fwd(c["qkv"], P, T, c["o"], c["lse"])
            hm = torch.empty((M, E), dtype=torch.float32, device=dev)
            linear(c["o"], 0, E, self.wbf[f"{i}.Wo"][0], self.view(f"{i}.bo"), E, 2, None, h, hm, M)
            c["h_mid"] = hm
            c["a2"] = torch.empty((M, E), dtype=BF16, device=dev)
            c["mu2"] = torch.empty(M, dtype=torch.float32, device=dev)
            c["rs2"] = torch.empty(M, dtype=torch.float32, device=dev)
            ln_fwd(hm, M, self.run(f"{i}.g2", 2 * E), c["a2"], c["mu2"], c["rs2"])
            c["f"] = torch.empty((M, FF), dtype=BF16, device=dev)
            linear(c["a2"], 0, E, self.wbf[f"{i}.W1"][0], self.view(f"{i}.bf1"), FF, 1, None, None, c["f"], M)
            h = torch.empty((M, E), dtype=torch.float32, device=dev)
            linear(c["f"], 0, FF, self.wbf[f"{i}.W2"][0], self.view(f"{i}.bf2"), E, 2, None, hm, h, M)
            acts.append(c)
        nb = (P + S - 1) // S
        lam = torch.empty((nb, T - d, S), dtype=torch.float32, device=dev)
        s = torch.empty(M, dtype=torch.float32, device=dev)
        muf = torch.empty(M, dtype=torch.float32, device=dev)
        rsf = torch.empty(M, dtype=torch.float32, device=dev)
        head_fwd(h, P, T, self.run("gf", 3 * E + 1), S, d, self.lo, self.hi, s, muf, rsf, lam)
        if keep:
            self.cache = dict(P=P, T=T, S=S, d=d, feats=feats, acts=acts, h=h, s=s, muf=muf, rsf=rsf)
        return lam

    def backward(self, glam):
        """Parameter gradients into ``self.grad`` from dL/dlambda of the rows."""
        c0 = self.cache
        P, T, S, d = c0["P"], c0["T"], c0["S"], c0["d"]
        M = P * T
        dev = self.device
        G = self.grad
        gh = torch.empty((M, E), dtype=torch.float32, device=dev)
        head_bwd(c0["h"], c0["s"], c0["muf"], c0["rsf"], self.run("gf", 3 * E + 1), glam, P, T, S, d, self.lo,
                 self.hi, gh, self.run("gf", 3 * E + 1, G), self.ws)
        gF = torch.empty((M, FF), dtype=BF16, device=dev)
        ga = torch.empty((M, E), dtype=torch.float32, device=dev)
        go = torch.empty((M, E), dtype=BF16, device=dev)
        dqkv = torch.empty((M, 3 * E), dtype=BF16, device=dev)
        for i in range(self.nl - 1, -1, -1):
            c = c0["acts"][i]
            wgrad(gh, 1, E, c["f"], FF, M, self.run(f"{i}.W2", E * FF + E, G), self.ws)
            linear(gh, 1, E, self.wbf[f"{i}.W2"][1], None, FF, 4, c["f"], None, gF, M)
            wgrad(gF, 0, FF, c["a2"], E, M, self.run(f"{i}.W1", FF * E + FF, G), self.ws)
            linear(gF, 0, FF, self.wbf[f"{i}.W1"][1], None, E, 3, None, None, ga, M)
            ln_bwd(ga, c["h_mid"], c["mu2"], c["rs2"], self.run(f"{i}.g2", 2 * E), M, gh,
                   self.run(f"{i}.g2", 2 * E, G), self.ws)
            wgrad(gh, 1, E, c["o"], E, M, self.run(f"{i}.Wo", E * E + E, G), self.ws)
            linear(gh, 1, E, self.wbf[f"{i}.Wo"][1], None, E, 0, None, None, go, M)
            attn_bwd(c["qkv"], c["o"], go, c["lse"], P, T, dqkv)
            wgrad(dqkv, 0, 3 * E, c["a"], E, M, self.run(f"{i}.Wqkv", 3 * E * E + 3 * E, G), self.ws)
            linear(dqkv, 0, 3 * E, self.wbf[f"{i}.Wqkv"][1], None, E, 3, None, None, ga, M)
            ln_bwd(ga, c["h_in"], c["mu1"], c["rs1"], self.run(f"{i}.g1", 2 * E), M, gh,
                   self.run(f"{i}.g1", 2 * E, G), self.ws)
        embed_bwd(gh, c0["feats"], M, self.F, self.run("We", E * self.F + E, G), self.ws)

    def adam(self, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        from . import net
        self.step += 1
        _chk(net.lib().whs_net_adam(_p(self.theta), _p(self.grad), _p(self.m), _p(self.v), self.theta.numel(), lr,
                                    b1, b2, eps, self.step, _s(self.device)), "whs_net_adam")
        self.cast()
