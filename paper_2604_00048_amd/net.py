"""The learned-weight form: network g_theta -> per-day weights -> smoother.

Bindings of the network kernels of ``libwhs.so`` (``include/whs_net.h``) and
the training / inference driver that chains them with the smoother's
``whs_solve`` / ``whs_backward`` (Sec. II-C: ``z = f_Lambda(x | W, D)`` with
``Lambda = g_theta(x, t)``).  Every numerical step runs in HIP kernels; this
module allocates tensors and orders the calls.

Network: convolutions over time, kernel 9, widths 8 -> 64 -> 64 -> 64 -> 1,
ReLU between layers, bfloat16 operands with FP32 accumulation; input channels
are the standardised series where observed, the observation flag and four
day-of-year harmonics.  Head: ``log10 lambda = lo + (hi - lo) sigmoid(h)``
(Sec. IV-B bounds the weight with a final sigmoid), one weight per difference
row taken from day ``k + d // 2``.
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

NET_SIGNATURES = {
    "whs_net_conv_fwd": (_I32, [_VP, _I32, _VP, _VP, _I32, _I32, _VP, _VP, _VP, _I64, _I32, _VP]),
    "whs_net_infer": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _I64, _I32, _VP]),
    "whs_net_wgrad_workspace_bytes": (_SZ, [_I32, _I32, _I32]),
    "whs_net_conv_wgrad": (_I32, [_VP, _I32, _VP, _I32, _VP, _VP, _SZ, _I32, _I64, _I32, _VP]),
    "whs_net_input": (_I32, [_VP, _VP, _I64, _I32, _I32, _F, _F, _VP, _VP, _VP]),
    "whs_net_head_fwd": (_I32, [_VP, _I64, _I32, _I32, _I32, _F, _F, _VP, _VP]),
    "whs_net_head_bwd": (_I32, [_VP, _VP, _I64, _I32, _I32, _I32, _F, _F, _VP, _VP]),
    "whs_net_head_bwd1": (_I32, [_VP, _VP, _I64, _I32, _I32, _I32, _F, _F, _VP, _VP]),
    "whs_net_last_bwd_workspace_bytes": (_SZ, [_I32]),
    "whs_net_last_bwd": (_I32, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _SZ, _I32, _I64, _I32, _VP]),
    "whs_net_mse": (_I32, [_VP, _VP, _VP, _I64, _F, _VP, _VP, _VP]),
    "whs_net_adam": (_I32, [_VP, _VP, _VP, _VP, _I64, _F, _F, _F, _F, _I32, _VP]),
    "whs_net_pack_weights": (_I32, [_VP, _I32, _I32, _I32, _VP, _VP, _VP]),
    "whs_net_scalar_head_fwd": (_I32, [_VP, _I64, _F, _F, _VP, _VP]),
    "whs_net_scalar_head_bwd": (_I32, [_VP, _VP, _I64, _F, _F, _VP, _VP]),
}

_net = None


def lib():
    global _net
    if _net is None:
        L = whs.lib()
        for name, (res, args) in NET_SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _net = L
    return _net


def _chk(code, what):
    if code != 0:
        raise RuntimeError(f"{what} failed with status {code}")


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


K = 9
LO, HI = -1.0, 5.0
# (cin, cout_real, cout_padded) per layer
LAYERS = [(8, 64, 64), (64, 64, 64), (64, 64, 64), (64, 1, 16)]


def time_features(T: int, start_year: int = 2016) -> torch.Tensor:
    """Per-day sine/cosine of the first two day-of-year harmonics, (T, 4) FP32."""
    doy = []
    y = start_year
    while len(doy) < T:
        n = 366 if (y % 4 == 0 and (y % 100 != 0 or y % 400 == 0)) else 365
        doy.extend(range(n))
        y += 1
    a = 2.0 * math.pi * torch.tensor(doy[:T], dtype=torch.float64) / 365.25
    return torch.stack([torch.sin(a), torch.cos(a), torch.sin(2 * a), torch.cos(2 * a)], 1).float()


def conv_fwd(inp, cin, w, bias, cout, mode, mask, out, P, T, bits=None):
    _chk(lib().whs_net_conv_fwd(_p(inp), cin, _p(w), _p(bias), cout, mode, _p(mask), _p(out), _p(bits), P, T,
                                _s(inp.device)), "whs_net_conv_fwd")
    return out


def conv_wgrad(inp, cin, gy, cout, grad, P, T, parts=1024, ws=None):
    n = int(lib().whs_net_wgrad_workspace_bytes(cin, cout, parts))
    if ws is None or ws.numel() * ws.element_size() < n:
        ws = torch.empty(n // 4 + 1, dtype=torch.float32, device=inp.device)
    _chk(lib().whs_net_conv_wgrad(_p(inp), cin, _p(gy), cout, _p(grad), _p(ws), ws.numel() * 4, parts, P, T,
                                  _s(inp.device)), "whs_net_conv_wgrad")
    return grad, ws


class ConvNet:
    """Parameters, optimiser state and saved activations of the network on one device."""

    def __init__(self, device, seed: int = 0):
        self.device = torch.device(device)
        g = torch.Generator().manual_seed(seed)
        self.master, self.m, self.v, self.wf, self.wd, self.grad = [], [], [], [], [], []
        for cin, co, cop in LAYERS:
            bound = math.sqrt(6.0 / (cin * K))
            W = (torch.rand((co, K, cin), generator=g, dtype=torch.float64) * 2 - 1) * bound
            flat = torch.cat([W.reshape(-1), torch.zeros(co, dtype=torch.float64)]).float().to(self.device)
            self.master.append(flat)
            self.m.append(torch.zeros_like(flat))
            self.v.append(torch.zeros_like(flat))
            self.grad.append(torch.zeros(cop * K * cin + cop, dtype=torch.float32, device=self.device))
            self.wf.append(torch.zeros(cop * K * cin, dtype=torch.int16, device=self.device))
            self.wd.append(torch.zeros(cin * K * cop, dtype=torch.int16, device=self.device))
        self.bias = [torch.zeros(cop, dtype=torch.float32, device=self.device) for _, _, cop in LAYERS]
        self.step = 0
        self._ws = None
        self.pack()

    def pack(self):
        """bfloat16 forward and input-gradient copies of the FP32 weights; padded biases."""
        for i, (cin, co, cop) in enumerate(LAYERS):
            _chk(lib().whs_net_pack_weights(_p(self.master[i]), co, cop, cin, _p(self.wf[i]), _p(self.wd[i]),
                                            _s(self.device)), "whs_net_pack_weights")
            self.bias[i][:co].copy_(self.master[i][co * K * cin:])

    def forward(self, x8: torch.Tensor, P: int, T: int, keep: bool = True):
        """h (P, T) FP32 from the (P, T, 8) bfloat16 input; keeps activations for backward
        and, for the input gradients, the ReLU bits of each hidden layer's output."""
        acts, bits = [x8], [None]
        a = x8
        for i, (cin, co, cop) in enumerate(LAYERS[:-1]):
            out = torch.empty((P, T, cop), dtype=torch.int16, device=self.device)
            b = torch.empty((P, T, cop // 8), dtype=torch.uint8, device=self.device) if keep else None
            conv_fwd(a, cin, self.wf[i], self.bias[i], cop, 0, None, out, P, T, bits=b)
            acts.append(out)
            bits.append(b)
            a = out
        h = torch.empty((P, T), dtype=torch.float32, device=self.device)
        cin, co, cop = LAYERS[-1]
        conv_fwd(a, cin, self.wf[-1], self.bias[-1], cop, 1, None, h, P, T)
        if keep:
            self.acts, self.bits = acts, bits
        return h

    def infer(self, x8: torch.Tensor, P: int, T: int, h=None):
        """h (P, T) FP32 from the (P, T, 8) bfloat16 input in one launch, the hidden
        activations kept on chip (nothing saved for backward)."""
        if h is None:
            h = torch.empty((P, T), dtype=torch.float32, device=self.device)
        _chk(lib().whs_net_infer(_p(x8), *[_p(w) for w in self.wf], *[_p(b) for b in self.bias], _p(h), P, T,
                                 _s(x8.device)), "whs_net_infer")
        return h

    def backward(self, gh16: torch.Tensor, P: int, T: int):
        """Parameter gradients from dL/dh stored as channel 0 of (P, T, 16) bfloat16."""
        g = gh16
        for i in range(len(LAYERS) - 1, -1, -1):
            cin, co, cop = LAYERS[i]
            _, self._ws = conv_wgrad(self.acts[i], cin, g, cop, self.grad[i], P, T, ws=self._ws)
            if i > 0:
                gx = torch.empty((P, T, cin), dtype=torch.int16, device=self.device)
                conv_fwd(g, cop, self.wd[i], None, cin, 3, self.bits[i], gx, P, T)
                g = gx

    def backward1(self, gh: torch.Tensor, P: int, T: int, parts: int = 1024):
        """Parameter gradients from dL/dh as one channel, (P, T) bfloat16
        (``head_bwd1``): the last layer's backward on that channel only
        (``whs_net_last_bwd``), then the hidden layers as in ``backward``."""
        i = len(LAYERS) - 1
        cin, co, cop = LAYERS[i]
        n = int(lib().whs_net_last_bwd_workspace_bytes(parts))
        if self._ws is None or self._ws.numel() * 4 < n:
            self._ws = torch.empty(n // 4 + 1, dtype=torch.float32, device=self.device)
        g = torch.empty((P, T, cin), dtype=torch.int16, device=self.device)
        _chk(lib().whs_net_last_bwd(_p(self.acts[i]), _p(gh), _p(self.wf[i]), _p(self.bits[i]), _p(g),
                                    _p(self.grad[i]), _p(self._ws), self._ws.numel() * 4, parts, P, T,
                                    _s(self.device)), "whs_net_last_bwd")
        for i in range(len(LAYERS) - 2, -1, -1):
            cin, co, cop = LAYERS[i]
            _, self._ws = conv_wgrad(self.acts[i], cin, g, cop, self.grad[i], P, T, ws=self._ws)
            if i > 0:
                gx = torch.empty((P, T, cin), dtype=torch.int16, device=self.device)
                conv_fwd(g, cop, self.wd[i], None, cin, 3, self.bits[i], gx, P, T)
                g = gx

    def adam(self, lr: float, b1=0.9, b2=0.999, eps=1e-8):
        self.step += 1
        for i, (cin, co, cop) in enumerate(LAYERS):
            # the real rows of the (possibly padded) gradient: weights then biases
            if cop == co:
                gr = self.grad[i]
            else:
                gw = self.grad[i][:cop * K * cin].view(cop, K, cin)[:co].reshape(-1)
                gb = self.grad[i][cop * K * cin:cop * K * cin + co]
                gr = torch.cat([gw, gb])
            n = self.master[i].numel()
            _chk(lib().whs_net_adam(_p(self.master[i]), _p(gr), _p(self.m[i]), _p(self.v[i]), n, lr, b1, b2, eps,
                                    self.step, _s(self.device)), "whs_net_adam")
        self.pack()


def net_input(x, w, P, T, S, mean, sd, feat, out=None):
    if out is None:
        out = torch.empty((P, T, 8), dtype=torch.int16, device=x.device)
    _chk(lib().whs_net_input(_p(x), _p(w), P, T, S, float(mean), float(1.0 / sd), _p(feat), _p(out), _s(x.device)),
         "whs_net_input")
    return out


def head_fwd(h, P, T, S, d, lam=None, lo=LO, hi=HI):
    nb = (P + S - 1) // S
    if lam is None:
        lam = torch.zeros((nb, T - d, S), dtype=torch.float32, device=h.device)
    _chk(lib().whs_net_head_fwd(_p(h), P, T, S, d, lo, hi, _p(lam), _s(h.device)), "whs_net_head_fwd")
    return lam


def head_bwd(h, glam, P, T, S, d, out=None, lo=LO, hi=HI):
    if out is None:
        out = torch.empty((P, T, 16), dtype=torch.int16, device=h.device)
    _chk(lib().whs_net_head_bwd(_p(h), _p(glam), P, T, S, d, lo, hi, _p(out), _s(h.device)), "whs_net_head_bwd")
    return out


def head_bwd1(h, glam, P, T, S, d, out=None, lo=LO, hi=HI):
    """dL/dh as one channel, (P, T) bfloat16 bits (int16)."""
    if out is None:
        out = torch.empty((P, T), dtype=torch.int16, device=h.device)
    _chk(lib().whs_net_head_bwd1(_p(h), _p(glam), P, T, S, d, lo, hi, _p(out), _s(h.device)), "whs_net_head_bwd1")
    return out


def scalar_head_fwd(theta, P, lam=None, lo=LO, hi=HI):
    """One weight for every series from the scalar parameter ``theta`` (FP32[1])."""
    if lam is None:
        lam = torch.empty(P, dtype=torch.float32, device=theta.device)
    _chk(lib().whs_net_scalar_head_fwd(_p(theta), P, lo, hi, _p(lam), _s(theta.device)), "whs_net_scalar_head_fwd")
    return lam


def scalar_head_bwd(theta, glam, P, grad=None, lo=LO, hi=HI):
    if grad is None:
        grad = torch.empty(1, dtype=torch.float32, device=theta.device)
    _chk(lib().whs_net_scalar_head_bwd(_p(theta), _p(glam), P, lo, hi, _p(grad), _s(theta.device)),
         "whs_net_scalar_head_bwd")
    return grad


def mse(z, x, hold, inv_n, g=None, loss=None):
    if g is None:
        g = torch.empty_like(z)
    _chk(lib().whs_net_mse(_p(z), _p(x), _p(hold), z.numel(), float(inv_n), _p(g), _p(loss), _s(z.device)),
         "whs_net_mse")
    return g
