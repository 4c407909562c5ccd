"""Parity of the weight networks at the sizes bench.py trains them on, in the
same launch configuration: the convolution network on a batch of 4096 series
of 3288 days, the transformer on 4096 series of 280 acquisitions and 4 bands.
The kernels run on the whole batch; sampled series (spread over the batch,
the last one included) are recomputed by the FP64 references from their own
inputs and compared: the network output within 1e-2 of its largest value (as
for the whole network at small sizes: one-step differences in stored
bfloat16 activations propagate), the weights of the difference rows within
1e-5 of the head applied to the kernel's own output."""

import numpy as np
import pytest
import torch

from oracle import convnet_ref as N
from oracle import transformer_ref as X
from paper_2604_00048_amd import learned, learned_tf, synth, tf

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def sample(P, n=5):
    return [int(i) for i in np.unique(np.linspace(0, P - 1, n).astype(np.int64))]


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def test_convolution_network_at_training_size():
    P, T = 4096, learned.T_DAYS
    b = learned.make_batch(P, 2604004805, 0, DEV)
    mean, sd = learned.input_stats(b)
    L = learned.Learned(DEV, mean, sd, seed=0)
    h, lam = L.weights(b)
    idx = sample(P)
    params = []
    for i, (cin, co, cop) in enumerate(learned.net.LAYERS):
        flat = L.model.master[i].cpu().double().numpy()
        params.append((flat[:co * 9 * cin].reshape(co, 9, cin), flat[co * 9 * cin:]))
    x = synth.unpack_series(b.x_train.cpu(), P)[idx, :, 0].double().numpy()
    w = synth.unpack_rows(b.w_train.cpu(), P)[idx].numpy()
    inv_sd = np.float32(1.0 / sd)
    x_in = N.standardize(x, w, np.float32(mean), 1.0 / inv_sd, N.time_features(T))
    h_ref, _ = N.forward(params, x_in)
    h_gpu = h.cpu().double().numpy()[idx]
    assert rel(h_gpu, h_ref) < 1e-2
    lam_gpu = synth.unpack_rows(lam.cpu(), P).double().numpy()[idx]
    assert np.max(np.abs(lam_gpu / N.head_rows(N.head(h_gpu), learned.D) - 1)) < 1e-5


def test_transformer_at_training_size():
    P, T, C = 4096, learned_tf.T_ACQ, learned_tf.C_BANDS
    b = learned_tf.make_batch(P, 2604004807, 0, DEV)
    mean, sd = learned_tf.band_stats(b)
    het = learned_tf.Hetero(DEV, C, mean, sd)
    lam = het.weights(b, keep=True)
    m = het.model
    th = m.theta.cpu().double().numpy()

    def get(name):
        off, shp = m.lay[name]
        return th[off:off + int(np.prod(shp))].reshape(shp)
    p = {k: get(k) for k in ("We", "be", "gf", "bf", "wh", "bh")}
    p["layers"] = [{k: get(f"{i}.{k}") for k, _ in tf.LAYER_KEYS} for i in range(m.nl)]
    idx = sample(P)
    x = synth.unpack_series(b.x_train.cpu(), P)[idx].double().numpy()
    w = synth.unpack_rows(b.w_train.cpu(), P)[idx].numpy()
    mean32 = het.mean.cpu().double().numpy()
    sd_eff = 1.0 / het.inv_sd.cpu().double().numpy()
    s_ref, _ = X.forward(p, X.features(x, w, mean32, sd_eff), b.days.cpu().numpy())
    s_gpu = m.cache["s"].cpu().double().numpy().reshape(P, T)[idx]
    assert rel(s_gpu, s_ref) < 1e-2
    lam_gpu = synth.unpack_rows(lam.cpu(), P).double().numpy()[idx]
    assert np.max(np.abs(lam_gpu / N.head_rows(N.head(s_gpu, X.LO, X.HI), learned_tf.D) - 1)) < 1e-5
