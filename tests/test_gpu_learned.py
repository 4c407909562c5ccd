"""The learned per-day weights beat the GCV-chosen scalar weight on held-out
points of fresh series (the gain the learned form exists for).  Parity of the
gain itself is unpinned: it is a measured property, reported with its size."""

import pytest
import torch

from paper_2604_00048_amd import learned

pytestmark = pytest.mark.gpu


def test_learned_weights_beat_gcv_on_fresh_series():
    dev = torch.device("cuda:0")
    L = learned.train(dev, steps=150, batch_size=4096, lr=1e-3, log=print)
    ev = learned.evaluate(L, dev, n_series=16384, chunk=16384)
    print(ev)
    assert ev["rmse_learned"] < ev["rmse_plain_gcv"], ev
