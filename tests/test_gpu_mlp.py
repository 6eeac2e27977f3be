"""GPU tests of the warm-start network kernels against the FP64 oracle
(oracle/mlp.py): forward, gradients (FP32 kernels vs FP64 reference,
relative error 1e-3 per parameter block) and one Adam step, at ragged sizes
that leave partial 64x64 tiles and at the full 64 -> 512 -> 512 -> 8001
shape."""

import numpy as np
import pytest

from gpu_common import log
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


SHAPES = [(64, 100, 130, 37), (5, 17, 3, 1), (64, 512, 8001, 64)]


def _setup(ni, h, no, B, seed):
    rng = np.random.default_rng(seed)
    p = OM.init_params(rng, ni, h, no).astype(np.float32)
    p[OM.param_count(ni, h, 0) - 0:] += 0.0
    x = rng.standard_normal((B, ni)).astype(np.float32)
    t = rng.standard_normal((B, no)).astype(np.float32)
    return p, x, t


def _blocks(v, ni, h, no):
    return OM.unpack(np.asarray(v, dtype=np.float64), ni, h, no)


@pytest.mark.parametrize("ni,h,no,B", SHAPES)
def test_forward_matches_oracle(ni, h, no, B):
    _torch()
    import paper_1312_3039_amd as hsd
    log(f"mlp forward {ni}-{h}-{h}-{no} batch {B}")
    p, x, _ = _setup(ni, h, no, B, 1)
    net = hsd.MLP(ni, h, no, max(B, 8))
    net.set_params(p)
    y = net.forward(x).cpu().numpy()
    ref, _ = OM.forward(p.astype(np.float64), x.astype(np.float64), ni, h, no)
    assert np.linalg.norm(y - ref) <= 1e-4 * np.linalg.norm(ref)


@pytest.mark.parametrize("ni,h,no,B", SHAPES)
def test_gradients_match_oracle(ni, h, no, B):
    _torch()
    import paper_1312_3039_amd as hsd
    log(f"mlp gradients {ni}-{h}-{h}-{no} batch {B}")
    p, x, t = _setup(ni, h, no, B, 2)
    net = hsd.MLP(ni, h, no, B)
    net.set_params(p)
    g, loss = net.gradients(x, t)
    L, gref = OM.loss_and_grads(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64),
                                ni, h, no)
    assert abs(float(loss.cpu()) - L) <= 1e-4 * L
    for gb, rb in zip(_blocks(g.cpu().numpy(), ni, h, no), _blocks(gref, ni, h, no)):
        assert np.linalg.norm(gb - rb) <= 1e-3 * max(np.linalg.norm(rb), 1e-12)


def test_adam_step_matches_oracle():
    _torch()
    import paper_1312_3039_amd as hsd
    ni, h, no, B = 64, 100, 130, 37
    p, x, t = _setup(ni, h, no, B, 3)
    net = hsd.MLP(ni, h, no, B)
    net.set_params(p)
    pp = p.astype(np.float64)
    m = np.zeros_like(pp)
    v = np.zeros_like(pp)
    for step in range(1, 4):
        net.train_step(x, t, 1e-3)
        _, g = OM.loss_and_grads(pp, x.astype(np.float64), t.astype(np.float64), ni, h, no)
        pp, m, v = OM.adam_step(pp, g, m, v, step, 1e-3)
    got = net.params().cpu().numpy()
    assert np.linalg.norm(got - pp) <= 1e-4 * np.linalg.norm(pp)


def test_training_reduces_loss():
    _torch()
    import paper_1312_3039_amd as hsd
    rng = np.random.default_rng(4)
    ni, h, no, B = 16, 64, 24, 128
    W = rng.standard_normal((no, ni))
    x = rng.standard_normal((B, ni)).astype(np.float32)
    t = np.tanh(x @ W.T).astype(np.float32)
    net = hsd.MLP(ni, h, no, B)
    net.set_params(OM.init_params(rng, ni, h, no))
    first = float(net.train_step(x, t, 3e-3).cpu())
    for _ in range(300):
        last = float(net.train_step(x, t, 3e-3).cpu())
    assert last < 0.1 * first
