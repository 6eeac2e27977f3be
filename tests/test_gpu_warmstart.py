"""GPU test of the learned warm start: on a small parametric family
(b(theta) = b0 + B theta with fixed A and c), a network trained by the
library's own kernels on solutions produced by the batched solver starts
held-out programs closer to their solutions than the cold start, and the
solves it starts need fewer iterations on average.  The fallback keeps the
cold start whenever the prediction's residuals are not below the cold
start's."""

import numpy as np
import pytest

from datagen import draw_parametric_family, draw_theta
from gpu_common import log

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_trained_network_reduces_iterations():
    _torch()
    from paper_1312_3039_amd import warmstart as W
    pd = draw_parametric_family(seed=77, n=120, m=360, nonneg=60, soc_lo=3, soc_hi=10,
                                density=0.05, p=16, b_std=0.01)
    fam = W.family_from_draw(pd)
    train = np.stack([draw_theta(s, p=16) for s in range(1024)])
    held = np.stack([draw_theta(10 ** 6 + s, p=16) for s in range(24)])
    log("warm start: generating 1024 training solves")
    sol = W.solve_family(fam, train, chunk=1024)
    ok = sol["status"] == 1
    assert ok.mean() > 0.95
    T = W.targets(sol)[ok]
    ws = W.WarmStarter(fam, hidden=256, batch=128)
    log("warm start: training")
    losses = ws.fit(train[ok], T, epochs=25, lr=1e-3)
    assert losses[-1] < 0.5 * losses[0]
    log("warm start: evaluating on 24 held-out programs")
    rows = W.evaluate(fam, ws, held)
    cold = np.array([r["cold_iters"] for r in rows])
    warm = np.array([r["warm_iters"] for r in rows])
    assert all(r["cold_status"] == 1 and r["warm_status"] == 1 for r in rows)
    for r in rows:
        assert abs(r["warm_obj"] - r["cold_obj"]) <= 1e-3 * (1 + abs(r["cold_obj"]))
    log(f"  mean iterations cold {cold.mean():.1f} warm {warm.mean():.1f}; "
        f"warm used on {sum(r['used_warm'] for r in rows)}/24")
    assert warm.mean() < 0.8 * cold.mean()


def test_fallback_rejects_a_bad_prediction():
    _torch()
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import warmstart as W
    pd = draw_parametric_family(seed=78, n=60, m=180, nonneg=30, soc_lo=3, soc_hi=8,
                                density=0.08, p=8, b_std=0.01)
    fam = W.family_from_draw(pd)
    # an untrained network with huge outputs: its start must be rejected
    ws = W.WarmStarter(fam, hidden=32, batch=16)
    import torch
    ws.net = hsd.MLP(8, 32, fam.n + fam.m + 1, 16)
    ws.net.set_params(np.full(ws.net.P, 0.5, dtype=np.float32))
    ws.mu = torch.zeros(fam.n + fam.m + 1, dtype=torch.float64, device="cuda")
    ws.sd = torch.full((fam.n + fam.m + 1,), 1e3, dtype=torch.float64, device="cuda")
    held = np.stack([draw_theta(5 + s, p=8) for s in range(4)])
    rows = W.evaluate(fam, ws, held)
    for r in rows:
        assert not r["used_warm"]
        assert r["warm_iters"] == r["cold_iters"]


def test_certificate_family_race_keeps_the_cold_certificate():
    """Certificate family (b with a large perturbation: the programs are
    primal infeasible): with an untrained network, the race between the
    cold start and the predicted start (judged by the termination tests'
    quantities after a few updates) never loses a certificate the cold
    start finds, and costs at most the dropped probe's updates more."""
    _torch()
    import torch
    import paper_1312_3039_amd as hsd
    from paper_1312_3039_amd import warmstart as W
    pd = draw_parametric_family(seed=79, n=60, m=180, nonneg=30, soc_lo=3, soc_hi=8,
                                density=0.08, p=8, b_std=0.3)
    fam = W.family_from_draw(pd)
    ws = W.WarmStarter(fam, hidden=32, batch=16)
    N = fam.n + fam.m + 1
    ws.net = hsd.MLP(8, 32, N, 16)
    rng = np.random.default_rng(3)
    ws.net.set_params(rng.standard_normal(ws.net.P).astype(np.float32))
    ws.mu = torch.zeros(N, dtype=torch.float64, device="cuda")
    ws.sd = torch.ones(N, dtype=torch.float64, device="cuda")
    held = np.stack([draw_theta(50 + s, p=8) for s in range(6)])
    log("certificate family: race of cold and predicted starts")
    probe = 20
    rows = W.evaluate_q(fam, ws, held, probe=probe)
    for r in rows:
        log(f"  cold {r['cold_status']} {r['cold_iters']} | warm path {r['warm_status']} "
            f"{r['warm_iters']} used_warm={r['used_warm']}")
        if r["cold_status"] == 3:
            assert r["warm_status"] == 3
        if not r["used_warm"] and r["cold_iters"] > probe:
            # the cold start won: it continued from its own saved state, bit for bit
            assert r["warm_iters"] == r["cold_iters"] + probe
