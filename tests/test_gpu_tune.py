"""The gradient tuning loop of the scorer, the gap and the threshold (the
paper tunes threshold and penalty against reference alignments, Sec. 5.2;
planted alignments stand in for them)."""
import numpy as np
import pytest

import oracle
from synth import corpus

pytestmark = pytest.mark.gpu


def _setup(pairs=64, first=0):
    import paper_1512_01641_amd as nw
    from paper_1512_01641_amd.tune import Tuner
    b = corpus.make_batch(4, pairs=pairs, first=first)
    ctx = nw.Context(0)
    mn = nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), nw.NWM_FP32)
    return b, mn, Tuner


def test_loss_and_gradient_match_the_oracle():
    import torch
    b, mn, Tuner = _setup()
    w = np.array([4.0, 0.5, -1.5])
    tu = Tuner(mn, b.gold_off, b.gold, w0=w, gap=-0.2)
    loss, gw, gg = tu.loss_and_grad()
    torch.cuda.synchronize()
    # the hinge: NW optimum minus the reference path's score is >= 0
    assert loss >= -1e-3 * b.B
    # the oracle on the GPU's own alignment: d/dw of sum_b Score_b - Gold_b
    S32 = mn.S[:mn.plan.S_elems].cpu().numpy()
    al = oracle.align(b.n, b.m, S32, tu.gap, tu.threshold)
    sc = oracle.score(b, scorer=w.astype(np.float32))
    E = np.zeros(mn.plan.S_elems, np.float64)
    gl = np.diff(b.gold_off)
    pair = np.repeat(np.arange(b.B), gl)
    flat = mn.s_off[pair] + b.gold[:, 0].astype(np.int64) * b.m[pair].astype(np.int64) + b.gold[:, 1]
    E[flat] = -1.0
    bw = oracle.backward(b.n, b.m, al, np.ones(b.B), sc["S64"], sc["S_raw"], sc["rho"], grad_S_extra=E,
                         want_grad_S=False)
    np.testing.assert_allclose(gw, bw["grad_wb"], rtol=2e-4, atol=1e-3)
    gold_gaps = float(np.sum(b.n.astype(np.int64) + b.m - 2 * gl))
    assert gg == pytest.approx(bw["grad_gap"] - gold_gaps, abs=1e-9)
    # and the loss itself against the oracle's FP32 DP score and FP64 gold path
    gold = float(S32[flat].astype(np.float64).sum()) + tu.gap * gold_gaps
    assert loss == pytest.approx(float(al["score"].astype(np.float64).sum()) - gold, rel=1e-6, abs=1e-3)


def test_training_lowers_the_loss_and_threshold_search(tmp_path):
    import torch
    b, mn, Tuner = _setup(pairs=96, first=100)
    tu = Tuner(mn, b.gold_off, b.gold, w0=(1.0, 0.0, 0.0), gap=-0.2, lr_w=0.02, lr_g=0.002)
    first = tu.loss_and_grad()[0]
    losses = [tu.step() for _ in range(25)]
    last = tu.loss_and_grad()[0]
    torch.cuda.synchronize()
    assert np.all(np.isfinite(losses))
    assert last < first, (first, last)
    assert tu.gap < 0
    # threshold: the grid search never picks a worse F1 than the starting point
    mn.mine(tu.w.astype(np.float32), tu.gap, tu.threshold)
    torch.cuda.synchronize()
    start_f1 = oracle.f1([mn.kept_pairs(q) for q in range(b.B)],
                         [b.gold[b.gold_off[q]:b.gold_off[q + 1]] for q in range(b.B)])
    t, f = tu.best_threshold(grid=np.concatenate([[tu.threshold], np.linspace(0.05, 0.95, 19)]))
    assert 0.0 <= f <= 100.0 and f >= start_f1 - 1e-9
    mn.mine(tu.w.astype(np.float32), tu.gap, t)
    torch.cuda.synchronize()
    f_chk = oracle.f1([mn.kept_pairs(q) for q in range(b.B)],
                      [b.gold[b.gold_off[q]:b.gold_off[q + 1]] for q in range(b.B)])
    assert f_chk == pytest.approx(f, abs=1e-6)
    # state round trip
    path = str(tmp_path / "tuner.json")
    tu.save(path)
    st = tu.state()
    tu.w[:] = 0
    tu.load(path)
    assert tu.state() == st
