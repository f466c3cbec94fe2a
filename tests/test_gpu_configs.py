"""Full-size runs of every workload shape on the GPU, in the batched launch
configuration the benchmark times, checked against the CPU oracle on sampled
pairs (the oracle recomputes those pairs on their own) and, for the DP, on
the GPU's own S for every sampled pair.

Sizes: cfg 1 200x220 (V 2048); cfg 2 4096 pairs lognormal median 60 (V 4096);
cfg 3 256 x 5000x5000 (V 16384, BF16); cfg 4 1024 pairs median 80 max 1000
(V 4096, forward + backward); cfg 5 100k pairs median 60 max 4000 with 8 %
empty-or-tiny sides (V 16384, Zipf 1.05, BF16).
"""
import sys

import numpy as np
import pytest

import oracle
from synth import corpus
from tests import helpers as H

pytestmark = pytest.mark.gpu

F32, BF16 = 0, 1


def _log(msg):
    print("[configs] " + msg, flush=True)
    sys.stdout.flush()


def _check_pairs(run, batch, pairs, prec, scorer=None):
    """S of the sampled pairs vs the FP64 oracle, and the DP bit-exact on
    the GPU's S of those pairs."""
    sub = batch.subset(pairs)
    ora = oracle.score(sub, scorer=scorer, nthreads=0)
    worst = 0.0
    S_gpu = []
    for q, b in enumerate(pairs):
        S = run.S(b)
        S_gpu.append(S)
        ref = ora["S64"][ora["s_off"][q]:ora["s_off"][q + 1]]
        if prec == F32:
            err = H.s_rel_err(S, ref)
            assert err.size == 0 or err.max() <= 1e-5, (b, err.max())
        else:
            err = np.abs(S.astype(np.float64) - ref)
            assert err.size == 0 or err.max() <= 2e-2, (b, err.max())
        worst = max(worst, float(err.max()) if err.size else 0.0)
    al = oracle.align(sub.n, sub.m, np.concatenate(S_gpu) if S_gpu else np.zeros(0, np.float32),
                      batch.gap, batch.threshold)
    for q, b in enumerate(pairs):
        assert np.float32(run.score[b]).view(np.uint32) == np.float32(al["score"][q]).view(np.uint32), b
        assert run.n_diag[b] == al["n_diag"][q], b
        assert run.n_kept[b] == al["n_kept"][q], b
        np.testing.assert_array_equal(run.kept(b), oracle.pair_kept(al, q), err_msg="pair %d" % b)
    return worst


def test_config1_full_fp32_bf16_and_f1():
    b = corpus.make_batch(1)
    for prec in (F32, BF16):
        run = H.GpuRun(b, prec=prec)
        _check_pairs(run, b, [0], prec)
    # planted-alignment F1 with the oriented scorer: FP64 oracle vs FP32 vs BF16
    w = H.load_oriented(1)
    ora = oracle.score(b, scorer=w)
    al = oracle.align(b.n, b.m, ora["S32"], b.gap, b.threshold)
    f64 = oracle.f1([oracle.pair_kept(al, 0)], [b.gold])
    assert f64 > 50.0
    for prec in (F32, BF16):
        run = H.GpuRun(b, prec=prec, scorer=w)
        f = oracle.f1([run.kept(0)], [b.gold])
        assert abs(f - f64) <= 0.5, (prec, f, f64)


def test_config2_full_batch():
    _log("cfg2: generating 4096 pairs")
    b = corpus.make_batch(2)
    pairs = H.sample_pairs(b, 48)
    for prec in (F32, BF16):
        _log("cfg2: GPU prec=%d" % prec)
        run = H.GpuRun(b, prec=prec)
        _check_pairs(run, b, pairs, prec)
        # DP bit-exact on the GPU's S for every pair of the batch
        _log("cfg2: oracle DP on all pairs")
        al = oracle.align(b.n, b.m, run.S_all(), b.gap, b.threshold)
        np.testing.assert_array_equal(run.score.view(np.uint32), al["score"].view(np.uint32))
        np.testing.assert_array_equal(run.n_diag, al["n_diag"])
        np.testing.assert_array_equal(run.n_kept, al["n_kept"])
        kept = run.kept_all()
        for q in range(b.B):
            o, k = int(al["path_off"][q]), int(al["n_kept"][q])
            np.testing.assert_array_equal(kept[o:o + k], al["kept"][o:o + k])
        del run


def test_config2_f1_parity_oriented():
    b = corpus.make_batch(2, pairs=256)
    w = H.load_oriented(2)
    ora = oracle.score(b, scorer=w)
    al = oracle.align(b.n, b.m, ora["S32"], b.gap, b.threshold)
    gold = [b.gold[b.gold_off[q]:b.gold_off[q + 1]] for q in range(b.B)]
    f64 = oracle.f1([oracle.pair_kept(al, q) for q in range(b.B)], gold)
    assert f64 > 50.0
    for prec in (F32, BF16):
        run = H.GpuRun(b, prec=prec, scorer=w)
        f = oracle.f1([run.kept(q) for q in range(b.B)], gold)
        assert abs(f - f64) <= 0.5, (prec, f, f64)


def _f1_parity(run, batch, pairs, scorer):
    """Planted-alignment F1 of the GPU's kept pairs on `pairs` against the
    FP64 oracle's (oracle S64 -> FP32 DP -> keep) on the same pairs."""
    sub = batch.subset(pairs)
    ora = oracle.score(sub, scorer=scorer)
    al = oracle.align(sub.n, sub.m, ora["S32"], batch.gap, batch.threshold)
    gold = [sub.gold[sub.gold_off[q]:sub.gold_off[q + 1]] for q in range(sub.B)]
    f64 = oracle.f1([oracle.pair_kept(al, q) for q in range(sub.B)], gold)
    f = oracle.f1([run.kept(b) for b in pairs], gold)
    worst = 0.0
    for q, b in enumerate(pairs):
        S = run.S(b)
        if S.size:
            worst = max(worst, float(np.abs(S.astype(np.float64) - ora["S64"][ora["s_off"][q]:ora["s_off"][q + 1]]).max()))
    return f, f64, worst


def test_config3_full_bf16():
    _log("cfg3: generating 256 pairs of 5000x5000")
    b = corpus.make_batch(3)
    _log("cfg3: GPU BF16 (6.4e9 cells)")
    run = H.GpuRun(b, prec=BF16)
    pairs = [0, 131, 255]
    _log("cfg3: oracle on pairs %s" % pairs)
    worst = _check_pairs(run, b, pairs, BF16)
    _log("cfg3: max |S - S64| on sampled pairs %.3g" % worst)
    del run
    # planted-alignment F1 with the oriented scorer, BF16 vs the FP64 oracle
    w = H.load_oriented(3)
    _log("cfg3: GPU BF16, oriented scorer")
    run = H.GpuRun(b, prec=BF16, scorer=w)
    pairs = [7, 200]
    f, f64, worst = _f1_parity(run, b, pairs, w)
    _log("cfg3: planted F1 BF16 %.3f vs FP64 %.3f on pairs %s; max |S - S64| %.3g" % (f, f64, pairs, worst))
    assert f64 > 50.0
    assert abs(f - f64) <= 0.5
    assert worst <= 2e-2


def test_config4_full_forward_backward():
    import torch
    import paper_1512_01641_amd as nw
    _log("cfg4: generating 1024 pairs")
    b = corpus.make_batch(4)
    w = H.load_oriented(4)
    run = H.GpuRun(b, prec=F32, scorer=w)
    pairs = H.sample_pairs(b, 24)
    _check_pairs(run, b, pairs, F32, scorer=w)
    mn = run.mn
    dev = mn.ctx.device
    a = np.linspace(0.5, 1.5, b.B).astype(np.float32)
    gS = torch.empty(mn.plan.S_elems, dtype=torch.float32, device=dev)
    gg = torch.zeros(1, dtype=torch.float64, device=dev)
    gwb = torch.zeros(3, dtype=torch.float64, device=dev)
    nw.align_backward(mn.plan, mn.batch, mn.tb, mn.n_diag, torch.as_tensor(a).to(dev), grad_S=gS, grad_gap=gg,
                      S=mn.S, S_raw=mn.S_raw, scorer=w, grad_wb=gwb, ws=mn.ws)
    torch.cuda.synchronize()
    # the oracle backward over the whole batch on the GPU's DP path
    al = oracle.align(b.n, b.m, run.S_all(), b.gap, b.threshold)
    sc = oracle.score(b, scorer=w)
    bw = oracle.backward(b.n, b.m, al, a.astype(np.float64), sc["S64"], sc["S_raw"], sc["rho"])
    np.testing.assert_array_equal(gS.cpu().numpy(), bw["grad_S"].astype(np.float32))
    assert gg.item() == pytest.approx(bw["grad_gap"], rel=1e-9)
    np.testing.assert_allclose(gwb.cpu().numpy(), bw["grad_wb"], rtol=2e-4, atol=1e-3)


def test_config5_full_bf16():
    _log("cfg5: generating 100000 pairs (about a minute)")
    b = corpus.make_batch(5)
    assert np.any(b.n == 0) or np.any(b.m == 0)
    _log("cfg5: GPU BF16")
    run = H.GpuRun(b, prec=BF16)
    pairs = H.sample_pairs(b, 64, seed=5)
    _log("cfg5: oracle on %d sampled pairs" % len(pairs))
    _check_pairs(run, b, pairs, BF16)
    # empty sides: score = fl32((n+m) g), nothing kept
    e = np.nonzero((b.n == 0) | (b.m == 0))[0]
    expect = np.where(b.n[e] + b.m[e] == 0, np.float32(0),
                      (b.n[e] + b.m[e]).astype(np.float32) * np.float32(b.gap)).astype(np.float32)
    np.testing.assert_array_equal(run.score[e].view(np.uint32), expect.view(np.uint32))
    assert np.all(run.n_kept[e] == 0)
    del run
    # planted-alignment F1 with the oriented scorer, BF16 vs the FP64 oracle
    w = H.load_oriented(5)
    _log("cfg5: GPU BF16, oriented scorer")
    run = H.GpuRun(b, prec=BF16, scorer=w)
    pairs = H.sample_pairs(b, 256, seed=55)
    f, f64, worst = _f1_parity(run, b, pairs, w)
    _log("cfg5: planted F1 BF16 %.3f vs FP64 %.3f on %d sampled pairs; max |S - S64| %.3g"
         % (f, f64, len(pairs), worst))
    assert f64 > 50.0
    assert abs(f - f64) <= 0.5
    assert worst <= 2e-2
    del run
    # the backward on a seeded 5 % tuning subsample (forward in BF16)
    _config5_backward_subsample(b, w)


def _config5_backward_subsample(b, w):
    import torch
    import paper_1512_01641_amd as nw
    rng = np.random.default_rng(1512)
    idx = np.sort(rng.choice(b.B, size=b.B // 20, replace=False))
    sub = b.subset(idx)
    _log("cfg5: backward on a 5%% subsample (%d pairs, %d cells)" % (sub.B, sub.cells()))
    run = H.GpuRun(sub, prec=BF16, scorer=w)
    mn = run.mn
    dev = mn.ctx.device
    a = (0.5 + (np.arange(sub.B) % 8) / 8.0).astype(np.float32)
    gS = torch.empty(max(mn.plan.S_elems, 1), dtype=torch.float32, device=dev)
    gg = torch.zeros(1, dtype=torch.float64, device=dev)
    gwb = torch.zeros(3, dtype=torch.float64, device=dev)
    nw.align_backward(mn.plan, mn.batch, mn.tb, mn.n_diag, torch.as_tensor(a).to(dev), grad_S=gS, grad_gap=gg,
                      S=mn.S, S_raw=mn.S_raw, scorer=w, grad_wb=gwb, ws=mn.ws)
    torch.cuda.synchronize()
    Sg = run.S_all()
    al = oracle.align(sub.n, sub.m, Sg, sub.gap, sub.threshold)   # the DP on the GPU's S
    np.testing.assert_array_equal(run.score.view(np.uint32), al["score"].view(np.uint32))
    sc = oracle.score(sub, scorer=w)
    Sr = mn.S_raw[:mn.plan.S_elems].cpu().numpy().astype(np.float64)
    bw = oracle.backward(sub.n, sub.m, al, a.astype(np.float64), Sg.astype(np.float64), Sr, sc["rho"])
    np.testing.assert_array_equal(gS[:mn.plan.S_elems].cpu().numpy(), bw["grad_S"].astype(np.float32))
    assert gg.item() == pytest.approx(bw["grad_gap"], rel=1e-12)
    np.testing.assert_allclose(gwb.cpu().numpy(), bw["grad_wb"], rtol=1e-4, atol=1e-6)
    # against the oracle's FP64 scores: the BF16 similarity's own error
    bw64 = oracle.backward(sub.n, sub.m, al, a.astype(np.float64), sc["S64"], sc["S_raw"], sc["rho"],
                           want_grad_S=False)
    np.testing.assert_allclose(gwb.cpu().numpy(), bw64["grad_wb"], rtol=1e-2)
    _log("cfg5: backward grad_wb %s, oracle FP64 %s" % (gwb.cpu().numpy(), bw64["grad_wb"]))
