"""Bi-directional mining (Sec. 5.4, Table 3 "BI") and the random-search tuning
script (Sec. 5.2) on the GPU, against the oracle.

Bars: the union of kept pairs is bit-exact against the oracle's set union
(given the same kept lists); the reverse direction's S meets the FP32 bar
(1e-5 relative to the FP64 oracle) and its DP is bit-exact given identical S;
the random search's per-trial similarity equals the oracle's (NW over the
aligned-pair sequences) on the GPU's S, trial by trial.
"""
import numpy as np
import pytest

import oracle
from synth import corpus
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _monotone(rng, n, m, k):
    k = min(k, n, m)
    return np.stack([np.sort(rng.choice(n, k, replace=False)), np.sort(rng.choice(m, k, replace=False))], 1)


def _union_gpu(n, m, fwd, rev):
    """nwm_union_kept through the C ABI on lists placed at the plan's offsets."""
    import torch
    import paper_1512_01641_amd as nw
    n = np.asarray(n, np.int32)
    m = np.asarray(m, np.int32)
    B = len(n)
    ctx = nw.Context(0)
    so = np.zeros(int(n.sum()) + 1, np.int64)
    to = np.zeros(int(m.sum()) + 1, np.int64)
    db = nw.DeviceBatch(n, m, so, np.zeros(0, np.int32), to, np.zeros(0, np.int32), 64, "cuda:0", max_sent_tokens=0)
    plan = nw.Plan(ctx, db, 1, 0)
    p_off = oracle.path_offsets(n, m)
    cap = int(p_off[-1])
    kf = np.full((max(cap, 1), 2), -7, np.int32)
    kr = np.full((max(cap, 1), 2), -7, np.int32)
    for b in range(B):
        kf[p_off[b]:p_off[b] + len(fwd[b])] = fwd[b]
        kr[p_off[b]:p_off[b] + len(rev[b])] = rev[b]
    dev = torch.device("cuda:0")
    t = lambda a: torch.as_tensor(a).to(dev)
    out = torch.full((max(2 * cap, 1), 2), -9, dtype=torch.int32, device=dev)
    n_out = torch.full((max(B, 1),), -1, dtype=torch.int32, device=dev)
    nf = t(np.array([len(x) for x in fwd] or [0], np.int32))
    nr = t(np.array([len(x) for x in rev] or [0], np.int32))
    nw.union_kept(plan, t(kf), nf, t(kr), nr, out, n_out)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    c = n_out.cpu().numpy()
    return [o[2 * p_off[b]:2 * p_off[b] + c[b]] for b in range(B)], c


def test_union_kernel_edge_cases_and_long_lists():
    rng = np.random.default_rng(21)
    n = [1, 5, 70, 300, 3000, 2500, 64, 128, 40, 1]
    m = [1, 7, 65, 280, 2800, 3100, 64, 128, 40, 9]
    fwd, rev_t = [], []
    for b in range(len(n)):
        F = _monotone(rng, n[b], m[b], int(rng.integers(0, min(n[b], m[b]) + 1)))
        R = _monotone(rng, n[b], m[b], int(rng.integers(0, min(n[b], m[b]) + 1)))
        fwd.append(F)
        rev_t.append(R)
    # special cases: both empty, one empty, identical, disjoint halves,
    # exactly one block each, reverse inside forward
    fwd[0], rev_t[0] = np.zeros((0, 2), int), np.zeros((0, 2), int)
    rev_t[1] = np.zeros((0, 2), int)
    rev_t[2] = fwd[2].copy()
    fwd[6] = np.stack([np.arange(0, 64, 2)] * 2, 1)
    rev_t[6] = np.stack([np.arange(1, 64, 2)] * 2, 1)
    fwd[7] = np.stack([np.arange(64)] * 2, 1)
    rev_t[7] = np.stack([np.arange(64, 128)] * 2, 1)
    rev_t[8] = fwd[8][::3].copy()
    fwd[9] = np.zeros((0, 2), int)
    rev_t[9] = np.array([[0, 4]])
    rev = [r[:, ::-1].copy() for r in rev_t]      # as the reverse plan reports them: (target, source)
    got, cnt = _union_gpu(n, m, fwd, rev)
    want = oracle.union_kept(fwd, rev)
    for b in range(len(n)):
        np.testing.assert_array_equal(got[b], want[b], err_msg="pair %d" % b)
        assert cnt[b] == len(want[b])


def test_bidirectional_mining_matches_oracle():
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(2, pairs=48)
    rb = corpus.reverse_batch(b)
    for prec in (0, 1):
        ctx = nw.Context(0)
        db = nw.DeviceBatch.from_host(b)
        bm = nw.BiMiner(ctx, db, nw.DeviceDict.from_host(b), nw.DeviceDict.from_host(rb), prec)
        bm.mine(b.scorer, rb.scorer, b.gap, b.threshold)
        torch.cuda.synchronize()
        Sf = bm.fwd.S[:bm.fwd.plan.S_elems].cpu().numpy()
        Sr = bm.rev.S[:bm.rev.plan.S_elems].cpu().numpy()
        S64r = oracle.score(rb)["S64"]
        if prec == 0:
            err = H.s_rel_err(Sr, S64r)
            assert err.max() <= 1e-5, err.max()
        else:
            err = np.abs(Sr.astype(np.float64) - S64r)
            assert err.max() <= 2e-2, err.max()
        of = oracle.align(b.n, b.m, Sf, b.gap, b.threshold)
        orv = oracle.align(rb.n, rb.m, Sr, rb.gap, rb.threshold)
        kf = [oracle.pair_kept(of, q) for q in range(b.B)]
        kr = [oracle.pair_kept(orv, q) for q in range(b.B)]
        want = oracle.union_kept(kf, kr)
        for q in range(b.B):
            got = bm.kept_pairs(q)
            np.testing.assert_array_equal(got, want[q], err_msg="pair %d" % q)
            # the union holds everything the forward direction keeps
            mono = set(map(tuple, kf[q].tolist()))
            assert mono <= set(map(tuple, got.tolist()))


@pytest.mark.parametrize("prec", [0, 1])
def test_bidirectional_f1_parity_oriented(prec):
    """Planted-alignment F1 of the bi-directional union (oriented scorer in
    both directions) within 0.5 points of the FP64 oracle's union, and the
    union finds every planted pair the forward direction finds."""
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(2, pairs=96)
    rb = corpus.reverse_batch(b)
    w = H.load_oriented(2)
    gold = [b.gold[b.gold_off[q]:b.gold_off[q + 1]] for q in range(b.B)]
    of = oracle.align(b.n, b.m, oracle.score(b, scorer=w)["S32"], b.gap, b.threshold)
    orv = oracle.align(rb.n, rb.m, oracle.score(rb, scorer=w)["S32"], rb.gap, rb.threshold)
    kf64 = [oracle.pair_kept(of, q) for q in range(b.B)]
    u64 = oracle.union_kept(kf64, [oracle.pair_kept(orv, q) for q in range(b.B)])
    f64_mono, f64_bi = oracle.f1(kf64, gold), oracle.f1(u64, gold)
    assert f64_bi > 50.0
    ctx = nw.Context(0)
    bm = nw.BiMiner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), nw.DeviceDict.from_host(rb), prec)
    bm.mine(w, w, b.gap, b.threshold)
    torch.cuda.synchronize()
    got = [bm.kept_pairs(q) for q in range(b.B)]
    mono = [bm.fwd.kept_pairs(q) for q in range(b.B)]
    f_bi, f_mono = oracle.f1(got, gold), oracle.f1(mono, gold)
    print("planted-pair F1 (prec %d): forward %.2f (FP64 %.2f), bi-directional %.2f (FP64 %.2f)"
          % (prec, f_mono, f64_mono, f_bi, f64_bi))
    assert abs(f_bi - f64_bi) <= 0.5 and abs(f_mono - f64_mono) <= 0.5
    tp = lambda K: sum(len(set(map(tuple, np.asarray(k).reshape(-1, 2).tolist())) &
                           set(map(tuple, g.tolist()))) for k, g in zip(K, gold))
    assert tp(got) >= tp(mono)


def test_random_search_matches_oracle_trial_by_trial():
    import torch
    import paper_1512_01641_amd as nw
    from paper_1512_01641_amd import tune
    b = corpus.make_batch(2, pairs=40)
    ctx = nw.Context(0)
    mn = nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), 0)
    res = tune.random_search(mn, b.scorer, b.gold_off, b.gold, trials=12, seed=3)
    torch.cuda.synchronize()
    S = mn.S[:mn.plan.S_elems].cpu().numpy()
    gold = [b.gold[b.gold_off[q]:b.gold_off[q + 1]] for q in range(b.B)]
    rng = np.random.default_rng(3)
    for th, g, sim in res["history"]:
        # the same draws, in the same order and FP32 rounding
        assert th == float(np.float32(rng.uniform(0.05, 0.95)))
        assert g == float(np.float32(rng.uniform(-1.0, -0.01)))
        o = oracle.align(b.n, b.m, S, g, th)
        want = oracle.similarity([oracle.pair_kept(o, q) for q in range(b.B)], gold)
        assert sim == pytest.approx(want, abs=1e-12)
    best = max(h[2] for h in res["history"])
    assert res["similarity"] == best and best > 20.0
