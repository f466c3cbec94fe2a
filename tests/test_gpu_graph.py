"""Replays of the captured HIP graph of the whole path (nwm_mine with graphs
on) against eager runs of the same entry points.  Every replay is checked,
with unrelated eager device work and synchronisations between replays."""
import numpy as np
import pytest

from synth import corpus

pytestmark = pytest.mark.gpu


def _snapshot(mn, B):
    P = mn.plan.S_elems
    return dict(S=mn.S[:P].cpu().numpy().view(np.uint32), S_raw=mn.S_raw[:P].cpu().numpy().view(np.uint32),
                score=mn.score[:B].cpu().numpy().view(np.uint32), n_diag=mn.n_diag[:B].cpu().numpy(),
                n_kept=mn.n_kept[:B].cpu().numpy(), kept=mn.kept.cpu().numpy())


def _assert_same(a, b, p_off, B, what):
    for k in ("S", "S_raw", "score", "n_diag", "n_kept"):
        np.testing.assert_array_equal(a[k], b[k], err_msg="%s: %s" % (what, k))
    for i in range(B):
        o, n = int(p_off[i]), int(a["n_kept"][i])
        np.testing.assert_array_equal(a["kept"][o:o + n], b["kept"][o:o + n], err_msg="%s: kept %d" % (what, i))


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replays_match_eager(prec):
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(2, pairs=96, first=1000)
    ctx = nw.Context(0)
    db = nw.DeviceBatch.from_host(b, "cuda:0")
    dd = nw.DeviceDict.from_host(b, "cuda:0")
    eager = nw.Miner(ctx, db, dd, prec)
    eager.mine(b.scorer, b.gap, b.threshold, want_raw=True)
    torch.cuda.synchronize()
    ref = _snapshot(eager, b.B)

    g = nw.Miner(ctx, db, dd, prec)
    noise = torch.empty(1 << 22, device="cuda:0")
    for rep in range(4):
        for t in (g.S, g.S_raw, g.score, g.n_diag, g.n_kept, g.kept):
            t.fill_(-7)
        g.mine(b.scorer, b.gap, b.threshold, graph=True, want_raw=True)
        torch.cuda.synchronize()
        _assert_same(_snapshot(g, b.B), ref, eager.p_off, b.B, "replay %d" % rep)
        noise.normal_()
        assert float(noise.abs().sum().item()) > 0
        eager.mine(b.scorer, b.gap, b.threshold, want_raw=True)
        torch.cuda.synchronize()

    # another threshold: the graph is captured again and matches eager again
    thr = 0.3
    eager.mine(b.scorer, b.gap, thr, want_raw=True)
    torch.cuda.synchronize()
    ref2 = _snapshot(eager, b.B)
    for rep in range(2):
        g.mine(b.scorer, b.gap, thr, graph=True, want_raw=True)
        torch.cuda.synchronize()
        _assert_same(_snapshot(g, b.B), ref2, eager.p_off, b.B, "threshold 0.3 replay %d" % rep)
    assert int(ref2["n_kept"].sum()) >= int(ref["n_kept"].sum())


def test_graph_replay_reads_current_inputs():
    """A replay reads the buffers' contents at launch time: new tokens written
    into the same device buffers give the eager result of the new tokens."""
    import torch
    import paper_1512_01641_amd as nw
    b1 = corpus.make_batch(2, pairs=48, first=0)
    b2 = corpus.make_batch(2, pairs=48, first=0)
    # same sizes, other target words (a bag of words ignores token order, so
    # the ids themselves change)
    b2.tgt_tok = ((b2.tgt_tok.astype(np.int64) * 7 + 3) % b2.V).astype(np.int32)
    ctx = nw.Context(0)
    db = nw.DeviceBatch.from_host(b1, "cuda:0")
    dd = nw.DeviceDict.from_host(b1, "cuda:0")
    g = nw.Miner(ctx, db, dd, 1)
    g.mine(b1.scorer, b1.gap, b1.threshold, graph=True, want_raw=True)
    torch.cuda.synchronize()
    r1 = _snapshot(g, b1.B)
    db.tgt_tok.copy_(torch.as_tensor(b2.tgt_tok))
    g.mine(b1.scorer, b1.gap, b1.threshold, graph=True, want_raw=True)
    torch.cuda.synchronize()
    r2 = _snapshot(g, b1.B)

    db2 = nw.DeviceBatch.from_host(b2, "cuda:0")
    e = nw.Miner(ctx, db2, dd, 1)
    e.mine(b1.scorer, b1.gap, b1.threshold, want_raw=True)
    torch.cuda.synchronize()
    _assert_same(r2, _snapshot(e, b1.B), e.p_off, b1.B, "after token update")
    assert not np.array_equal(r1["S"], r2["S"])


@pytest.mark.parametrize("prec", [0, 1])
def test_overlapped_mine_matches_separate_entry_points(prec):
    # nwm_mine without graphs runs the long-chain pairs' DP on a second
    # stream, overlapped with the other pairs; the results equal
    # nwm_score_pairs + nwm_align_batch bit for bit.  The batch mixes a few
    # long pairs (several strips) with many short ones, and empty sides.
    import torch
    import paper_1512_01641_amd as nw
    n = [700, 40, 0, 65, 650, 30, 128, 7, 20, 300] * 6
    m = [690, 35, 9, 70, 600, 0, 129, 8, 25, 310] * 6
    b = corpus.make_batch(2, sizes=(n, m))
    ctx = nw.Context(0)
    db = nw.DeviceBatch.from_host(b, "cuda:0")
    dd = nw.DeviceDict.from_host(b, "cuda:0")
    eager = nw.Miner(ctx, db, dd, prec)
    eager.mine(b.scorer, b.gap, b.threshold, want_raw=True)
    torch.cuda.synchronize()
    ref = _snapshot(eager, b.B)
    o = nw.Miner(ctx, db, dd, prec)
    for rep in range(3):
        for t in (o.S, o.S_raw, o.score, o.n_diag, o.n_kept, o.kept):
            t.fill_(-5)
        nw.mine(o.plan, db, dd, b.scorer, b.gap, b.threshold, o.S, o.S_raw, o.score, o.n_diag, o.kept, o.n_kept,
                o.tb, o.ws)
        torch.cuda.synchronize()
        _assert_same(_snapshot(o, b.B), ref, eager.p_off, b.B, "overlapped %d" % rep)
