"""nwm_align_batch_noalloc (the DP, traceback and keep with the library's
fixed device scratch instead of a workspace) against nwm_align_batch on the
same plan and S, through the C ABI: score bits, aligned-pair counts and kept
pairs bit for bit, and the oracle DP on the same S.  Two calls in a row, the
second on a smaller batch (the scratch keeps the first call's contents), then
the first batch again; a plan too large for the scratch is refused before
anything is launched."""
import numpy as np
import pytest

import oracle
from synth import corpus
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _outputs(nw, torch, mn, B):
    dev = mn.ctx.device
    return dict(score=torch.full((max(B, 1),), -3.0, dtype=torch.float32, device=dev),
                n_diag=torch.full((max(B, 1),), -3, dtype=torch.int32, device=dev),
                n_kept=torch.full((max(B, 1),), -3, dtype=torch.int32, device=dev),
                kept=torch.full((max(mn.plan.kept_cap, 1), 2), -3, dtype=torch.int32, device=dev),
                tb=torch.empty(max(mn.plan.tb_bytes, 1), dtype=torch.uint8, device=dev))


def _host(o, B):
    return dict(score=o["score"][:B].cpu().numpy(), n_diag=o["n_diag"][:B].cpu().numpy(),
                n_kept=o["n_kept"][:B].cpu().numpy(), kept=o["kept"].cpu().numpy())


def _check(nw, torch, b, prec):
    print("case: %d pairs (n max %d), prec %d" % (b.B, int(b.n.max()), prec), flush=True)
    ctx = nw.Context(0)
    mn = nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), prec)
    mn.score_pairs(b.scorer, want_raw=False)
    P = mn.plan.S_elems
    S = mn.S[:P]
    ref = _outputs(nw, torch, mn, b.B)
    nw.align_batch(mn.plan, S, b.gap, b.threshold, ref["score"], ref["n_diag"], ref["kept"], ref["n_kept"],
                   ref["tb"], mn.ws)
    got = _outputs(nw, torch, mn, b.B)
    nw.align_batch_noalloc(mn.plan, S, b.gap, b.threshold, got["score"], got["n_diag"], got["kept"],
                           got["n_kept"], got["tb"])
    torch.cuda.synchronize()
    r, g = _host(ref, b.B), _host(got, b.B)
    np.testing.assert_array_equal(g["score"].view(np.uint32), r["score"].view(np.uint32))
    np.testing.assert_array_equal(g["n_diag"], r["n_diag"])
    np.testing.assert_array_equal(g["n_kept"], r["n_kept"])
    p_off = oracle.path_offsets(b.n, b.m)
    for q in range(b.B):
        o, k = int(p_off[q]), int(r["n_kept"][q])
        np.testing.assert_array_equal(g["kept"][o:o + k], r["kept"][o:o + k], err_msg="pair %d" % q)
    # and the oracle DP on the same S
    al = oracle.align(b.n, b.m, S.cpu().numpy(), b.gap, b.threshold)
    H.assert_align_equal(g, al, b.n, b.m)
    assert not np.isnan(g["score"]).any()


def test_noalloc_align_matches_workspace_entry_point():
    import torch
    import paper_1512_01641_amd as nw
    # several tall pairs (boundary rows between strips) among short ones
    n = [700, 40, 0, 65, 650, 30, 128, 7, 20, 300, 1500, 90]
    m = [690, 35, 9, 70, 600, 0, 129, 8, 25, 310, 1300, 64]
    big = corpus.make_batch(2, sizes=(n * 4, m * 4))
    small = corpus.make_batch(2, pairs=40, first=300)
    _check(nw, torch, big, 0)
    _check(nw, torch, small, 1)    # second call: a smaller batch
    _check(nw, torch, big, 1)      # the first batch again, after the smaller one


def test_noalloc_refuses_plans_beyond_its_scratch():
    import torch
    import paper_1512_01641_amd as nw
    # two pairs of 5000 x 30000 sentences publish 2 x 78 rows of 30194 slots
    # (about 38 MB): beyond the 32 MiB scratch.  Nothing is launched.
    n = np.array([5000, 5000], np.int32)
    m = np.array([30000, 30000], np.int32)
    ctx = nw.Context(0)
    db = nw.DeviceBatch(n, m, np.zeros(int(n.sum()) + 1, np.int64), np.zeros(0, np.int32),
                        np.zeros(int(m.sum()) + 1, np.int64), np.zeros(0, np.int32), 64, "cuda:0",
                        max_sent_tokens=0)
    plan = nw.Plan(ctx, db, 1, 0)
    one = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    ione = torch.zeros(4, dtype=torch.int32, device="cuda:0")
    with pytest.raises(nw.NwmError) as ei:
        nw.align_batch_noalloc(plan, one, -0.2, 0.5, one, ione, ione, ione, ione)
    assert ei.value.status == 5   # NWM_EUNSUPPORTED
    torch.cuda.synchronize()
