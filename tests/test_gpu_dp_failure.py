"""The DP's failure report (nwm_align_check), forced from the host.

The strips of a tall pair hand rows to each other through memory, and a
strip that waits longer than its poll limit gives up.  NWM_PARAM_DP_TEST_HOLD
makes the first strip of every pair taller than one strip publish nothing, so
the strip below waits out a small poll limit (NWM_PARAM_DP_SPIN_LIMIT) and
gives up; every kernel still ends normally.  Expected: nwm_align_check
reports NWM_EDEVICE, the failed pairs have a NaN score and nothing aligned or
kept, the pairs of one strip are untouched (bit-exact against the oracle), and
after the parameters are reset the same plan aligns every pair bit-exactly
and reports NWM_OK.
"""
import numpy as np
import pytest

import oracle
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _mine(nw, mn, b):
    # nwm_mine without graphs: the multi-stream schedule, three fill launches
    nw.mine(mn.plan, mn.batch, mn.dic, b.scorer, b.gap, b.threshold, mn.S, None, mn.score, mn.n_diag, mn.kept,
            mn.n_kept, mn.tb, mn.ws)


@pytest.mark.parametrize("via_mine", [False, True])
def test_dp_hand_off_timeout_is_reported(via_mine):
    import torch
    import paper_1512_01641_amd as nw
    from synth import corpus
    sizes = ([150, 40, 64, 65, 300, 12], [90, 50, 70, 64, 20, 33])
    b = corpus.make_batch(2, pairs=6, sizes=sizes)
    tall = b.n > 64
    ctx = nw.Context(0)
    mn = nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), 0)
    mn.plan.set_param("dp_spin_limit", 64)
    mn.plan.set_param("dp_test_hold", 1)
    print("case: hold first strips, spin limit 64, via_mine=%s" % via_mine, flush=True)
    if via_mine:
        _mine(nw, mn, b)
    else:
        mn.score_pairs(b.scorer)
        mn.align(b.gap, b.threshold)
    assert nw.align_check(mn.plan, mn.ws) is True
    with pytest.raises(nw.NwmError) as ei:
        mn.check()
    assert ei.value.status == 4   # NWM_EDEVICE
    torch.cuda.synchronize()
    S = mn.S[:mn.plan.S_elems].cpu().numpy()
    al = oracle.align(b.n, b.m, S, b.gap, b.threshold)
    score = mn.score[:b.B].cpu().numpy()
    n_diag = mn.n_diag[:b.B].cpu().numpy()
    n_kept = mn.n_kept[:b.B].cpu().numpy()
    assert np.all(np.isnan(score[tall]))
    assert np.all(n_diag[tall] == 0) and np.all(n_kept[tall] == 0)
    ok = ~tall
    np.testing.assert_array_equal(score[ok].view(np.uint32), al["score"][ok].view(np.uint32))
    np.testing.assert_array_equal(n_diag[ok], al["n_diag"][ok])
    np.testing.assert_array_equal(n_kept[ok], al["n_kept"][ok])
    # back to the defaults: every pair, and the check passes
    mn.plan.set_param("dp_test_hold", 0)
    mn.plan.set_param("dp_spin_limit", 0)
    print("case: defaults again", flush=True)
    if via_mine:
        _mine(nw, mn, b)
    else:
        mn.align(b.gap, b.threshold)
    assert nw.align_check(mn.plan, mn.ws) is False
    mn.check()
    got = dict(score=mn.score[:b.B].cpu().numpy(), n_diag=mn.n_diag[:b.B].cpu().numpy(),
               n_kept=mn.n_kept[:b.B].cpu().numpy(), kept=mn.kept.cpu().numpy())
    H.assert_align_equal(got, al, b.n, b.m)
