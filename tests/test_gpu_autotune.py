"""The launch-parameter autotuner: every parameter value gives the same
results bit for bit, the tuner applies and caches its choice, and a cached
choice is reused without timing."""
import json

import numpy as np
import pytest

from synth import corpus

pytestmark = pytest.mark.gpu


def _snap(mn, B):
    P = mn.plan.S_elems
    return (mn.S[:P].cpu().numpy().view(np.uint32).copy(), mn.score[:B].cpu().numpy().view(np.uint32).copy(),
            mn.n_diag[:B].cpu().numpy().copy(), mn.n_kept[:B].cpu().numpy().copy(), mn.kept.cpu().numpy().copy())


def _same(a, b, p_off, n_kept, B):
    for x, y in zip(a[:4], b[:4]):
        np.testing.assert_array_equal(x, y)
    for q in range(B):
        o, k = int(p_off[q]), int(n_kept[q])
        np.testing.assert_array_equal(a[4][o:o + k], b[4][o:o + k])


def test_params_do_not_change_results_and_tuner_caches(tmp_path):
    import torch
    import paper_1512_01641_amd as nw
    from paper_1512_01641_amd import autotune as at
    b = corpus.make_batch(2, pairs=192, first=2000)
    ctx = nw.Context(0)
    mn = nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), nw.NWM_BF16)
    mn.mine(b.scorer, b.gap, b.threshold)
    torch.cuda.synchronize()
    ref = _snap(mn, b.B)
    for name, values in at.SPACE.items():
        for v in values:
            mn.plan.set_param(name, v)
            assert mn.plan.get_param(name) == v
            for graph in (False, True):
                mn.mine(b.scorer, b.gap, b.threshold, graph=graph)
                torch.cuda.synchronize()
                _same(_snap(mn, b.B), ref, mn.p_off, ref[3], b.B)
        mn.plan.set_param(name, values[0])
    with pytest.raises(nw.NwmError):
        mn.plan.set_param("score_xcd_map", 2)
    cache = str(tmp_path / "tune.json")
    r1 = at.autotune(mn, b.scorer, b.gap, b.threshold, reps=2, cache_path=cache)
    assert not r1["cached"] and r1["ms"] > 0
    for k, v in r1["params"].items():
        assert mn.plan.get_param(k) == v
    with open(cache) as f:
        assert at.signature(mn) in json.load(f)
    r2 = at.autotune(mn, b.scorer, b.gap, b.threshold, cache_path=cache)
    assert r2["cached"] and r2["params"] == r1["params"]
    mn.mine(b.scorer, b.gap, b.threshold)
    torch.cuda.synchronize()
    _same(_snap(mn, b.B), ref, mn.p_off, ref[3], b.B)
