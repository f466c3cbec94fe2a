"""Host logic of the benchmark: the algorithmic work per kernel class and the
choice of the dominant kernel (no GPU)."""
import numpy as np

import bench
from synth import corpus


def test_work_model_counts():
    b = corpus.make_batch(2, sizes=([70, 0, 130, 5], [64, 9, 65, 200]))
    model, cells, n_kc = bench.work_model(b)
    assert cells == 70 * 64 + 0 + 130 * 65 + 5 * 200
    assert model["nw_fill"][1] == 4.25 * cells
    # compacted chunks by brute force: row tiles x ceil(distinct target words / 32) per column tile
    tf = np.concatenate([[0], np.cumsum(b.m)])
    want = 0
    for p in range(b.B):
        n, m = int(b.n[p]), int(b.m[p])
        if n == 0 or m == 0:
            continue
        for c0 in range(0, m, 64):
            words = set()
            for j in range(c0, min(m, c0 + 64)):
                s = tf[p] + j
                words |= set(b.tgt_tok[b.tgt_off[s]:b.tgt_off[s + 1]].tolist())
            want += ((n + 63) // 64) * ((len(words) + 31) // 32)
    assert n_kc == want
    assert model["score"] == ("mfma", 2.0 * 64 * 64 * 32 * want, model["score"][2])
    for k, (bound, work, _) in model.items():
        assert bound in ("hbm", "mfma") and work > 0, k


def test_rooflines_and_dominant():
    b = corpus.make_batch(2, pairs=16)
    model, cells, _ = bench.work_model(b)
    kernel_ms = {"score": 0.2, "nw_fill": 0.5, "merge": 0.1, "walk": 0.05}
    rl = bench.rooflines(model, kernel_ms, "bf16")
    assert set(rl) == set(kernel_ms)
    assert rl["nw_fill"]["unit"] == "GB/s" and rl["score"]["unit"] == "TFLOP/s"
    ach = 4.25 * cells / 0.5e-3 / 1e9
    assert abs(rl["nw_fill"]["achieved"] - round(ach, 2)) < 1e-6
    assert abs(rl["nw_fill"]["frac"] - round(ach / 8000.0, 4)) < 1e-9
    assert max(rl, key=lambda k: rl[k]["kernel_ms"]) == "nw_fill"
    assert isinstance(bench.cpu_model(), str)
