"""Write tests/golden/oriented_scorer.json (run: python tests/golden/make_oriented_scorer.py).

The seeded N(0,1) scorer says little about translation (its sign is random),
so planted-alignment F1 is checked with an "oriented" scorer calibrated once
by the CPU oracle: w1 = 0 and (w0, b) chosen so that the median planted
sentence pair has z = +1 and the median non-planted pair z = -1, on 64 seeded
60 x 60 pairs generated with each workload's vocabulary size and Zipf
exponent.  Only the oracle and the input generator are used.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from synth import corpus  # noqa: E402


def calibrate(cfg):
    c = corpus.CONFIGS[cfg]
    b = corpus.make_batch(cfg, pairs=64, sizes=(np.full(64, 60), np.full(64, 60)))
    sc = oracle.score(b, scorer=[1.0, 0.0, 0.0])
    S_raw = sc["S_raw"]
    gold = np.zeros(S_raw.shape[0], bool)
    for q in range(b.B):
        g = b.gold[b.gold_off[q]:b.gold_off[q + 1]]
        gold[sc["s_off"][q] + g[:, 0].astype(np.int64) * b.m[q] + g[:, 1]] = True
    sp = float(np.median(S_raw[gold]))
    sr = float(np.median(S_raw[~gold]))
    w0 = 2.0 / (sp - sr)
    bias = -1.0 - w0 * sr
    return {"w": [w0, 0.0, bias], "median_planted_sraw": sp, "median_other_sraw": sr, "V": c["V"],
            "zipf": c["zipf"]}


def main():
    out = {"_source": "tests/golden/make_oriented_scorer.py (CPU oracle calibration, seeded)"}
    for cfg in sorted(corpus.CONFIGS):
        out[str(cfg)] = calibrate(cfg)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oriented_scorer.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
