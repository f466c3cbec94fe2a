"""Gradient tuning of the scorer, the gap and the threshold against reference
alignments (the paper tunes threshold and penalty against human alignments,
Sec. 5.2; planted alignments of the synthetic corpora stand in for them).

Loss per document pair b (a structured hinge, >= 0):
    L_b = Score_b(S, g) - Gold_b(S, g),
    Gold_b = sum_{(i,j) in G*_b} S[i][j] + g * (n_b + m_b - 2 |G*_b|),
i.e. the NW optimum minus the score of the reference alignment seen as an NW
path.  L_b = 0 iff the reference path is optimal.  Gradients:
    dL/dS = P_b - 1[G*_b]  (through the sigmoid scorer to w0, w1, b),
    dL/dg = (n_b + m_b - 2 k_b) - (n_b + m_b - 2 |G*_b|).
The library computes the path term and the dense -1[G*] term in one
nwm_align_backward call (grad_S_extra), FP64-reduced over the batch.
The threshold is then set by a 1-D search maximising kept-pair F1.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import Miner, align_backward


class Tuner:
    def __init__(self, miner: Miner, gold_off, gold, w0=(1.0, 0.0, 0.0), gap=-0.2, threshold=0.5,
                 lr_w=0.05, lr_g=0.01):
        self.mn = miner
        self.gold_off = np.asarray(gold_off, np.int64)
        self.gold = np.asarray(gold, np.int32).reshape(-1, 2)
        self.w = np.asarray(w0, np.float64).copy()
        self.gap = float(gap)
        self.threshold = float(threshold)
        self.lr_w, self.lr_g = lr_w, lr_g
        self.step_no = 0
        b = miner.batch
        dev = miner.ctx.device
        n = b.n.astype(np.int64)
        m = b.m.astype(np.int64)
        gl = np.diff(self.gold_off)
        self.gold_gaps = float(np.sum(n + m - 2 * gl))
        # dense -1[G*] in the S layout (host logic of the tuning loop)
        pair = np.repeat(np.arange(b.B), gl)
        flat = miner.s_off[pair] + self.gold[:, 0].astype(np.int64) * m[pair] + self.gold[:, 1]
        E = torch.zeros(max(miner.plan.S_elems, 1), dtype=torch.float32, device=dev)
        if len(flat):
            E[torch.as_tensor(flat, device=dev)] = -1.0
        self.E = E
        self.gold_flat = torch.as_tensor(flat, device=dev)
        self.ones = torch.ones(max(b.B, 1), dtype=torch.float32, device=dev)

    def loss_and_grad(self):
        mn = self.mn
        B = mn.batch.B
        mn.mine(self.w.astype(np.float32), self.gap, self.threshold, want_raw=True)
        dev = mn.ctx.device
        gwb = torch.zeros(3, dtype=torch.float64, device=dev)
        gg = torch.zeros(1, dtype=torch.float64, device=dev)
        align_backward(mn.plan, mn.batch, mn.tb, mn.n_diag, self.ones[:max(B, 1)], grad_S_extra=self.E,
                       grad_gap=gg, S=mn.S, S_raw=mn.S_raw, scorer=self.w.astype(np.float32), grad_wb=gwb, ws=mn.ws)
        score_sum = float(mn.score[:B].double().sum().item())
        gold_S = float(mn.S[self.gold_flat].double().sum().item()) if len(self.gold_flat) else 0.0
        loss = score_sum - (gold_S + self.gap * self.gold_gaps)
        grad_w = gwb.cpu().numpy()
        grad_g = float(gg.item()) - self.gold_gaps
        return loss, grad_w, grad_g

    def best_threshold(self, grid=None):
        """Threshold maximising micro F1 of kept pairs against the reference."""
        mn = self.mn
        B = mn.batch.B
        grid = np.linspace(0.05, 0.95, 19) if grid is None else grid
        # every aligned pair is kept at threshold -inf: read the path once
        mn.align(self.gap, -3.0e38)
        torch.cuda.synchronize()
        nk = mn.n_kept[:B].cpu().numpy()
        kept = mn.kept.cpu().numpy()
        S = mn.S
        rows = []
        for b in range(B):
            o = int(mn.p_off[b])
            rows.append(kept[o:o + int(nk[b])])
        allp = np.concatenate(rows) if rows else np.zeros((0, 2), np.int32)
        pair = np.repeat(np.arange(B), nk)
        flat = mn.s_off[pair] + allp[:, 0].astype(np.int64) * mn.batch.m[pair] + allp[:, 1]
        sv = S[torch.as_tensor(flat, device=S.device)].cpu().numpy() if len(flat) else np.zeros(0, np.float32)
        gold = set(zip(np.repeat(np.arange(B), np.diff(self.gold_off)).tolist(),
                       self.gold[:, 0].tolist(), self.gold[:, 1].tolist()))
        hit = np.array([(int(p), int(i), int(j)) in gold for p, (i, j) in zip(pair, allp)], bool)
        best = (self.threshold, -1.0)
        for t in grid:
            k = sv >= np.float32(t)
            tp = int(np.sum(hit & k))
            nk_ = int(np.sum(k))
            if tp == 0:
                f = 0.0
            else:
                P, R = tp / nk_, tp / max(len(gold), 1)
                f = 200.0 * P * R / (P + R)
            if f > best[1]:
                best = (float(t), f)
        self.threshold = best[0]
        return best

    def step(self):
        loss, gw, gg = self.loss_and_grad()
        self.w -= self.lr_w * gw
        self.gap = min(-1e-3, self.gap - self.lr_g * gg)
        self.step_no += 1
        return loss

    def state(self):
        return {"w": self.w.tolist(), "gap": self.gap, "threshold": self.threshold, "step": self.step_no}

    def save(self, path):
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.state(), f)
        os.replace(tmp, path)

    def load(self, path):
        with open(path) as f:
            s = json.load(f)
        self.w = np.asarray(s["w"], np.float64)
        self.gap = float(s["gap"])
        self.threshold = float(s["threshold"])
        self.step_no = int(s["step"])


def similarity(auto_sets, ref_sets) -> float:
    """Resemblance (percent) of automatic to reference alignments (Sec. 5.2:
    the two aligned-pair sequences compared by NW, match 1 and 0 otherwise).
    Both sequences of a document pair are strictly increasing in i and in j,
    so the NW optimum is the number of pairs they share:
    100 * 2 * sum |A & G| / sum (|A| + |G|), 100 if both are empty."""
    m = tot = 0
    for A, G in zip(auto_sets, ref_sets):
        A = np.asarray(A).reshape(-1, 2)
        G = np.asarray(G).reshape(-1, 2)
        if len(A) and len(G):
            ka = A[:, 0].astype(np.int64) << 32 | A[:, 1].astype(np.int64)
            kg = G[:, 0].astype(np.int64) << 32 | G[:, 1].astype(np.int64)
            m += len(np.intersect1d(ka, kg, assume_unique=True))
        tot += len(A) + len(G)
    return 100.0 if tot == 0 else 200.0 * m / tot


def random_search(miner: Miner, scorer, gold_off, gold, trials: int = 32, tau=(0.05, 0.95), gap=(-1.0, -0.01),
                  seed: int = 0):
    """The paper's tuning script (Sec. 5.2): naive random selection of the
    threshold and the gap penalty, keeping the pair whose alignments are most
    similar to the reference ones.  S does not depend on either, so the batch
    is scored once and each trial runs the DP + keep only.  Draws per trial:
    threshold ~ U(tau), then gap ~ U(gap), both rounded to FP32.  Returns the
    best (first on ties) and the history [(threshold, gap, similarity)]."""
    rng = np.random.default_rng(seed)
    B = miner.batch.B
    gold_off = np.asarray(gold_off, np.int64)
    gold = np.asarray(gold, np.int32).reshape(-1, 2)
    ref = [gold[gold_off[b]:gold_off[b + 1]] for b in range(B)]
    miner.score_pairs(scorer, want_raw=False)
    hist = []
    for _ in range(trials):
        th = float(np.float32(rng.uniform(*tau)))
        g = float(np.float32(rng.uniform(*gap)))
        miner.align(g, th)
        torch.cuda.synchronize()
        nk = miner.n_kept[:B].cpu().numpy()
        kept = miner.kept.cpu().numpy()
        auto = [kept[int(miner.p_off[b]):int(miner.p_off[b]) + int(nk[b])] for b in range(B)]
        hist.append((th, g, similarity(auto, ref)))
    best = max(range(len(hist)), key=lambda k: (hist[k][2], -k)) if hist else None
    out = {"history": hist}
    if best is not None:
        out.update(threshold=hist[best][0], gap=hist[best][1], similarity=hist[best][2])
    return out
