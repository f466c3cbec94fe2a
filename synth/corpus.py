"""Seeded synthetic comparable corpora with a planted sentence alignment.

This module only draws input data.  It holds none of the mining method's
arithmetic (no scoring, no alignment): it is the one module shared by the CPU
oracle, the HIP path, the tests and the benchmark.

The paper mines Wikipedia article pairs with a classifier trained on TED data
(Sec. 4) and times 1,000 random article pairs (Sec. 5.4, Table 4).  None of that
data exists here; every workload is a seeded stand-in with the shapes below.

Recipe (all draws from ``numpy.random.default_rng([151201641, cfg, stream, idx])``):

* stream 0: per-pair sentence counts ``n`` (source) and ``m`` (target);
* stream 1: the bilingual dictionary ``D`` (V x V, ``deg`` distinct targets
  per source word, Dirichlet(1) weights drawn in FP64, stored FP32);
* stream 2: the scorer ``(w0, w1, b) ~ N(0, 1)``, FP32;
* stream 3, idx=b: the content of document pair ``b``.

Token ids are Zipf(s) over ranks 1..V (P(r) ~ r^-s, id = r-1), independently
per language.  Sentence lengths are uniform on {5..40}.  A target document is
made from its source document by deleting ``del`` source sentences, translating
every kept source token through ``D`` with probability 0.8 (else a random target
Zipf token; length is preserved) and inserting ``ins`` fresh random target
sentences at uniform positions, with ``ins - del = m - n`` and
``ins + del ~= round(0.3 n)``.  The planted alignment is the monotone map from
kept source sentences to their translations.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 151201641

# Workload shapes.  sizes: ("fixed", n, m) or ("lognormal", median, lo, hi).
CONFIGS = {
    1: dict(pairs=1, V=2048, zipf=1.1, sizes=("fixed", 200, 220), tiny=0.0),
    2: dict(pairs=4096, V=4096, zipf=1.1, sizes=("lognormal", 60, 20, 2000), tiny=0.0),
    3: dict(pairs=256, V=16384, zipf=1.1, sizes=("fixed", 5000, 5000), tiny=0.0),
    4: dict(pairs=1024, V=4096, zipf=1.1, sizes=("lognormal", 80, 1, 1000), tiny=0.0),
    5: dict(pairs=100000, V=16384, zipf=1.05, sizes=("lognormal", 60, 1, 4000), tiny=0.08),
}

LEN_LO, LEN_HI = 5, 40          # sentence length range (tokens), inclusive
LOGNORMAL_SIGMA = 1.0
SKEW = 0.3                      # +-30 % target/source length skew
INDEL_RATE = 0.3                # insertion + deletion events per source sentence
TOKEN_NOISE = 0.2               # probability a translated token is random noise
DICT_DEG = 4                    # translations per source word
GAP = -0.2
THRESHOLD = 0.5


def _rng(cfg: int, stream: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED, cfg, stream, idx])


@dataclasses.dataclass
class Batch:
    """A batch of document pairs, all arrays host NumPy.

    Sentences of all pairs are concatenated in pair order; pair ``b`` owns
    source sentences ``[sum(n[:b]), sum(n[:b+1]))``.  ``src_off`` is the CSR
    token offset array over all source sentences (length ``sum(n)+1``).
    """
    cfg: int
    V: int
    n: np.ndarray            # int32 [B]
    m: np.ndarray            # int32 [B]
    src_off: np.ndarray      # int64 [sum n + 1]
    src_tok: np.ndarray      # int32
    tgt_off: np.ndarray      # int64 [sum m + 1]
    tgt_tok: np.ndarray      # int32
    d_row_off: np.ndarray    # int32 [V+1]
    d_col: np.ndarray        # int32 [nnz]
    d_val: np.ndarray        # float32 [nnz]
    d_deg: int               # max entries per dictionary row
    scorer: np.ndarray       # float32 [3] = (w0, w1, b)
    gold_off: np.ndarray     # int64 [B+1]
    gold: np.ndarray         # int32 [G, 2] planted (i, j), 0-based, ascending
    gap: float = GAP
    threshold: float = THRESHOLD

    @property
    def B(self) -> int:
        return int(self.n.shape[0])

    def cells(self) -> int:
        return int(np.dot(self.n.astype(np.int64), self.m.astype(np.int64)))

    def subset(self, idx) -> "Batch":
        """A new batch holding pairs ``idx`` (in that order)."""
        idx = np.asarray(idx, dtype=np.int64)
        sfirst = np.concatenate([[0], np.cumsum(self.n, dtype=np.int64)])
        tfirst = np.concatenate([[0], np.cumsum(self.m, dtype=np.int64)])
        s_sent, t_sent, golds = [], [], []
        for b in idx:
            s_sent.append(np.arange(sfirst[b], sfirst[b + 1]))
            t_sent.append(np.arange(tfirst[b], tfirst[b + 1]))
            golds.append(self.gold[self.gold_off[b]:self.gold_off[b + 1]])
        s_sent = np.concatenate(s_sent) if s_sent else np.zeros(0, np.int64)
        t_sent = np.concatenate(t_sent) if t_sent else np.zeros(0, np.int64)
        src_off, src_tok = _gather_csr(self.src_off, self.src_tok, s_sent)
        tgt_off, tgt_tok = _gather_csr(self.tgt_off, self.tgt_tok, t_sent)
        gl = np.array([len(g) for g in golds], dtype=np.int64)
        return dataclasses.replace(
            self, n=self.n[idx].copy(), m=self.m[idx].copy(),
            src_off=src_off, src_tok=src_tok, tgt_off=tgt_off, tgt_tok=tgt_tok,
            gold_off=np.concatenate([[0], np.cumsum(gl)]).astype(np.int64),
            gold=(np.concatenate(golds) if golds else np.zeros((0, 2), np.int32)).astype(np.int32).reshape(-1, 2))


def _gather_csr(off, vals, rows):
    lens = (off[rows + 1] - off[rows]).astype(np.int64)
    new_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    if len(rows) == 0 or new_off[-1] == 0:
        return new_off, np.zeros(0, np.int32)
    starts = np.repeat(off[rows] - new_off[:-1], lens)
    return new_off, vals[np.arange(new_off[-1]) + starts].astype(np.int32)


def zipf_cdf(V: int, s: float) -> np.ndarray:
    r = np.arange(1, V + 1, dtype=np.float64)
    p = r ** (-s)
    c = np.cumsum(p)
    return c / c[-1]


def _zipf(rng, cdf, size):
    ids = np.searchsorted(cdf, rng.random(size), side="right")
    return np.minimum(ids, len(cdf) - 1).astype(np.int32)


def make_dictionary(cfg: int, V: int, deg: int = DICT_DEG):
    """Sparse row-stochastic dictionary: ``deg`` distinct targets per source id."""
    rng = _rng(cfg, 1)
    cols = rng.integers(0, V, size=(V, deg))
    for _ in range(1000):
        s = np.sort(cols, axis=1)
        bad = np.any(s[:, 1:] == s[:, :-1], axis=1)
        if not bad.any():
            break
        cols[bad] = rng.integers(0, V, size=(int(bad.sum()), deg))
    w = rng.dirichlet(np.ones(deg), size=V)
    row_off = (np.arange(V + 1) * deg).astype(np.int32)
    return row_off, cols.reshape(-1).astype(np.int32), w.reshape(-1).astype(np.float32)


def make_scorer(cfg: int) -> np.ndarray:
    return _rng(cfg, 2).standard_normal(3).astype(np.float32)


def make_sizes(cfg: int, pairs: int | None = None):
    c = CONFIGS[cfg]
    B = c["pairs"] if pairs is None else pairs
    kind = c["sizes"]
    if kind[0] == "fixed":
        return np.full(B, kind[1], np.int32), np.full(B, kind[2], np.int32)
    _, med, lo, hi = kind
    rng = _rng(cfg, 0)
    n = np.clip(np.rint(rng.lognormal(math.log(med), LOGNORMAL_SIGMA, B)), lo, hi)
    m = np.clip(np.rint(n * rng.uniform(1 - SKEW, 1 + SKEW, B)), lo, hi)
    if c["tiny"] > 0:
        tiny = rng.random(B) < c["tiny"]
        side = rng.integers(0, 2, B)
        small = rng.integers(0, 5, B)
        n = np.where(tiny & (side == 0), small, n)
        m = np.where(tiny & (side == 1), small, m)
    return n.astype(np.int32), m.astype(np.int32)


def indel_counts(n: int, m: int):
    """(deletions, insertions) with ins - del = m - n and ins + del ~ 0.3 n."""
    E = int(round(INDEL_RATE * n))
    diff = m - n
    dele = max(0, (E - diff) // 2)
    ins = dele + diff
    if ins < 0:
        ins, dele = 0, n - m
    return dele, ins


def make_pair(cfg: int, b: int, n: int, m: int, V: int, cdf, d_col2, d_cum2,
              noise=TOKEN_NOISE, indels=True):
    """Content of document pair ``b``: (src_lens, src_tok, tgt_lens, tgt_tok, gold)."""
    rng = _rng(cfg, 3, b)
    s_len = rng.integers(LEN_LO, LEN_HI + 1, size=n)
    s_tok = _zipf(rng, cdf, int(s_len.sum()))
    if indels:
        dele, ins = indel_counts(n, m)
    else:
        dele, ins = max(0, n - m), max(0, m - n)
    deleted = np.sort(rng.choice(n, size=dele, replace=False)) if dele else np.zeros(0, np.int64)
    keep = np.ones(n, bool)
    keep[deleted] = False
    kept_src = np.nonzero(keep)[0]
    # translate kept sentences token by token
    s_first = np.concatenate([[0], np.cumsum(s_len)])
    tok_sent = np.repeat(np.arange(n), s_len)
    ktok_mask = keep[tok_sent]
    kt = s_tok[ktok_mask]
    K = kt.shape[0]
    coin = rng.random(K) >= noise
    r = rng.random(K)
    pick = (r[:, None] > d_cum2[kt, :-1]).sum(axis=1)
    u_tr = d_col2[kt, pick]
    u_noise = _zipf(rng, cdf, K)
    tr_tok = np.where(coin, u_tr, u_noise).astype(np.int32)
    tr_len = s_len[kept_src]
    # insertions at uniform target positions
    slots = np.zeros(m, bool)
    if ins:
        slots[rng.choice(m, size=ins, replace=False)] = True
    ins_len = rng.integers(LEN_LO, LEN_HI + 1, size=ins)
    ins_tok = _zipf(rng, cdf, int(ins_len.sum()))
    # assemble target document
    t_len = np.zeros(m, np.int64)
    t_len[~slots] = tr_len
    t_len[slots] = ins_len
    t_first = np.concatenate([[0], np.cumsum(t_len)])
    t_tok = np.empty(int(t_first[-1]), np.int32)
    tr_first = np.concatenate([[0], np.cumsum(tr_len)])
    ins_first = np.concatenate([[0], np.cumsum(ins_len)])
    tr_slots = np.nonzero(~slots)[0]
    ins_slots = np.nonzero(slots)[0]
    # vectorised scatter of both token streams into place
    if len(tr_slots):
        dst = np.repeat(t_first[tr_slots] - tr_first[:-1], tr_len) + np.arange(tr_first[-1])
        t_tok[dst] = tr_tok
    if len(ins_slots):
        dst = np.repeat(t_first[ins_slots] - ins_first[:-1], ins_len) + np.arange(ins_first[-1])
        t_tok[dst] = ins_tok
    gold = np.stack([kept_src, tr_slots], axis=1).astype(np.int32) if len(kept_src) else np.zeros((0, 2), np.int32)
    del s_first
    return s_len, s_tok, t_len, t_tok, gold


def make_batch(cfg: int, pairs: int | None = None, first: int = 0, V: int | None = None,
               noise: float = TOKEN_NOISE, indels: bool = True, sizes=None) -> Batch:
    """Build ``pairs`` document pairs (default: the config's count) starting at pair ``first``.

    Pair ``b`` depends only on ``(cfg, b)`` and its sizes, so any slice of a
    config can be generated on its own.
    """
    c = CONFIGS[cfg]
    V = c["V"] if V is None else V
    if sizes is None:
        n_all, m_all = make_sizes(cfg, (first + pairs) if pairs is not None else None)
        n_all, m_all = n_all[first:], m_all[first:]
    else:
        n_all, m_all = (np.asarray(x, np.int32) for x in sizes)
    B = len(n_all)
    cdf = zipf_cdf(V, c["zipf"])
    d_row_off, d_col, d_val = make_dictionary(cfg, V)
    d_col2 = d_col.reshape(V, DICT_DEG)
    d_cum2 = np.cumsum(d_val.reshape(V, DICT_DEG).astype(np.float64), axis=1)
    s_lens, s_toks, t_lens, t_toks, golds = [], [], [], [], []
    for k in range(B):
        sl, st, tl, tt, g = make_pair(cfg, first + k, int(n_all[k]), int(m_all[k]), V, cdf,
                                      d_col2, d_cum2, noise=noise, indels=indels)
        s_lens.append(sl); s_toks.append(st); t_lens.append(tl); t_toks.append(tt); golds.append(g)
    cat = lambda xs, dt: (np.concatenate(xs) if xs else np.zeros(0)).astype(dt)
    s_len = cat(s_lens, np.int64)
    t_len = cat(t_lens, np.int64)
    gl = np.array([len(g) for g in golds], np.int64)
    return Batch(
        cfg=cfg, V=V, n=n_all.astype(np.int32), m=m_all.astype(np.int32),
        src_off=np.concatenate([[0], np.cumsum(s_len)]).astype(np.int64),
        src_tok=cat(s_toks, np.int32),
        tgt_off=np.concatenate([[0], np.cumsum(t_len)]).astype(np.int64),
        tgt_tok=cat(t_toks, np.int32),
        d_row_off=d_row_off, d_col=d_col, d_val=d_val, d_deg=DICT_DEG,
        scorer=make_scorer(cfg),
        gold_off=np.concatenate([[0], np.cumsum(gl)]).astype(np.int64),
        gold=(np.concatenate(golds) if golds else np.zeros((0, 2))).astype(np.int32).reshape(-1, 2),
    )


def reverse_dictionary(b: Batch, deg: int = DICT_DEG):
    """A target-to-source dictionary drawn from the same translation table:
    row u lists the source words t whose forward row holds u, keeping the
    ``deg`` largest weights D[t][u] (ties: smaller t first), rescaled to sum
    to 1.  Target words no source word translates to get an empty row."""
    V = b.V
    src = np.repeat(np.arange(V, dtype=np.int64), np.diff(b.d_row_off))
    u = b.d_col.astype(np.int64)
    w = b.d_val.astype(np.float64)
    order = np.lexsort((src, -w, u))          # by target word, then weight desc, then source word
    u, src, w = u[order], src[order], w[order]
    first = np.concatenate([[0], np.flatnonzero(np.diff(u)) + 1])
    rank = np.arange(len(u)) - np.repeat(first, np.diff(np.concatenate([first, [len(u)]])))
    keep = rank < deg
    u, src, w = u[keep], src[keep], w[keep]
    cnt = np.bincount(u, minlength=V)
    row_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    tot = np.repeat(np.add.reduceat(w, row_off[:-1][cnt > 0]), cnt[cnt > 0])
    return row_off, src.astype(np.int32), (w / tot).astype(np.float32)


def reverse_batch(b: Batch) -> Batch:
    """The same document pairs seen from the other side: target sentences as
    the source side, the reverse dictionary, planted pairs as (j, i)."""
    d_row_off, d_col, d_val = reverse_dictionary(b)
    gold = b.gold[:, ::-1].copy() if len(b.gold) else b.gold.reshape(-1, 2).copy()
    golds = []
    for k in range(b.B):
        g = gold[b.gold_off[k]:b.gold_off[k + 1]]
        golds.append(g[np.argsort(g[:, 0], kind="stable")])
    return dataclasses.replace(
        b, n=b.m.copy(), m=b.n.copy(), src_off=b.tgt_off, src_tok=b.tgt_tok, tgt_off=b.src_off, tgt_tok=b.src_tok,
        d_row_off=d_row_off, d_col=d_col, d_val=d_val,
        d_deg=int(np.diff(d_row_off).max()) if len(d_row_off) > 1 else 0,
        gold=(np.concatenate(golds) if golds else gold).astype(np.int32).reshape(-1, 2))


def identity_batch(cfg: int, n: int, V: int = 2048, b: int = 0) -> Batch:
    """Source document with its exact translation through a permutation
    dictionary (one target per word, weight 1), no noise and no indels.
    Sentences are made pairwise distinct (as token sets)."""
    rng = _rng(cfg, 9, b)
    perm = rng.permutation(V).astype(np.int32)
    cdf = zipf_cdf(V, 1.1)
    lens, toks, seen = [], [], set()
    while len(lens) < n:
        L = int(rng.integers(LEN_LO, LEN_HI + 1))
        t = _zipf(rng, cdf, L)
        key = frozenset(t.tolist())
        if key in seen:
            continue
        seen.add(key)
        lens.append(L); toks.append(t)
    s_len = np.array(lens, np.int64)
    s_tok = np.concatenate(toks).astype(np.int32)
    t_tok = perm[s_tok]
    off = np.concatenate([[0], np.cumsum(s_len)]).astype(np.int64)
    gold = np.stack([np.arange(n), np.arange(n)], 1).astype(np.int32)
    return Batch(cfg=cfg, V=V, n=np.array([n], np.int32), m=np.array([n], np.int32),
                 src_off=off, src_tok=s_tok, tgt_off=off.copy(), tgt_tok=t_tok,
                 d_row_off=np.arange(V + 1, dtype=np.int32), d_col=perm.copy(),
                 d_val=np.ones(V, np.float32), d_deg=1,
                 scorer=np.array([4.0, 0.0, -1.0], np.float32),
                 gold_off=np.array([0, n], np.int64), gold=gold)
