"""CPU oracle for the mining hot path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It shares no code with the HIP path: the arithmetic lives in
``nwm_oracle.c`` (scores in FP64, DP in FP32 with one fixed per-cell operation
order), the exact brute force in ``brute.py`` and the planted-alignment F1
below.  ``build()`` compiles the C file with gcc.

Functions and the passages they follow (Wolk & Marasek, arXiv 1512.01641):
  score()    -- Sec. 4: classifier likelihood normalised into [0,1] (SVM
                distance through a sigmoid) over a dictionary with translation
                probabilities.  Features are the dictionary-coverage contraction
                S_raw = ((X.D).Y^T) and the length ratio rho (a reading: the
                paper does not list its features).
  align()    -- Sec. 5.1 (Figs. 1-2, eq. (1)) NW fill + traceback, and Sec. 4's
                threshold filter (keep iff S >= threshold).
  backward() -- subgradient of the NW score (path indicator, gap count) chained
                through the sigmoid scorer; drives the tuning of Sec. 5.2.
  f1()       -- micro F1 of kept pairs against the planted alignment.
  union_kept() -- Sec. 5.4 / Table 3 "BI": bi-directional mining keeps the
                pairs either direction's classifier keeps; read here as the
                set union of the two kept sets (each sentence pair once),
                the reverse direction's (target, source) pairs swapped.
  similarity() -- Sec. 5.2: how closely an automatic alignment resembles a
                reference one, by NW over the two aligned-pair sequences
                (match 1, mismatch and gaps 0), in percent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nwm_oracle.c")
_LIB = os.path.join(_HERE, "libnwm_oracle.so")
_lib = None

DIAG, UP, LEFT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fexcess-precision=standard", "-fopenmp", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        F = ctypes.c_float
        lib.nwo_score.argtypes = [I, I, P, P, P, P, P, P, P, P, P, D, D, D, P, P, P, P, P, I]
        lib.nwo_score.restype = I
        lib.nwo_align.argtypes = [I, P, P, P, P, F, F, P, P, P, P, P, P, P, P, I]
        lib.nwo_align.restype = I
        lib.nwo_backward.argtypes = [I, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
        lib.nwo_backward.restype = I
        lib.nwo_max_threads.restype = I
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().nwo_max_threads())


def s_offsets(n, m) -> np.ndarray:
    """Element offset of each pair's n x m block in a packed S array (+ total)."""
    c = np.asarray(n, np.int64) * np.asarray(m, np.int64)
    return np.concatenate([[0], np.cumsum(c)]).astype(np.int64)


def path_offsets(n, m) -> np.ndarray:
    """Pair offset of each pair's aligned-pair list (capacity min(n, m))."""
    c = np.minimum(np.asarray(n, np.int64), np.asarray(m, np.int64))
    return np.concatenate([[0], np.cumsum(c)]).astype(np.int64)


def score(batch, scorer=None, nthreads: int = 0):
    """FP64 similarity of every sentence pair of every document pair.

    Returns dict with S_raw, rho, S64 (float64) and S32 (float32), packed by
    ``s_off`` (pair b at ``s_off[b]``, row-major n_b x m_b)."""
    lib = _load()
    w = np.asarray(batch.scorer if scorer is None else scorer, np.float64)
    n = np.ascontiguousarray(batch.n, np.int32)
    m = np.ascontiguousarray(batch.m, np.int32)
    s_off = s_offsets(n, m)
    tot = int(s_off[-1])
    S_raw = np.empty(tot, np.float64)
    rho = np.empty(tot, np.float64)
    S64 = np.empty(tot, np.float64)
    S32 = np.empty(tot, np.float32)
    arrs = [np.ascontiguousarray(a) for a in (batch.src_off, batch.src_tok, batch.tgt_off, batch.tgt_tok,
                                              batch.d_row_off, batch.d_col, batch.d_val)]
    rc = lib.nwo_score(len(n), int(batch.V), _p(n), _p(m), *[_p(a) for a in arrs],
                       float(w[0]), float(w[1]), float(w[2]), _p(s_off),
                       _p(S_raw), _p(rho), _p(S64), _p(S32), int(nthreads))
    if rc:
        raise RuntimeError("nwo_score failed: %d" % rc)
    return dict(S_raw=S_raw, rho=rho, S64=S64, S32=S32, s_off=s_off)


def align(n, m, S32, gap: float, threshold: float, nthreads: int = 0, matrices: bool = False):
    """NW fill + traceback + threshold filter for every pair.

    ``S32`` is the packed FP32 similarity (pair b at ``s_offsets(n,m)[b]``).
    Returns dict: score [B] f32, n_diag [B], n_kept [B], path_off [B+1],
    path / kept (int32 [cap, 2], pair b's rows start at path_off[b]) and, if
    ``matrices``, pair 0's full H and T matrices."""
    lib = _load()
    n = np.ascontiguousarray(n, np.int32)
    m = np.ascontiguousarray(m, np.int32)
    B = len(n)
    s_off = s_offsets(n, m)
    p_off = path_offsets(n, m)
    S32 = np.ascontiguousarray(S32, np.float32)
    assert S32.shape[0] >= s_off[-1]
    score_ = np.empty(B, np.float32)
    n_diag = np.empty(B, np.int32)
    n_kept = np.empty(B, np.int32)
    path = np.zeros((max(int(p_off[-1]), 1), 2), np.int32)
    kept = np.zeros((max(int(p_off[-1]), 1), 2), np.int32)
    H = T = None
    if matrices and B:
        cells = (int(n[0]) + 1) * (int(m[0]) + 1)
        H = np.empty(cells, np.float32)
        T = np.empty(cells, np.uint8)
    rc = lib.nwo_align(B, _p(n), _p(m), _p(s_off), _p(S32), float(gap), float(threshold), _p(p_off),
                       _p(score_), _p(n_diag), _p(path), _p(kept), _p(n_kept), _p(H), _p(T), int(nthreads))
    if rc:
        raise RuntimeError("nwo_align failed: %d" % rc)
    out = dict(score=score_, n_diag=n_diag, n_kept=n_kept, path_off=p_off, path=path, kept=kept)
    if matrices and B:
        out["H"] = H.reshape(int(n[0]) + 1, int(m[0]) + 1)
        out["T"] = T.reshape(int(n[0]) + 1, int(m[0]) + 1)
    return out


def pair_path(res, b):
    """Aligned (DIAG) pairs of pair b as an int32 [k, 2] array."""
    o = int(res["path_off"][b])
    return res["path"][o:o + int(res["n_diag"][b])]


def pair_kept(res, b):
    o = int(res["path_off"][b])
    return res["kept"][o:o + int(res["n_kept"][b])]


def backward(n, m, res, grad_score, S64, S_raw, rho, grad_S_extra=None, want_grad_S=True):
    """FP64 backward of sum_b grad_score[b] * Score_b (+ <grad_S_extra, S>).

    Returns dict(grad_S (or None), grad_gap, grad_wb[3])."""
    lib = _load()
    n = np.ascontiguousarray(n, np.int32)
    m = np.ascontiguousarray(m, np.int32)
    s_off = s_offsets(n, m)
    a = np.ascontiguousarray(grad_score, np.float64)
    E = None if grad_S_extra is None else np.ascontiguousarray(grad_S_extra, np.float64)
    gS = np.empty(int(s_off[-1]), np.float64) if want_grad_S else None
    gg = np.zeros(1, np.float64)
    gwb = np.zeros(3, np.float64)
    rc = lib.nwo_backward(len(n), _p(n), _p(m), _p(s_off), _p(res["path_off"]), _p(res["path"]),
                          _p(np.ascontiguousarray(res["n_diag"], np.int32)), _p(a), _p(E),
                          _p(np.ascontiguousarray(S64)), _p(np.ascontiguousarray(S_raw)),
                          _p(np.ascontiguousarray(rho)), _p(gS), _p(gg), _p(gwb))
    if rc:
        raise RuntimeError("nwo_backward failed")
    return dict(grad_S=gS, grad_gap=float(gg[0]), grad_wb=gwb)


def f1(kept_sets, gold_sets) -> float:
    """Micro F1 (in points) of kept pairs against planted pairs over a batch.

    TP = |K & G|, P = TP/|K|, R = TP/|G|, F1 = 2PR/(P+R); 0 if TP = 0;
    100 if both K and G are empty."""
    tp = nk = ng = 0
    for K, G in zip(kept_sets, gold_sets):
        K = set(map(tuple, np.asarray(K).reshape(-1, 2).tolist()))
        G = set(map(tuple, np.asarray(G).reshape(-1, 2).tolist()))
        tp += len(K & G)
        nk += len(K)
        ng += len(G)
    if nk == 0 and ng == 0:
        return 100.0
    if tp == 0:
        return 0.0
    P = tp / nk
    R = tp / ng
    return 200.0 * P * R / (P + R)


def union_kept(kept_fwd, kept_rev):
    """Per document pair: the sentence pairs kept by the forward direction
    (i, j) or by the reverse direction (given as (j, i)), each once, in
    ascending (i, j) order.  Arguments: sequences of [k, 2] arrays."""
    out = []
    for F, R in zip(kept_fwd, kept_rev):
        F = np.asarray(F, np.int64).reshape(-1, 2)
        R = np.asarray(R, np.int64).reshape(-1, 2)
        u = set(map(tuple, F.tolist())) | set((j, i) for i, j in R.tolist())
        out.append(np.array(sorted(u), np.int32).reshape(-1, 2))
    return out


def _nw_match_count(A, G) -> int:
    """NW over two sequences of aligned pairs, match 1, mismatch 0, gaps 0:
    the best total is the number of matched pairs.  Row by row: with gaps
    free, a row of the DP is the running maximum of max(up, diag + match)."""
    if len(A) == 0 or len(G) == 0:
        return 0
    keyA = [tuple(x) for x in np.asarray(A).reshape(-1, 2).tolist()]
    keyG = [tuple(x) for x in np.asarray(G).reshape(-1, 2).tolist()]
    prev = np.zeros(len(keyG) + 1, np.int64)
    for a in keyA:
        match = np.fromiter((1 if g == a else 0 for g in keyG), np.int64, len(keyG))
        cur = np.empty_like(prev)
        cur[0] = 0
        cur[1:] = np.maximum(prev[1:], prev[:-1] + match)
        prev = np.maximum.accumulate(cur)
    return int(prev[-1])


def similarity(auto_sets, ref_sets) -> float:
    """Sec. 5.2: resemblance (percent) of automatic alignments to reference
    ones, the sentence-pair sequences compared by NW (match 1, else 0):
    100 * 2 * sum_b M_b / sum_b (|A_b| + |G_b|), M_b the NW optimum of pair b;
    100 when both sides are empty everywhere."""
    m = tot = 0
    for A, G in zip(auto_sets, ref_sets):
        A = np.asarray(A).reshape(-1, 2)
        G = np.asarray(G).reshape(-1, 2)
        m += _nw_match_count(A, G)
        tot += len(A) + len(G)
    return 100.0 if tot == 0 else 200.0 * m / tot
