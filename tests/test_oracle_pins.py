"""Pins of the CPU oracle to facts other than itself (CPU only).

Each test names the passage or mathematical fact it checks:
  * the paper's worked examples (Sec. 5.1, Figs. 4 and 6; fixtures in
    tests/golden/paper_figures.json);
  * eq. (1)'s textbook scoring (+-1 match/mismatch, -2 gap) against exact
    brute force;
  * exact brute force over every alignment for n, m <= 6 with dyadic inputs;
  * closed forms, invariants (monotone, shift, scale, transpose, gap count);
  * the scorer against a dense NumPy (X.D).Y^T and special cases;
  * the backward against the subgradient inequality and finite differences.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
from synth import corpus

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_figures.json")


def _align1(S, g, thr=0.5, matrices=False):
    S = np.asarray(S, np.float32)
    n, m = S.shape if S.size else (S.shape[0], S.shape[1] if S.ndim == 2 else 0)
    r = oracle.align([n], [m], S.ravel(), g, thr, matrices=matrices)
    return float(r["score"][0]), [tuple(x) for x in oracle.pair_path(r, 0).tolist()], r


def _identity_S(rows, cols):
    return np.array([[1.0 if a == b else 0.0 for b in cols] for a in rows], np.float32)


def _fig(name):
    with open(GOLD) as f:
        return json.load(f)[name]


def _aligned_from_lines(cols_line, rows_line):
    """(row index, col index) of the columns of a printed alignment where both
    sides carry a word."""
    i = j = 0
    out = []
    for c, r in zip(cols_line, rows_line):
        if c != "-" and r != "-":
            out.append((i, j))
        if r != "-":
            i += 1
        if c != "-":
            j += 1
    return out


# --- Sec. 5.1, Figure 6 -------------------------------------------------------
@pytest.mark.parametrize("g", [-0.2, -0.125, -0.01, -0.24])
def test_fig6_alignment(g):
    fx = _fig("fig6")
    S = _identity_S(fx["rows"], fx["cols"])
    expect = [(fx["rows"].index(a), fx["cols"].index(b)) for a, b in fx["marked_cells"]]
    score, path, _ = _align1(S, g)
    assert path == expect
    exact, bpath, count = brute.best_alignment(S.tolist(), Fraction(g))
    assert count == 1 and bpath == expect
    assert abs(score - float(exact)) <= 4 * np.spacing(np.float32(abs(float(exact))))


def test_fig6_exact_scores():
    fx = _fig("fig6")
    S = _identity_S(fx["rows"], fx["cols"])
    # dyadic gap: every operation exact, score = 3 + 4g
    assert _align1(S, -0.125)[0] == 2.5
    # FP32 at g = -0.2: the FP32 sum along the path (no exact tie anywhere)
    assert np.float32(_align1(S, -0.2)[0]) == np.float32(2.1999998)
    # below -1/4 the pure diagonal (score 2) wins
    score, path, _ = _align1(S, -0.3)
    assert score == 2.0 and path == [(k, k) for k in range(5)]


# --- Sec. 5.1, Figure 4: the tie rule -------------------------------------------
def test_fig4_tie_break_reproduces_printed_alignment():
    fx = _fig("fig4")
    S = _identity_S(fx["rows"], fx["cols"])
    expect = _aligned_from_lines(fx["printed_cols_line"], fx["printed_rows_line"])
    exact, bpath, count = brute.best_alignment(S.tolist(), Fraction(-1, 8))
    assert count == 2, "Fig. 4 has two optimal alignments at g = -1/8"
    assert bpath == expect
    score, path, _ = _align1(S, -0.125)
    assert score == 2.5 and path == expect


def test_fig4_fp32_rounding_breaks_the_tie():
    # In FP32 at g = -0.2 the two optima differ by rounding: diag = 1.6f beats
    # up = 1.5999999f at cell (4,2), so the second "d" is aligned.
    fx = _fig("fig4")
    S = _identity_S(fx["rows"], fx["cols"])
    _, path, _ = _align1(S, -0.2)
    assert path == [(0, 0), (3, 1), (4, 2)]


# --- eq. (1): textbook NW scoring ---------------------------------------------
def test_eq1_textbook_scoring_vs_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n, m = rng.integers(0, 7, 2)
        a = rng.integers(0, 3, n)
        b = rng.integers(0, 3, m)
        S = np.where(a[:, None] == b[None, :], 1.0, -1.0).astype(np.float32).reshape(n, m)
        score, path, _ = _align1(S, -2.0)
        exact, bpath, _ = brute.best_alignment(S.tolist(), Fraction(-2), n, m)
        assert score == float(exact) and path == bpath


# --- exact brute force over all alignments -------------------------------------
@pytest.mark.parametrize("n", range(0, 7))
def test_brute_force_all_sizes(n):
    rng = np.random.default_rng(100 + n)
    for m in range(0, 7):
        assert len(brute.paths(n, m)) == brute.delannoy(n, m)
        for _ in range(2):
            S = (rng.integers(0, 65, (n, m)) / 64.0).astype(np.float32)
            g = -float(rng.integers(1, 41)) / 64.0
            score, path, _ = _align1(S, g)
            exact, bpath, _ = brute.best_alignment(S.tolist(), Fraction(g), n, m)
            assert score == float(exact), (n, m)
            assert path == bpath, (n, m)


def _moves_from_T(T, n, m):
    """Full move sequence (forward order) of the traceback through T."""
    i, j, rev = n, m, []
    while i > 0 or j > 0:
        d = "L" if i == 0 else "U" if j == 0 else "DUL"[T[i, j]]
        rev.append(d)
        i -= d in "DU"
        j -= d in "DL"
    return tuple(reversed(rev))


def test_brute_force_with_ties():
    # coarse values make many exact ties; the tie rule must pick the same
    # optimum move for move, gaps included
    rng = np.random.default_rng(5)
    for _ in range(80):
        n, m = rng.integers(1, 6, 2)
        S = (rng.integers(0, 3, (n, m)) / 2.0).astype(np.float32)
        g = -0.25
        score, path, r = _align1(S, g, matrices=True)
        exact, bpath, _ = brute.best_alignment(S.tolist(), Fraction(g), n, m)
        assert score == float(exact) and path == bpath
        assert _moves_from_T(r["T"], n, m) == brute.best_alignment.last_moves


# --- closed forms ---------------------------------------------------------------
@pytest.mark.parametrize("g", [-0.2, -0.7, -1.0 / 3.0])
def test_empty_sides(g):
    for n, m in [(0, 7), (9, 0), (0, 0)]:
        S = np.zeros((n, m), np.float32)
        score, path, _ = _align1(S, g)
        assert np.float32(score) == np.float32(np.float32(n + m) * np.float32(g))
        assert path == []


def test_constant_similarity_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(30):
        n, m = rng.integers(1, 40, 2)
        c = float(rng.integers(0, 33)) / 32.0
        g = -float(rng.integers(1, 17)) / 32.0
        score, path, _ = _align1(np.full((n, m), c, np.float32), g)
        assert score == min(n, m) * c + abs(int(n) - int(m)) * g
        assert len(path) == min(n, m)


# --- invariants -----------------------------------------------------------------
def _rand_instance(rng, n, m, dyadic=True):
    if dyadic:
        return (rng.integers(0, 257, (n, m)) / 256.0).astype(np.float32)
    return rng.random((n, m)).astype(np.float32)


def test_path_is_monotone_and_gap_identity():
    # NW paths never move up or left: no sentence is used twice (the failure
    # of unconstrained A* in Sec. 5.1, Figs. 3 and 5)
    rng = np.random.default_rng(7)
    for _ in range(30):
        n, m = rng.integers(0, 60, 2)
        S = _rand_instance(rng, n, m, dyadic=False)
        r = oracle.align([n], [m], S.ravel(), -0.2, 0.5)
        p = oracle.pair_path(r, 0)
        assert np.all(np.diff(p[:, 0]) > 0) and np.all(np.diff(p[:, 1]) > 0)
        k = int(r["n_diag"][0])
        assert k == len(p) <= min(n, m)


def test_scale_invariance_bitwise():
    # scaling S and g by 2^e is exact in FP32, so scores scale bitwise and the
    # path is identical
    rng = np.random.default_rng(8)
    for e in (-3, 1, 4):
        n, m = rng.integers(1, 50, 2)
        S = _rand_instance(rng, n, m, dyadic=False)
        s0, p0, _ = _align1(S, -0.2)
        s1, p1, _ = _align1(S * np.float32(2.0 ** e), np.float32(-0.2) * np.float32(2.0 ** e))
        assert np.float32(s1) == np.float32(s0) * np.float32(2.0 ** e)
        assert p0 == p1


def test_shift_invariance_dyadic():
    # every path has k DIAG and n+m-2k gap steps, so S+c with g+c/2 adds
    # (n+m)c/2 to every path
    rng = np.random.default_rng(9)
    for _ in range(20):
        n, m = rng.integers(1, 30, 2)
        S = _rand_instance(rng, n, m)
        c = float(rng.integers(1, 9)) / 16.0
        s0, p0, _ = _align1(S, -0.5)
        s1, p1, _ = _align1(S + np.float32(c), -0.5 + c / 2)
        assert s1 == s0 + (n + m) * c / 2
        assert p0 == p1


def test_transpose_invariance():
    rng = np.random.default_rng(10)
    for _ in range(20):
        n, m = rng.integers(1, 40, 2)
        S = _rand_instance(rng, n, m)
        s0, p0, _ = _align1(S, -0.25)
        s1, p1, _ = _align1(S.T.copy(), -0.25)
        assert s0 == s1
        exact, _, count = brute.best_alignment(S.tolist(), Fraction(-1, 4)) if n * m <= 16 else (None, None, None)
        if count == 1:
            assert [(j, i) for i, j in p1] == p0


def test_monotone_in_S_and_gap():
    rng = np.random.default_rng(12)
    for _ in range(30):
        n, m = rng.integers(1, 40, 2)
        S = _rand_instance(rng, n, m, dyadic=False)
        S2 = S + rng.random((n, m)).astype(np.float32) * (rng.random((n, m)) < 0.3)
        s0, _, _ = _align1(S, -0.3)
        s1, _, _ = _align1(S2.astype(np.float32), -0.3)
        s2, _, _ = _align1(S, -0.2)
        assert s1 >= s0 and s2 >= s0


def test_bounds():
    rng = np.random.default_rng(13)
    for _ in range(20):
        n, m = rng.integers(1, 40, 2)
        S = _rand_instance(rng, n, m)
        g = -0.125
        s, _, _ = _align1(S, g)
        lo = min(n, m) * float(S.min()) + abs(int(n) - int(m)) * g
        hi = min(n, m) * float(S.max()) + abs(int(n) - int(m)) * g
        assert lo <= s <= hi


# --- threshold (Sec. 4: pairs below the threshold are excluded) ---------------
def test_threshold_is_inclusive():
    S = np.array([[0.5, 0.0], [0.0, 0.49999997]], np.float32)
    r = oracle.align([2], [2], S.ravel(), -1.0, 0.5)
    assert oracle.pair_path(r, 0).tolist() == [[0, 0], [1, 1]]
    assert oracle.pair_kept(r, 0).tolist() == [[0, 0]]


# --- scorer ---------------------------------------------------------------------
def _dense(batch):
    V = batch.V
    D = np.zeros((V, V))
    for t in range(V):
        for e in range(batch.d_row_off[t], batch.d_row_off[t + 1]):
            D[t, batch.d_col[e]] += batch.d_val[e]
    return D


def test_scorer_matches_dense_contraction():
    b = corpus.make_batch(1, V=256).subset([0])
    # keep the dense check small: first 40 source and 50 target sentences
    b.n[:] = 40
    b.m[:] = 50
    b.src_off = b.src_off[:41]
    b.tgt_off = b.tgt_off[:51]
    out = oracle.score(b)
    X = np.zeros((40, b.V))
    for i in range(40):
        toks = b.src_tok[b.src_off[i]:b.src_off[i + 1]]
        np.add.at(X[i], toks, 1.0 / len(toks))
    Y = np.zeros((50, b.V))
    for j in range(50):
        Y[j, b.tgt_tok[b.tgt_off[j]:b.tgt_off[j + 1]]] = 1.0
    ref = (X @ _dense(b)) @ Y.T
    np.testing.assert_allclose(out["S_raw"].reshape(40, 50), ref, rtol=1e-12, atol=1e-14)
    assert out["S_raw"].min() >= 0.0 and out["S_raw"].max() <= 1.0 + 1e-6


def test_scorer_exact_translation_is_one():
    b = corpus.identity_batch(1, 25)
    out = oracle.score(b)
    S_raw = out["S_raw"].reshape(25, 25)
    np.testing.assert_array_equal(np.diag(S_raw), 1.0)
    # permutation dictionary: S_raw = fraction of source tokens (with
    # multiplicity) whose translation occurs in the target sentence
    for i, j in [(0, 3), (7, 2), (11, 19)]:
        s = b.src_tok[b.src_off[i]:b.src_off[i + 1]]
        t = set(b.tgt_tok[b.tgt_off[j]:b.tgt_off[j + 1]].tolist())
        frac = sum(1 for x in s if int(b.d_col[x]) in t) / len(s)
        assert S_raw[i, j] == pytest.approx(frac, abs=1e-15)


def test_scorer_sigmoid_special_cases():
    b = corpus.make_batch(1, V=512)
    out = oracle.score(b, scorer=[0.0, 0.0, 0.0])
    assert np.all(out["S64"] == 0.5)
    bb = 1.7
    out = oracle.score(b, scorer=[0.0, 0.0, bb])
    np.testing.assert_allclose(out["S64"], 1.0 / (1.0 + np.exp(-bb)), rtol=1e-15)
    out2 = oracle.score(b, scorer=[0.0, 0.0, -bb])
    np.testing.assert_allclose(out["S64"] + out2["S64"], 1.0, rtol=1e-15)
    # length feature: rho = min/max of sentence lengths
    out = oracle.score(b, scorer=[0.0, 1.0, 0.0])
    ls = np.diff(b.src_off)[:5]
    lt = np.diff(b.tgt_off)[:5]
    rho = out["rho"].reshape(200, 220)[:5, :5]
    np.testing.assert_allclose(rho, np.minimum.outer(ls, lt) / np.maximum.outer(ls, lt), rtol=1e-15)


def test_scorer_empty_sentences():
    b = corpus.make_batch(1, V=128).subset([0])
    b.n[:] = 2
    b.m[:] = 2
    b.src_off = np.array([0, 0, 3], np.int64)
    b.tgt_off = np.array([0, 0, 4], np.int64)
    out = oracle.score(b, scorer=[2.0, 1.0, 0.0])
    S_raw = out["S_raw"].reshape(2, 2)
    rho = out["rho"].reshape(2, 2)
    assert S_raw[0, 0] == 0 and S_raw[0, 1] == 0 and rho[0, 0] == 1.0 and rho[0, 1] == 0.0


# --- diagonal recovery on identical documents ----------------------------------
def test_identical_documents_align_on_the_diagonal():
    b = corpus.identity_batch(1, 40)
    out = oracle.score(b)
    S = out["S32"].reshape(40, 40)
    assert np.all(np.diag(S)[:, None] >= S)          # row dominance
    r = oracle.align(b.n, b.m, out["S32"], -0.2, 0.5)
    assert oracle.pair_path(r, 0).tolist() == [[i, i] for i in range(40)]
    assert oracle.pair_kept(r, 0).tolist() == [[i, i] for i in range(40)]
    assert oracle.f1([oracle.pair_kept(r, 0)], [b.gold]) == 100.0


# --- backward -------------------------------------------------------------------
def test_subgradient_inequality():
    rng = np.random.default_rng(21)
    for _ in range(20):
        n, m = rng.integers(1, 25, 2)
        S = _rand_instance(rng, n, m)
        g = -float(rng.integers(1, 33)) / 64.0
        s0, p0, r = _align1(S, g)
        k = len(p0)
        G = n + m - 2 * k
        for _ in range(5):
            S1 = _rand_instance(rng, n, m)
            g1 = -float(rng.integers(1, 33)) / 64.0
            s1, _, _ = _align1(S1, g1)
            lin = s0 + sum(float(S1[i, j]) - float(S[i, j]) for i, j in p0) + G * (g1 - g)
            assert s1 >= lin - 1e-9


def test_backward_matches_finite_differences():
    b = corpus.make_batch(4, pairs=6)
    w = np.array([3.0, 0.5, -1.0])
    sc = oracle.score(b, scorer=w)
    res = oracle.align(b.n, b.m, sc["S32"], b.gap, b.threshold)
    a = np.linspace(0.5, 1.5, b.B)
    bw = oracle.backward(b.n, b.m, res, a, sc["S64"], sc["S_raw"], sc["rho"])
    # dL/dg: centred difference of sum_b a_b * Score_b(g)
    h = 1e-3
    up = oracle.align(b.n, b.m, sc["S32"], b.gap + h, b.threshold)
    dn = oracle.align(b.n, b.m, sc["S32"], b.gap - h, b.threshold)
    if all(np.array_equal(oracle.pair_path(up, q), oracle.pair_path(res, q)) and
           np.array_equal(oracle.pair_path(dn, q), oracle.pair_path(res, q)) for q in range(b.B)):
        fd = float(np.dot(a, up["score"].astype(np.float64) - dn["score"].astype(np.float64))) / (2 * h)
        assert fd == pytest.approx(bw["grad_gap"], rel=2e-3)
    # dL/d(w0, w1, b) on the fixed path, in FP64: sum_b a_b sum_path S(w)
    def path_sum(wv):
        s = oracle.score(b, scorer=wv)["S64"]
        tot = 0.0
        for q in range(b.B):
            o = sc["s_off"][q]
            for i, j in oracle.pair_path(res, q):
                tot += a[q] * s[o + i * b.m[q] + j]
        return tot
    for c in range(3):
        e = np.zeros(3); e[c] = 1e-5
        fd = (path_sum(w + e) - path_sum(w - e)) / 2e-5
        assert fd == pytest.approx(bw["grad_wb"][c], rel=1e-6, abs=1e-9)
    # grad_S is the path indicator times a_b
    gS = bw["grad_S"]
    for q in range(b.B):
        o = sc["s_off"][q]
        blk = gS[o:o + b.n[q] * b.m[q]].reshape(b.n[q], b.m[q])
        ind = np.zeros_like(blk)
        for i, j in oracle.pair_path(res, q):
            ind[i, j] = a[q]
        np.testing.assert_array_equal(blk, ind)


@pytest.mark.parametrize("a_scale", [0.0, 1.0])
def test_backward_dense_extra_term_matches_finite_differences(a_scale):
    """Sec. 5.2 tuning gradient with an extra dense upstream E = dL/dS:
    L(w) = sum_b a_b * PathSum_b(S(w)) + sum_ij E_ij * S_ij(w) on the fixed
    traced path.  Centred differences of L in w0, w1 and b (FP64 scores, the
    path held fixed) pin the chain dL/dz = (a P + E) S (1 - S) and its sums
    against S_raw, rho and 1; grad_S must be E + a P cell for cell.  With
    a = 0 the dense term is checked on its own."""
    b = corpus.make_batch(4, pairs=5)
    w = np.array([2.5, -0.75, -0.5])
    sc = oracle.score(b, scorer=w)
    res = oracle.align(b.n, b.m, sc["S32"], b.gap, b.threshold)
    a = a_scale * np.linspace(0.5, 1.5, b.B)
    E = np.random.default_rng(23).normal(size=sc["S64"].shape[0])
    bw = oracle.backward(b.n, b.m, res, a, sc["S64"], sc["S_raw"], sc["rho"], grad_S_extra=E)

    def loss(wv):
        s = oracle.score(b, scorer=wv)["S64"]
        tot = float(np.dot(E, s))
        for q in range(b.B):
            o = sc["s_off"][q]
            for i, j in oracle.pair_path(res, q):
                tot += a[q] * s[o + i * b.m[q] + j]
        return tot
    for c in range(3):
        e = np.zeros(3)
        e[c] = 1e-5
        fd = (loss(w + e) - loss(w - e)) / 2e-5
        assert fd == pytest.approx(bw["grad_wb"][c], rel=1e-6, abs=1e-8)
    # dL/dS = E + a P, element for element (P = the traced path's DIAG cells)
    expect = E.copy()
    for q in range(b.B):
        o = sc["s_off"][q]
        for i, j in oracle.pair_path(res, q):
            expect[o + i * b.m[q] + j] += a[q]
    np.testing.assert_array_equal(bw["grad_S"], expect)
    # the gap gradient does not see E
    G = (b.n + b.m - 2 * res["n_diag"]).astype(np.float64)
    assert bw["grad_gap"] == pytest.approx(float(np.dot(a, G)), rel=1e-12, abs=0)


def test_backward_fd_in_S_on_unique_paths():
    rng = np.random.default_rng(22)
    n, m = 12, 15
    S = rng.random((n, m)).astype(np.float32)
    s0, p0, r = _align1(S, -0.2)
    h = np.float32(1.0 / 64)
    for (i, j) in [(0, 0), (3, 4), (p0[0][0], p0[0][1]), (p0[-1][0], p0[-1][1])]:
        Sp = S.copy(); Sp[i, j] += h
        Sm = S.copy(); Sm[i, j] -= h
        sp, pp, _ = _align1(Sp, -0.2)
        sm, pm, _ = _align1(Sm, -0.2)
        if pp == p0 and pm == p0:
            fd = (sp - sm) / (2 * float(h))
            expect = 1.0 if (i, j) in p0 else 0.0
            assert abs(fd - expect) < 1e-4


# --- F1 ---------------------------------------------------------------------------
def test_f1():
    assert oracle.f1([[]], [[]]) == 100.0
    assert oracle.f1([[(0, 0)]], [[(1, 1)]]) == 0.0
    assert oracle.f1([[(0, 0), (1, 1)]], [[(0, 0), (2, 2)]]) == pytest.approx(50.0)
    assert oracle.f1([[(0, 0)], [(1, 1), (2, 2)]], [[(0, 0)], [(1, 1)]]) == pytest.approx(200 * (2 / 3) / (2 / 3 + 1))


# --- generator --------------------------------------------------------------------
def test_generator_is_deterministic_and_sliceable():
    a = corpus.make_batch(2, pairs=12)
    b = corpus.make_batch(2, pairs=12)
    for f in ("n", "m", "src_off", "src_tok", "tgt_off", "tgt_tok", "gold", "d_col", "d_val"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    c = corpus.make_batch(2, pairs=4, first=8)
    s = a.subset([8, 9, 10, 11])
    for f in ("n", "m", "src_off", "src_tok", "tgt_off", "tgt_tok", "gold"):
        np.testing.assert_array_equal(getattr(c, f), getattr(s, f))


def test_generator_planted_alignment():
    b = corpus.make_batch(1)
    assert b.n[0] == 200 and b.m[0] == 220
    dele, ins = corpus.indel_counts(200, 220)
    assert (dele, ins) == (20, 40)
    g = b.gold
    assert len(g) == 180
    assert np.all(np.diff(g[:, 0]) > 0) and np.all(np.diff(g[:, 1]) > 0)
    # translated sentences keep their source length
    ls = np.diff(b.src_off)[g[:, 0]]
    lt = np.diff(b.tgt_off)[g[:, 1]]
    np.testing.assert_array_equal(ls, lt)
    # the dictionary is row-stochastic with distinct targets
    V = b.V
    cols = b.d_col.reshape(V, 4)
    assert np.all(np.sort(cols, 1)[:, 1:] != np.sort(cols, 1)[:, :-1])
    np.testing.assert_allclose(b.d_val.reshape(V, 4).sum(1), 1.0, rtol=1e-6)


# --- bi-directional mining: union of kept sets (Sec. 5.4, Table 3 "BI") -------------
def _monotone(rng, n, k):
    """k pairs strictly increasing in i and in j, coordinates < n."""
    k = min(k, n)
    return np.stack([np.sort(rng.choice(n, k, replace=False)), np.sort(rng.choice(n, k, replace=False))], 1)


def test_union_kept_hand_example():
    fwd = [np.array([[0, 0], [2, 1], [4, 4]])]
    rev = [np.array([[0, 0], [2, 3], [5, 6]])]     # (j, i): (0,0) (3,2) (6,5)
    u = oracle.union_kept(fwd, rev)[0]
    np.testing.assert_array_equal(u, [[0, 0], [2, 1], [3, 2], [4, 4], [6, 5]])


def test_union_kept_inclusion_exclusion_and_order():
    rng = np.random.default_rng(5)
    for t in range(200):
        n = int(rng.integers(1, 300))
        F = _monotone(rng, n, int(rng.integers(0, n + 1)))
        Rf = _monotone(rng, n, int(rng.integers(0, n + 1)))
        if t % 3 == 0 and len(F):          # force shared pairs
            Rf = F[np.sort(rng.choice(len(F), int(rng.integers(0, len(F) + 1)), replace=False))]
        u = oracle.union_kept([F], [Rf[:, ::-1]])[0]
        kf = F[:, 0].astype(np.int64) * 4096 + F[:, 1]
        kr = Rf[:, 0].astype(np.int64) * 4096 + Rf[:, 1]
        ku = u[:, 0].astype(np.int64) * 4096 + u[:, 1]
        assert len(u) == len(F) + len(Rf) - len(np.intersect1d(kf, kr))
        assert np.all(np.diff(ku) > 0)                   # ascending, each once
        assert np.all(np.isin(kf, ku)) and np.all(np.isin(kr, ku))


def test_reverse_dictionary_is_the_transposed_table():
    b = corpus.make_batch(2, pairs=2)
    ro, col, val = corpus.reverse_dictionary(b)
    fwd = {}
    for t in range(b.V):
        for k in range(b.d_row_off[t], b.d_row_off[t + 1]):
            fwd[(t, int(b.d_col[k]))] = float(b.d_val[k])
    for u in range(0, b.V, 7):
        row = range(ro[u], ro[u + 1])
        assert len(row) <= corpus.DICT_DEG
        if len(row) == 0:
            assert not any(uu == u for (_, uu) in fwd)
            continue
        ws = [fwd[(int(col[k]), u)] for k in row]          # every entry is a forward entry t -> u
        assert ws == sorted(ws, reverse=True)
        assert abs(float(np.sum(val[ro[u]:ro[u + 1]], dtype=np.float64)) - 1.0) < 1e-6
        np.testing.assert_allclose(val[ro[u]:ro[u + 1]], np.array(ws) / np.sum(ws), rtol=1e-6)


# --- tuning script similarity (Sec. 5.2) ----------------------------------------------
def test_similarity_hand_example_and_special_cases():
    A = [np.array([[0, 0], [1, 1], [2, 3]])]
    G = [np.array([[0, 0], [2, 3]])]
    assert oracle.similarity(A, G) == pytest.approx(80.0)      # 2 * 2 / (3 + 2)
    e = np.zeros((0, 2), np.int32)
    assert oracle.similarity([e], [e]) == 100.0
    assert oracle.similarity([A[0]], [e]) == 0.0
    assert oracle.similarity(A, A) == 100.0


def test_similarity_nw_equals_shared_pairs_for_monotone_sequences():
    # two strictly increasing sequences: the NW optimum (match 1, else 0) is
    # the number of common elements
    rng = np.random.default_rng(6)
    for _ in range(100):
        n = int(rng.integers(1, 80))
        A = _monotone(rng, n, int(rng.integers(0, n + 1)))
        G = _monotone(rng, n, int(rng.integers(0, n + 1)))
        if len(A) and rng.random() < 0.5:
            G = A[np.sort(rng.choice(len(A), int(rng.integers(0, len(A) + 1)), replace=False))]
        common = len(set(map(tuple, A.tolist())) & set(map(tuple, G.tolist())))
        assert oracle._nw_match_count(A, G) == common
    # not monotone: the NW optimum is an LCS, below the set intersection
    A = np.array([[0, 0], [1, 1]])
    G = np.array([[1, 1], [0, 0]])
    assert oracle._nw_match_count(A, G) == 1
