"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars:
  * DP: bit-exact given identical S (score bits, aligned pairs, kept pairs);
  * S in FP32: |S - S64| <= 1e-5 * max(|S64|, FLT_MIN) against the FP64 oracle;
  * S with BF16 operands: |S - S64| <= 2e-2;
  * backward: grad_S equals the oracle's path indicator bit for bit, the gap
    gradient matches, the weight gradient within FP32-partial rounding.
"""
import numpy as np
import pytest

import oracle
from synth import corpus
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _fig(rows, cols):
    return np.array([[1.0 if a == b else 0.0 for b in cols] for a in rows], np.float32)


# --- DP on identical S ------------------------------------------------------------
@pytest.mark.parametrize("g", [-0.2, -0.125, -0.3])
def test_dp_paper_figures(g):
    for rows, cols in [("tablets make people spoil children".split(), "tablets make children very addicted".split()),
                       ("a d c d e".split(), "a d e g f".split())]:
        S = _fig(rows, cols)
        gpu = H.gpu_align_only([5], [5], S.ravel(), g, -1e30)
        ora = oracle.align([5], [5], S.ravel(), g, -1e30)
        H.assert_align_equal(gpu, ora, [5], [5], check_path_as_kept=True)


def test_dp_brute_force_sizes():
    rng = np.random.default_rng(1)
    ns, ms, blocks = [], [], []
    for n in range(0, 7):
        for m in range(0, 7):
            for _ in range(2):
                ns.append(n); ms.append(m)
                blocks.append((rng.integers(0, 65, (n, m)) / 64.0).astype(np.float32).ravel())
    S = np.concatenate(blocks).astype(np.float32)
    for g in (-0.25, -0.078125):
        gpu = H.gpu_align_only(ns, ms, S, g, -1e30)
        ora = oracle.align(ns, ms, S, g, -1e30)
        H.assert_align_equal(gpu, ora, ns, ms, check_path_as_kept=True)


def test_dp_ragged_strips_and_ties():
    # sizes around the 64-row strip, the 32-column staging block and the
    # 64-step traceback word group; coarse values create many exact ties
    rng = np.random.default_rng(2)
    sizes = [(1, 1), (1, 300), (300, 1), (63, 64), (64, 63), (64, 64), (65, 65), (127, 33), (129, 31),
             (200, 220), (191, 257), (2, 500), (500, 2), (130, 96)]
    ns = [a for a, _ in sizes]
    ms = [b for _, b in sizes]
    for kind in ("coarse", "fine"):
        if kind == "coarse":
            blocks = [(rng.integers(0, 3, n * m) / 2.0).astype(np.float32) for n, m in sizes]
        else:
            blocks = [rng.random(n * m).astype(np.float32) for n, m in sizes]
        S = np.concatenate(blocks)
        for g, thr in ((-0.25, 0.5), (-0.2, -1e30)):
            gpu = H.gpu_align_only(ns, ms, S, g, thr)
            ora = oracle.align(ns, ms, S, g, thr)
            H.assert_align_equal(gpu, ora, ns, ms, check_path_as_kept=thr < -1e29)


@pytest.mark.parametrize("g", [0.0, -0.0, 0.25])
def test_dp_zero_and_positive_gaps_signed_zero_similarities(g):
    # a gap of -0 makes H[i][0] = -0 (the fill keeps its compare chain there);
    # S holds -0 entries and coarse values with many exact ties
    rng = np.random.default_rng(5)
    sizes = [(3, 4), (64, 65), (130, 70), (7, 1), (1, 9), (70, 130)]
    ns = [a for a, _ in sizes]
    ms = [b for _, b in sizes]
    blocks = []
    for n, m in sizes:
        blk = (rng.integers(0, 3, n * m) / 2.0).astype(np.float32)
        blk[(blk == 0.0) & (rng.random(n * m) < 0.5)] = np.float32(-0.0)
        blocks.append(blk)
    S = np.concatenate(blocks)
    gpu = H.gpu_align_only(ns, ms, S, g, 0.5)
    ora = oracle.align(ns, ms, S, g, 0.5)
    H.assert_align_equal(gpu, ora, ns, ms)


def test_dp_empty_sides():
    ns = [0, 5, 0, 3, 7]
    ms = [4, 0, 0, 3, 1]
    rng = np.random.default_rng(3)
    S = rng.random(int(np.dot(ns, ms))).astype(np.float32)
    gpu = H.gpu_align_only(ns, ms, S, -0.2, 0.5)
    ora = oracle.align(ns, ms, S, -0.2, 0.5)
    H.assert_align_equal(gpu, ora, ns, ms)


@pytest.mark.parametrize("g", [-0.2, -0.0])
@pytest.mark.parametrize("staging", [1, 2])
def test_dp_register_staging_bitexact(g, staging):
    # the fill's other S stagings (1: registers, 2: the LDS ring one strip
    # per workgroup, every hand-off through memory): brute-force sizes,
    # ragged strips with exact ties, empty sides and tall pairs (hand-offs),
    # bit-exact
    rng = np.random.default_rng(7)
    sizes = [(0, 4), (5, 0), (1, 1), (3, 6), (6, 3), (1, 300), (300, 1), (63, 64), (64, 63), (65, 65), (127, 33),
             (129, 31), (200, 220), (2, 500), (500, 2), (700, 650), (1300, 90)]
    ns = [a for a, _ in sizes]
    ms = [b for _, b in sizes]
    for kind in ("coarse", "fine"):
        if kind == "coarse":
            blocks = [(rng.integers(0, 3, n * m) / 2.0).astype(np.float32) for n, m in sizes]
        else:
            blocks = [rng.random(n * m).astype(np.float32) for n, m in sizes]
        S = np.concatenate(blocks)
        gpu = H.gpu_align_only(ns, ms, S, g, 0.5, params={"fill_staging": staging})
        ora = oracle.align(ns, ms, S, g, 0.5)
        H.assert_align_equal(gpu, ora, ns, ms)


def test_dp_large_pair_bitexact():
    rng = np.random.default_rng(4)
    ns, ms = [1500, 700], [1300, 2100]
    S = np.concatenate([rng.random(n * m).astype(np.float32) for n, m in zip(ns, ms)])
    gpu = H.gpu_align_only(ns, ms, S, -0.2, 0.5)
    ora = oracle.align(ns, ms, S, -0.2, 0.5)
    H.assert_align_equal(gpu, ora, ns, ms)


# --- scores ---------------------------------------------------------------------------
def _check_scores(batch, prec, tol_rel=None, tol_abs=None, scorer=None, params=None):
    gpu = H.run_gpu(batch, prec=prec, scorer=scorer, params=params)
    ora = oracle.score(batch, scorer=scorer)
    if tol_rel is not None:
        err = H.s_rel_err(gpu["S"], ora["S64"])
        assert err.max() <= tol_rel, err.max()
    if tol_abs is not None:
        err = np.abs(gpu["S"].astype(np.float64) - ora["S64"])
        assert err.max() <= tol_abs, err.max()
    return gpu, ora


def test_scores_fp32_config1():
    b = corpus.make_batch(1)
    gpu, ora = _check_scores(b, 0, tol_rel=1e-5)
    np.testing.assert_allclose(gpu["S_raw"], ora["S_raw"], rtol=1e-5, atol=1e-7)


def test_scores_bf16_config1():
    b = corpus.make_batch(1)
    _check_scores(b, 1, tol_abs=2e-2)


def test_scores_oriented_scorer_fp32_bf16():
    # large |w0| amplifies the contraction error: the hardest case for both
    b = corpus.make_batch(1)
    w = np.array([12.0, -1.5, -2.0], np.float32)
    _check_scores(b, 0, tol_rel=1e-5, scorer=w)
    _check_scores(b, 1, tol_abs=2e-2, scorer=w)


@pytest.mark.parametrize("prec", [0, 1])
def test_scores_ragged_batch_with_empty_pairs(prec):
    # several tiles and ragged tails on both sides, with pairs that have an
    # empty source side, an empty target side, or both, mixed in
    n, m = corpus.make_sizes(2, 40)
    n, m = n.copy(), m.copy()
    n[3], m[7], n[11], m[11], n[39] = 0, 0, 0, 0, 0
    m[20] = 1
    n[21] = 1
    b = corpus.make_batch(2, pairs=40, sizes=(n, m))
    assert b.cells() > 0 and np.count_nonzero(b.n.astype(np.int64) * b.m == 0) == 4
    if prec == 0:
        gpu, ora = _check_scores(b, 0, tol_rel=1e-5)
    else:
        gpu, ora = _check_scores(b, 1, tol_abs=2e-2)
    # the DP on the GPU's S, bit-exact; empty sides score fl32((n + m) g)
    al = oracle.align(b.n, b.m, gpu["S"], b.gap, b.threshold)
    np.testing.assert_array_equal(gpu["score"].view(np.uint32), al["score"].view(np.uint32))
    np.testing.assert_array_equal(gpu["n_diag"], al["n_diag"])
    np.testing.assert_array_equal(gpu["n_kept"], al["n_kept"])
    for q in (3, 7, 11, 39):
        assert gpu["n_kept"][q] == 0 and gpu["n_diag"][q] == 0
        assert gpu["score"][q] == np.float32(b.n[q] + b.m[q]) * np.float32(b.gap)


def _wide_vocabulary_batch():
    """Two pairs of 70 x 70 sentences over V = 4096 with uniformly drawn words:
    a 64-sentence target tile holds about 2500 distinct words (more than 64
    compacted chunks: the chunk-range window slides) and 150-token source
    sentences put more A entries into one compacted chunk than the registers
    hold (the overflow loop runs)."""
    import dataclasses
    b = corpus.make_batch(2, pairs=2, sizes=([70, 70], [70, 70]), V=4096)
    rng = np.random.default_rng(11)
    s_len = rng.integers(100, 151, size=140)
    t_len = rng.integers(40, 61, size=140)
    s_len[5] = 0    # an empty source sentence
    t_len[77] = 0   # an empty target sentence
    return dataclasses.replace(
        b, src_off=np.concatenate([[0], np.cumsum(s_len)]).astype(np.int64),
        src_tok=rng.integers(0, 4096, size=int(s_len.sum())).astype(np.int32),
        tgt_off=np.concatenate([[0], np.cumsum(t_len)]).astype(np.int64),
        tgt_tok=rng.integers(0, 4096, size=int(t_len.sum())).astype(np.int32))


def _varying_degree_batch():
    """Six pairs over a dictionary whose rows hold 0 to 11 entries (rows
    longer than four take the merge's extra passes), with source sentences of
    0 to 90 tokens (past the first 48 the merge goes one token per lane) and
    repeated tokens inside a sentence."""
    import dataclasses
    b = corpus.make_batch(2, pairs=6, sizes=([5, 70, 64, 1, 130, 33], [9, 66, 64, 40, 20, 1]))
    rng = np.random.default_rng(12)
    V = b.V
    deg = rng.integers(0, 12, size=V)
    deg[:8] = [0, 11, 5, 4, 3, 8, 1, 0]
    cols = [np.sort(rng.choice(V, int(k), replace=False)) for k in deg]
    d_row_off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    d_col = np.concatenate(cols).astype(np.int32)
    d_val = rng.random(int(deg.sum())).astype(np.float32)
    n_src = int(b.n.sum())
    s_len = rng.integers(0, 91, size=n_src)
    s_len[:6] = [0, 1, 47, 48, 49, 90]
    src_tok = rng.integers(0, 64, size=int(s_len.sum())).astype(np.int32)   # few words: repeats
    src_tok[: int(s_len[:8].sum())] = rng.integers(0, 8, size=int(s_len[:8].sum()))   # the chosen rows
    return dataclasses.replace(b, src_off=np.concatenate([[0], np.cumsum(s_len)]).astype(np.int64),
                               src_tok=src_tok, d_row_off=d_row_off, d_col=d_col, d_val=d_val,
                               d_deg=int(deg.max()))


def test_scores_varying_dictionary_degree_and_long_sentences():
    w = _varying_degree_batch()
    for compact in (1, 0):
        p = {"score_compact": compact}
        gpu, ora = _check_scores(w, 0, tol_rel=1e-5, params=p)
        np.testing.assert_allclose(gpu["S_raw"], ora["S_raw"], rtol=1e-5, atol=1e-7)
        _check_scores(w, 1, tol_abs=2e-2, params=p)


@pytest.mark.parametrize("compact", [1, 0])
def test_scores_compacted_and_dense_contraction(compact):
    # both contraction modes against the oracle: the ragged 40-pair batch and
    # the wide-vocabulary batch (window slide, register overflow)
    p = {"score_compact": compact}
    b = corpus.make_batch(2, pairs=40)
    gpu, ora = _check_scores(b, 0, tol_rel=1e-5, params=p)
    np.testing.assert_allclose(gpu["S_raw"], ora["S_raw"], rtol=1e-5, atol=1e-7)
    _check_scores(b, 1, tol_abs=2e-2, params=p)
    w = _wide_vocabulary_batch()
    gpu, ora = _check_scores(w, 0, tol_rel=1e-5, params=p)
    np.testing.assert_allclose(gpu["S_raw"], ora["S_raw"], rtol=1e-5, atol=1e-7)
    _check_scores(w, 1, tol_abs=2e-2, params=p)


def _fused_edge_batch():
    """Five pairs whose row tiles are full, partial and of one row, over a
    dictionary with rows of 0 to 4 entries, with source sentences of 0 to 48
    tokens (the bound of the fused expansion, reached exactly) and repeated
    tokens inside a sentence (merged entries)."""
    import dataclasses
    b = corpus.make_batch(2, pairs=5, sizes=([1, 63, 64, 65, 130], [7, 70, 64, 1, 129]))
    rng = np.random.default_rng(13)
    V = b.V
    deg = rng.integers(0, 5, size=V)
    deg[:8] = [0, 4, 3, 2, 1, 0, 4, 4]
    cols = [np.sort(rng.choice(V, int(k), replace=False)) for k in deg]
    d_row_off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int32)
    d_col = np.concatenate(cols).astype(np.int32)
    d_val = rng.random(int(deg.sum())).astype(np.float32)
    n_src = int(b.n.sum())
    s_len = rng.integers(0, 49, size=n_src)
    s_len[:6] = [0, 1, 16, 47, 48, 48]
    src_tok = rng.integers(0, 64, size=int(s_len.sum())).astype(np.int32)   # few words: repeats
    src_tok[: int(s_len[:8].sum())] = rng.integers(0, 8, size=int(s_len[:8].sum()))
    return dataclasses.replace(b, src_off=np.concatenate([[0], np.cumsum(s_len)]).astype(np.int64),
                               src_tok=src_tok, d_row_off=d_row_off, d_col=d_col, d_val=d_val, d_deg=4)


@pytest.mark.parametrize("compact", [1, 0])
def test_fused_expansion_matches_two_kernel_path(compact):
    # the fused source-side expansion (merge and row-tile lists in one kernel)
    # against merge + list build: S and S_raw bit for bit (its lists keep
    # entries the two-kernel path drops, which no tile's contraction reads),
    # and the oracle bars; a batch past its bounds takes the two kernels
    for b in (_fused_edge_batch(), corpus.make_batch(2, pairs=40)):
        for prec in (0, 1):
            p = {"score_compact": compact}
            two = H.run_gpu(b, prec=prec, params=dict(p, expand_fused=0), timing=True)
            one = H.run_gpu(b, prec=prec, params=dict(p, expand_fused=1), timing=True)
            assert one["launches"]["expand_a"] > 0 and one["launches"]["merge"] == 0
            assert two["launches"]["expand_a"] == 0 and two["launches"]["merge"] > 0
            np.testing.assert_array_equal(one["S"].view(np.uint32), two["S"].view(np.uint32))
            np.testing.assert_array_equal(one["S_raw"].view(np.uint32), two["S_raw"].view(np.uint32))
            ora = oracle.score(b)
            if prec == 0:
                assert H.s_rel_err(one["S"], ora["S64"]).max() <= 1e-5
            else:
                assert np.abs(one["S"].astype(np.float64) - ora["S64"]).max() <= 2e-2
    wide = H.run_gpu(_varying_degree_batch(), params={"score_compact": compact, "expand_fused": 1}, timing=True)
    assert wide["launches"]["expand_a"] == 0 and wide["launches"]["merge"] > 0


def test_contraction_k_width_two_chunks_per_round():
    # the compacted contraction with two 32-word chunks per round: the same
    # bits as one chunk per round (same summation order) and the oracle bars,
    # on the ragged batch (odd chunk counts) and the wide-vocabulary batch
    # (more than 64 compacted chunks: window slide, register overflow)
    for b in (corpus.make_batch(2, pairs=40), _wide_vocabulary_batch()):
        for prec in (0, 1):
            one = H.run_gpu(b, prec=prec, params={"score_kgroup": 1})
            two, ora = _check_scores(b, prec, tol_rel=1e-5 if prec == 0 else None,
                                     tol_abs=2e-2 if prec == 1 else None, params={"score_kgroup": 2})
            np.testing.assert_array_equal(two["S"].view(np.uint32), one["S"].view(np.uint32))
            np.testing.assert_array_equal(two["S_raw"].view(np.uint32), one["S_raw"].view(np.uint32))
            H.assert_align_equal(two, oracle.align(b.n, b.m, two["S"], b.gap, b.threshold), b.n, b.m)


def test_end_to_end_dp_bitexact_on_gpu_scores():
    b = corpus.make_batch(2, pairs=64)
    for prec in (0, 1):
        gpu = H.run_gpu(b, prec=prec)
        ora = oracle.align(b.n, b.m, gpu["S"], b.gap, b.threshold)
        H.assert_align_equal(gpu, ora, b.n, b.m)


def test_determinism():
    b = corpus.make_batch(2, pairs=24)
    a1 = H.run_gpu(b, prec=1)
    a2 = H.run_gpu(b, prec=1)
    np.testing.assert_array_equal(a1["S"].view(np.uint32), a2["S"].view(np.uint32))
    np.testing.assert_array_equal(a1["score"].view(np.uint32), a2["score"].view(np.uint32))
    np.testing.assert_array_equal(a1["n_kept"], a2["n_kept"])
    for q in range(b.B):
        o, k = int(a1["p_off"][q]), int(a1["n_kept"][q])
        np.testing.assert_array_equal(a1["kept"][o:o + k], a2["kept"][o:o + k])


def test_identical_documents_recover_the_diagonal():
    b = corpus.identity_batch(1, 90)
    gpu = H.run_gpu(b, prec=0)
    k = int(gpu["n_kept"][0])
    np.testing.assert_array_equal(gpu["kept"][:k], np.stack([np.arange(90)] * 2, 1))


# --- backward ----------------------------------------------------------------------------
def test_backward_matches_oracle():
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(4, pairs=16)
    w = np.array([3.0, 0.5, -1.0], np.float32)
    gpu = H.run_gpu(b, prec=0, scorer=w)
    mn = gpu["miner"]
    dev = mn.ctx.device
    a = np.linspace(0.5, 1.5, b.B).astype(np.float32)
    gS = torch.empty(mn.plan.S_elems, dtype=torch.float32, device=dev)
    gg = torch.zeros(1, dtype=torch.float64, device=dev)
    gwb = torch.zeros(3, dtype=torch.float64, device=dev)
    nw.align_backward(mn.plan, mn.batch, mn.tb, mn.n_diag, torch.as_tensor(a).to(dev), grad_S=gS, grad_gap=gg,
                      S=mn.S, S_raw=mn.S_raw, scorer=w, grad_wb=gwb, ws=mn.ws)
    torch.cuda.synchronize()
    # oracle on the GPU's S (identical DP input), FP64 chain on the oracle's S
    res = oracle.align(b.n, b.m, gpu["S"], b.gap, b.threshold)
    sc = oracle.score(b, scorer=w)
    bw = oracle.backward(b.n, b.m, res, a.astype(np.float64), sc["S64"], sc["S_raw"], sc["rho"])
    np.testing.assert_array_equal(gS.cpu().numpy(), bw["grad_S"].astype(np.float32))
    assert gg.item() == pytest.approx(bw["grad_gap"], rel=1e-6)
    np.testing.assert_allclose(gwb.cpu().numpy(), bw["grad_wb"], rtol=1e-4, atol=1e-5)
