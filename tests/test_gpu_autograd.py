"""The differentiable API on the GPU: NWAlign, LogisticScore and MineScore
called through torch.autograd, against the CPU oracle's backward (Sec. 5.2
tuning gradient: path indicator for dScore/dS, gap count for dScore/dgap,
chained through the logistic scorer of Sec. 4) and against centred finite
differences of the GPU's own forward on unique-path instances.

Bars: dL/dS equal to the oracle's a_b * P bit for bit (the DP is bit-exact,
and a_b has few mantissa bits); dL/dgap equal to the FP64 sum of a_b * G_b;
dL/dw within 1e-4 relative of the oracle backward fed the GPU's own S and
S_raw (FP32 per cell, FP64 batch reduction).
"""
import numpy as np
import pytest

import oracle
from synth import corpus
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _miner(b, prec=0):
    import paper_1512_01641_amd as nw
    ctx = nw.Context(0)
    return nw.Miner(ctx, nw.DeviceBatch.from_host(b), nw.DeviceDict.from_host(b), prec)


def _upstream(B):
    # few mantissa bits: a_b * (path indicator) and a_b * G_b are exact in FP32
    return (0.5 + (np.arange(B) % 8) / 8.0).astype(np.float32)


def test_nwalign_autograd_matches_oracle_path_indicator():
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(4, pairs=24)
    sc = oracle.score(b)
    mn = _miner(b)
    dev = mn.ctx.device
    S = torch.as_tensor(sc["S32"]).to(dev).requires_grad_(True)
    gap = torch.tensor(b.gap, dtype=torch.float32, device=dev, requires_grad=True)
    a = torch.as_tensor(_upstream(b.B)).to(dev)
    score = nw.NWAlign.apply(S, gap, mn, b.threshold)
    # another alignment on the same miner before the backward: the saved
    # traceback keeps the gradient of the first one
    mn.align(-0.9, b.threshold)
    (a * score).sum().backward()
    torch.cuda.synchronize()
    al = oracle.align(b.n, b.m, sc["S32"], b.gap, b.threshold)
    np.testing.assert_array_equal(score.detach().cpu().numpy().view(np.uint32), al["score"].view(np.uint32))
    bw = oracle.backward(b.n, b.m, al, a.cpu().numpy().astype(np.float64), sc["S64"], sc["S_raw"], sc["rho"])
    np.testing.assert_array_equal(S.grad.cpu().numpy(), bw["grad_S"].astype(np.float32))
    assert gap.grad.item() == pytest.approx(bw["grad_gap"], rel=1e-12)
    # a plain-number gap: no gap gradient, no error
    S2 = torch.as_tensor(sc["S32"]).to(dev).requires_grad_(True)
    nw.NWAlign.apply(S2, float(b.gap), mn, b.threshold).sum().backward()
    torch.cuda.synchronize()
    assert S2.grad is not None


def test_logistic_score_autograd_without_alignment():
    """LogisticScore on a fresh miner (no alignment ever ran): the backward
    reads no traceback; dL/dw of L = <E, S(w)> against the oracle."""
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(2, pairs=20)
    mn = _miner(b)
    dev = mn.ctx.device
    w = torch.tensor([3.0, -0.5, -1.0], dtype=torch.float32, device=dev, requires_grad=True)
    S = nw.LogisticScore.apply(w, mn)
    E = np.random.default_rng(31).normal(size=S.numel()).astype(np.float32)
    (torch.as_tensor(E).to(dev) * S).sum().backward()
    torch.cuda.synchronize()
    sc = oracle.score(b, scorer=w.detach().cpu().numpy())
    err = H.s_rel_err(S.detach().cpu().numpy(), sc["S64"])
    assert err.max() <= 1e-5
    # the oracle's chain on the GPU's own S and S_raw (FP64 arithmetic)
    empty = dict(path_off=np.zeros(b.B + 1, np.int64), path=np.zeros((1, 2), np.int32),
                 n_diag=np.zeros(b.B, np.int32))
    Sg = S.detach().cpu().numpy().astype(np.float64)
    Sr = mn.S_raw[:mn.plan.S_elems].cpu().numpy().astype(np.float64)
    bw = oracle.backward(b.n, b.m, empty, np.zeros(b.B), Sg, Sr, sc["rho"], grad_S_extra=E.astype(np.float64),
                         want_grad_S=False)
    np.testing.assert_allclose(w.grad.cpu().numpy(), bw["grad_wb"], rtol=1e-4, atol=1e-6)
    # and on the oracle's FP64 scores (the FP32 similarity's own error)
    bw64 = oracle.backward(b.n, b.m, empty, np.zeros(b.B), sc["S64"], sc["S_raw"], sc["rho"],
                           grad_S_extra=E.astype(np.float64), want_grad_S=False)
    np.testing.assert_allclose(w.grad.cpu().numpy(), bw64["grad_wb"], rtol=1e-3, atol=1e-5)


@pytest.mark.parametrize("prec", [0, 1])
def test_minescore_autograd_matches_oracle(prec):
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(4, pairs=32)
    wv = H.load_oriented(4)
    mn = _miner(b, prec)
    dev = mn.ctx.device
    w = torch.as_tensor(wv).to(dev).requires_grad_(True)
    gap = torch.tensor(b.gap, dtype=torch.float32, device=dev, requires_grad=True)
    a = torch.as_tensor(_upstream(b.B)).to(dev)
    score = nw.MineScore.apply(w, gap, mn, b.threshold)
    (a * score).sum().backward()
    torch.cuda.synchronize()
    P = mn.plan.S_elems
    Sg = mn.S[:P].cpu().numpy()
    Sr = mn.S_raw[:P].cpu().numpy().astype(np.float64)
    al = oracle.align(b.n, b.m, Sg, b.gap, b.threshold)   # the DP on the GPU's S
    np.testing.assert_array_equal(score.detach().cpu().numpy().view(np.uint32), al["score"].view(np.uint32))
    sc = oracle.score(b, scorer=wv)
    an = a.cpu().numpy().astype(np.float64)
    bw = oracle.backward(b.n, b.m, al, an, Sg.astype(np.float64), Sr, sc["rho"], want_grad_S=False)
    np.testing.assert_allclose(w.grad.cpu().numpy(), bw["grad_wb"], rtol=1e-4, atol=1e-6)
    assert gap.grad.item() == pytest.approx(bw["grad_gap"], rel=1e-12)
    # a plain-number gap works and gives only the weight gradient
    w2 = torch.as_tensor(wv).to(dev).requires_grad_(True)
    nw.MineScore.apply(w2, float(b.gap), mn, b.threshold).sum().backward()
    torch.cuda.synchronize()
    assert w2.grad is not None and torch.isfinite(w2.grad).all()


def test_minescore_gap_gradient_finite_differences():
    """Centred differences of the GPU forward in the gap, on pairs whose
    traced path is the same at gap - h, gap and gap + h (unique-path
    instances: the score is affine in the gap there)."""
    import torch
    import paper_1512_01641_amd as nw
    b = corpus.make_batch(4, pairs=16)
    mn = _miner(b)
    dev = mn.ctx.device
    w = torch.as_tensor(H.load_oriented(4)).to(dev)
    h = 1.0 / 256

    def run(g):
        gap = torch.tensor(g, dtype=torch.float32, device=dev, requires_grad=True)
        s = nw.MineScore.apply(w, gap, mn, -1.0)    # threshold below every S: kept = path
        s.sum().backward()
        torch.cuda.synchronize()
        kept = [mn.kept_pairs(q).copy() for q in range(b.B)]
        return s.detach().cpu().numpy().astype(np.float64), gap.grad.item(), kept

    s0, g0, k0 = run(b.gap)
    sp, _, kp = run(b.gap + h)
    sm, _, km = run(b.gap - h)
    same = [np.array_equal(k0[q], kp[q]) and np.array_equal(k0[q], km[q]) for q in range(b.B)]
    print("unique-path pairs at gap +- h: %d of %d" % (sum(same), b.B))
    assert sum(same) >= 1
    for q in range(b.B):
        if not same[q]:
            continue
        G = int(b.n[q] + b.m[q] - 2 * len(k0[q]))
        fd = (sp[q] - sm[q]) / (2 * h)
        # FP32 path sums: rounding of order sqrt(n + m) ulps per score
        assert abs(fd - G) <= 1e-2 * max(1.0, abs(G)), (q, fd, G)
    assert g0 == pytest.approx(sum(int(b.n[q] + b.m[q]) - 2 * len(k0[q]) for q in range(b.B)), rel=1e-12)
