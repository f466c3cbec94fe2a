"""libnwmine: comparable-corpus mining hot path on one MI355X (gfx950).

Thin Python binding over the C ABI in include/libnwmine.h.  PyTorch provides
device memory and streams only; every step of the path runs in the library's
HIP kernels.  There is no CPU fallback: importing works anywhere, but every
call needs the built ``libnwmine.so`` and a gfx950 GPU, and raises otherwise.

Method: Wolk & Marasek, arXiv 1512.01641 -- sentence-pair similarity from a
classifier over a bilingual dictionary (Sec. 4), Needleman-Wunsch alignment of
the two sentence sequences (Sec. 5.1), a threshold filter (Sec. 4) and tuning
of threshold and penalty (Sec. 5.2).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import NWM_BF16, NWM_FP32, NwmError

__all__ = ["Context", "DeviceBatch", "DeviceDict", "Plan", "Miner", "BiMiner", "score_pairs", "align_batch",
           "align_check", "align_batch_noalloc", "align_backward", "mine", "union_kept", "NWAlign", "MineScore",
           "LogisticScore", "NWM_FP32", "NWM_BF16", "NwmError"]


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A library context on one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = _abi.load()
        h = ctypes.c_void_p()
        _abi.check(self.lib.nwm_create(ctypes.byref(h), int(device)), "nwm_create")
        self.h = h
        self.device = torch.device("cuda", int(device))

    def close(self):
        if getattr(self, "h", None):
            self.lib.nwm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceBatch:
    """Sentence token CSR of a batch of document pairs on the GPU.

    ``n``, ``m``: per-pair sentence counts (host); ``src_off``/``tgt_off``:
    int64 token offsets over all sentences (pairs concatenated in order);
    ``src_tok``/``tgt_tok``: int32 token ids."""

    def __init__(self, n, m, src_off, src_tok, tgt_off, tgt_tok, V: int, device, max_sent_tokens=None):
        self.n = np.ascontiguousarray(n, np.int32)
        self.m = np.ascontiguousarray(m, np.int32)
        self.V = int(V)
        dev = torch.device(device)
        self.src_off = torch.as_tensor(np.ascontiguousarray(src_off, np.int64)).to(dev)
        self.src_tok = torch.as_tensor(np.ascontiguousarray(src_tok, np.int32)).to(dev)
        self.tgt_off = torch.as_tensor(np.ascontiguousarray(tgt_off, np.int64)).to(dev)
        self.tgt_tok = torch.as_tensor(np.ascontiguousarray(tgt_tok, np.int32)).to(dev)
        self.src_tokens = int(src_off[-1]) if len(src_off) else 0
        self.tgt_tokens = int(tgt_off[-1]) if len(tgt_off) else 0
        if max_sent_tokens is None:
            so = np.asarray(src_off)
            max_sent_tokens = int(np.diff(so).max()) if len(so) > 1 else 0
        self.max_sent_tokens = int(max_sent_tokens)
        to = np.asarray(tgt_off)
        self.max_tgt_sent_tokens = int(np.diff(to).max()) if len(to) > 1 else 0
        self.device = dev

    def reversed(self) -> "DeviceBatch":
        """The same document pairs with the roles of the two sides swapped
        (target sentences as the source side); shares the device arrays."""
        r = DeviceBatch.__new__(DeviceBatch)
        r.n, r.m, r.V, r.device = self.m, self.n, self.V, self.device
        r.src_off, r.src_tok, r.tgt_off, r.tgt_tok = self.tgt_off, self.tgt_tok, self.src_off, self.src_tok
        r.src_tokens, r.tgt_tokens = self.tgt_tokens, self.src_tokens
        r.max_sent_tokens, r.max_tgt_sent_tokens = self.max_tgt_sent_tokens, self.max_sent_tokens
        return r

    @classmethod
    def from_host(cls, b, device="cuda:0"):
        """From any object with the fields of ``synth.corpus.Batch``."""
        return cls(b.n, b.m, b.src_off, b.src_tok, b.tgt_off, b.tgt_tok, b.V, device)

    @property
    def B(self):
        return int(self.n.shape[0])

    def c(self):
        return _abi.Batch(self.B, self.V, self.n.ctypes.data_as(ctypes.c_void_p),
                          self.m.ctypes.data_as(ctypes.c_void_p), self.src_tokens, self.tgt_tokens,
                          self.max_sent_tokens, _ptr(self.src_off), _ptr(self.src_tok), _ptr(self.tgt_off),
                          _ptr(self.tgt_tok))


class DeviceDict:
    """Bilingual dictionary D as a device CSR (V rows)."""

    def __init__(self, row_off, col, val, V: int, device, max_deg=None):
        self.V = int(V)
        dev = torch.device(device)
        ro = np.ascontiguousarray(row_off, np.int32)
        self.row_off = torch.as_tensor(ro).to(dev)
        self.col = torch.as_tensor(np.ascontiguousarray(col, np.int32)).to(dev)
        self.val = torch.as_tensor(np.ascontiguousarray(val, np.float32)).to(dev)
        self.max_deg = int(np.diff(ro).max()) if max_deg is None else int(max_deg)

    @classmethod
    def from_host(cls, b, device="cuda:0"):
        return cls(b.d_row_off, b.d_col, b.d_val, b.V, device, getattr(b, "d_deg", None))

    def c(self):
        return _abi.Dict(self.V, self.max_deg, _ptr(self.row_off), _ptr(self.col), _ptr(self.val))


class Plan:
    """Plan of one batch shape: offsets, tile lists, DP order, buffer sizes."""

    def __init__(self, ctx: Context, batch: DeviceBatch, max_deg: int, prec: int = NWM_FP32):
        self.ctx = ctx
        self.lib = ctx.lib
        self.batch = batch
        h = ctypes.c_void_p()
        _abi.check(self.lib.nwm_plan_create(ctx.h, ctypes.byref(batch.c()), int(max_deg), int(prec),
                                            ctypes.byref(h)), "nwm_plan_create")
        self.h = h
        self.prec = prec
        s = _abi.Sizes()
        _abi.check(self.lib.nwm_plan_sizes(h, ctypes.byref(s)), "nwm_plan_sizes")
        self.S_elems, self.kept_cap, self.tb_bytes, self.ws_bytes = (int(s.S_elems), int(s.kept_cap),
                                                                     int(s.tb_bytes), int(s.ws_bytes))

    def workspace(self):
        return torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=self.ctx.device)

    def set_param(self, name: str, value: int):
        """A launch parameter (see nwm_param): fill_waves_per_cu,
        merge_waves_per_cu, score_xcd_map, dp_hot_percent."""
        _abi.check(self.lib.nwm_plan_set_param(self.h, _abi.PARAMS[name], int(value)), "nwm_plan_set_param")

    def get_param(self, name: str) -> int:
        v = ctypes.c_int32(0)
        _abi.check(self.lib.nwm_plan_get_param(self.h, _abi.PARAMS[name], ctypes.byref(v)), "nwm_plan_get_param")
        return int(v.value)

    def set_graph(self, on: bool):
        _abi.check(self.lib.nwm_plan_set_graph(self.h, int(bool(on))), "nwm_plan_set_graph")

    def set_timing(self, on: bool):
        _abi.check(self.lib.nwm_plan_set_timing(self.h, int(bool(on))), "nwm_plan_set_timing")

    KERNEL_CLASSES = ("merge", "build_a", "build_b", "score", "nw_fill", "walk", "keep", "backward", "expand_a")

    def kernel_ms(self, reset: bool = True):
        """{kernel class: (summed ms, launches)} since the last reset."""
        k = len(self.KERNEL_CLASSES)
        ms = (ctypes.c_double * k)()
        cnt = (ctypes.c_int32 * k)()
        _abi.check(self.lib.nwm_plan_kernel_ms(self.h, ms, cnt, int(bool(reset))), "nwm_plan_kernel_ms")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNEL_CLASSES)}

    def close(self):
        if getattr(self, "h", None):
            self.lib.nwm_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scorer(w):
    w = [float(x) for x in (w.detach().cpu().tolist() if torch.is_tensor(w) else w)]
    return _abi.Scorer(w[0], w[1], w[2])


def score_pairs(plan: Plan, batch: DeviceBatch, dic: DeviceDict, scorer, S, S_raw=None, ws=None):
    """nwm_score_pairs on the current stream."""
    ws = plan.workspace() if ws is None else ws
    _abi.check(plan.lib.nwm_score_pairs(plan.h, ctypes.byref(batch.c()), ctypes.byref(dic.c()), _scorer(scorer),
                                        _ptr(S), _ptr(S_raw), _ptr(ws), _stream(plan.ctx.device)),
               "nwm_score_pairs")


def align_batch(plan: Plan, S, gap: float, threshold: float, score, n_diag, kept, n_kept, tb, ws=None):
    """nwm_align_batch on the current stream."""
    _abi.check(plan.lib.nwm_align_batch(plan.h, _ptr(S), float(gap), float(threshold), _ptr(score), _ptr(n_diag),
                                        _ptr(kept), _ptr(n_kept), _ptr(tb), _ptr(ws), _stream(plan.ctx.device)),
               "nwm_align_batch")


def align_batch_noalloc(plan: Plan, S, gap: float, threshold: float, score, n_diag, kept, n_kept, tb):
    """nwm_align_batch_noalloc on the current stream: nwm_align_batch with
    the library's fixed device scratch instead of a workspace."""
    _abi.check(plan.lib.nwm_align_batch_noalloc(plan.h, _ptr(S), float(gap), float(threshold), _ptr(score),
                                                _ptr(n_diag), _ptr(kept), _ptr(n_kept), _ptr(tb),
                                                _stream(plan.ctx.device)), "nwm_align_batch_noalloc")


def align_check(plan: Plan, ws) -> bool:
    """nwm_align_check: waits for the current stream and returns True if a DP
    wave of the last alignment on `ws` gave up (those pairs have a NaN score
    and no aligned pairs), False otherwise."""
    failed = ctypes.c_int32(0)
    st = plan.lib.nwm_align_check(plan.h, _ptr(ws), ctypes.byref(failed), _stream(plan.ctx.device))
    if st not in (_abi.NWM_OK, _abi.NWM_EDEVICE) or (st == _abi.NWM_EDEVICE and not failed.value):
        _abi.check(st, "nwm_align_check")
    return bool(failed.value)


def align_backward(plan: Plan, batch: DeviceBatch, tb, n_diag, grad_score, grad_S_extra=None, grad_S=None,
                   grad_gap=None, S=None, S_raw=None, scorer=(0.0, 0.0, 0.0), grad_wb=None, ws=None):
    """nwm_align_backward on the current stream.  grad_score may be None (no
    score term: tb and n_diag are then not read)."""
    ws = plan.workspace() if ws is None else ws
    _abi.check(plan.lib.nwm_align_backward(plan.h, ctypes.byref(batch.c()), _ptr(tb), _ptr(n_diag),
                                           _ptr(grad_score), _ptr(grad_S_extra), _ptr(grad_S), _ptr(grad_gap),
                                           _ptr(S), _ptr(S_raw), _scorer(scorer), _ptr(grad_wb), _ptr(ws),
                                           _stream(plan.ctx.device)), "nwm_align_backward")


def mine(plan: Plan, batch: DeviceBatch, dic: DeviceDict, scorer, gap: float, threshold: float, S, S_raw, score,
         n_diag, kept, n_kept, tb, ws=None):
    ws = plan.workspace() if ws is None else ws
    _abi.check(plan.lib.nwm_mine(plan.h, ctypes.byref(batch.c()), ctypes.byref(dic.c()), _scorer(scorer), float(gap),
                                 float(threshold), _ptr(S), _ptr(S_raw), _ptr(score), _ptr(n_diag), _ptr(kept),
                                 _ptr(n_kept), _ptr(tb), _ptr(ws), _stream(plan.ctx.device)), "nwm_mine")


def union_kept(plan: Plan, kept_fwd, n_kept_fwd, kept_rev, n_kept_rev, kept_out, n_out):
    """Union of the kept pairs of the forward plan and of the reverse plan
    (whose pairs are (target, source)), each sentence pair once, ascending."""
    _abi.check(plan.lib.nwm_union_kept(plan.h, _ptr(kept_fwd), _ptr(n_kept_fwd), _ptr(kept_rev), _ptr(n_kept_rev),
                                       _ptr(kept_out), _ptr(n_out), _stream(plan.ctx.device)), "nwm_union_kept")


class Miner:
    """Owns a plan and the device buffers of one batch: score -> align -> keep."""

    def __init__(self, ctx: Context, batch: DeviceBatch, dic: DeviceDict, prec: int = NWM_FP32):
        self.ctx, self.batch, self.dic = ctx, batch, dic
        self.plan = Plan(ctx, batch, dic.max_deg, prec)
        dev = ctx.device
        p = self.plan
        self.ws = p.workspace()
        self.S = torch.empty(max(p.S_elems, 1), dtype=torch.float32, device=dev)
        self.S_raw = torch.empty(max(p.S_elems, 1), dtype=torch.float32, device=dev)
        B = batch.B
        # zeroed: a backward before any alignment reads an empty path
        self.score = torch.zeros(max(B, 1), dtype=torch.float32, device=dev)
        self.n_diag = torch.zeros(max(B, 1), dtype=torch.int32, device=dev)
        self.n_kept = torch.zeros(max(B, 1), dtype=torch.int32, device=dev)
        self.kept = torch.empty((max(p.kept_cap, 1), 2), dtype=torch.int32, device=dev)
        self.tb = torch.empty(max(p.tb_bytes, 1), dtype=torch.uint8, device=dev)
        self.s_off = np.concatenate([[0], np.cumsum(batch.n.astype(np.int64) * batch.m)]).astype(np.int64)
        self.p_off = np.concatenate([[0], np.cumsum(np.minimum(batch.n, batch.m).astype(np.int64))]).astype(np.int64)

    def score_pairs(self, scorer, want_raw=True):
        score_pairs(self.plan, self.batch, self.dic, scorer, self.S, self.S_raw if want_raw else None, self.ws)

    def align(self, gap: float, threshold: float, S=None):
        align_batch(self.plan, self.S if S is None else S, gap, threshold, self.score, self.n_diag, self.kept,
                    self.n_kept, self.tb, self.ws)

    def mine(self, scorer, gap: float, threshold: float, graph: bool = False, want_raw: bool = False):
        """Score then align.  graph=True replays one captured HIP graph of the
        whole path (captured on the first call with these arguments).  S_raw
        is written only with want_raw (the backward needs it, mining does not)."""
        if not graph:
            self.score_pairs(scorer, want_raw=want_raw)
            self.align(gap, threshold)
            return
        if not getattr(self, "_graph_on", False):
            self.plan.set_graph(True)
            self._graph_on = True
        mine(self.plan, self.batch, self.dic, scorer, gap, threshold, self.S, self.S_raw if want_raw else None,
             self.score, self.n_diag, self.kept, self.n_kept, self.tb, self.ws)

    def check(self):
        """Raise NwmError(NWM_EDEVICE) if a DP wave of the last alignment gave
        up waiting for the strip above it (waits for the current stream)."""
        if align_check(self.plan, self.ws):
            raise NwmError(_abi.NWM_EDEVICE, "nwm_align_check")

    def kept_pairs(self, b: int):
        """Kept (i, j) pairs of pair b (host copy)."""
        o = int(self.p_off[b])
        k = int(self.n_kept[b].item())
        return self.kept[o:o + k].cpu().numpy()


class BiMiner:
    """Bi-directional mining (Sec. 5.4, Table 3 "BI"): the forward miner, a
    reverse miner over the same document pairs (target sentences as the
    source side, a target-to-source dictionary and its own scorer), and the
    union of what the two keep."""

    def __init__(self, ctx: Context, batch: DeviceBatch, dic_fwd: DeviceDict, dic_rev: DeviceDict,
                 prec: int = NWM_FP32):
        self.fwd = Miner(ctx, batch, dic_fwd, prec)
        self.rev = Miner(ctx, batch.reversed(), dic_rev, prec)
        dev = ctx.device
        B = batch.B
        self.p_off = self.fwd.p_off
        self.kept = torch.empty((max(2 * self.fwd.plan.kept_cap, 1), 2), dtype=torch.int32, device=dev)
        self.n_kept = torch.empty(max(B, 1), dtype=torch.int32, device=dev)

    def union(self):
        union_kept(self.fwd.plan, self.fwd.kept, self.fwd.n_kept, self.rev.kept, self.rev.n_kept, self.kept,
                   self.n_kept)

    def mine(self, scorer_fwd, scorer_rev, gap: float, threshold: float, graph: bool = False):
        self.fwd.mine(scorer_fwd, gap, threshold, graph=graph)
        self.rev.mine(scorer_rev, gap, threshold, graph=graph)
        self.union()

    def kept_pairs(self, b: int):
        """Union of pair b (host copy), (source, target) ascending."""
        o = 2 * int(self.p_off[b])
        k = int(self.n_kept[b].item())
        return self.kept[o:o + k].cpu().numpy()


def _gap_grad(ctx, gg):
    """dL/dgap in the type and on the device of the gap argument, or None
    when the gap is a plain number or needs no gradient."""
    if gg is None or not ctx.gap_tensor:
        return None
    return gg.to(dtype=ctx.gap_dtype, device=ctx.gap_device).reshape(ctx.gap_shape)


def _save_gap(ctx, gap):
    ctx.gap_tensor = torch.is_tensor(gap)
    if ctx.gap_tensor:
        ctx.gap_dtype, ctx.gap_device, ctx.gap_shape = gap.dtype, gap.device, gap.shape


class LogisticScore(torch.autograd.Function):
    """S = sigmoid(w0 S_raw + w1 rho + b) for every sentence pair (Sec. 4),
    returned as a flat [S_elems] tensor in the plan's layout.  Backward:
    dL/dw from dL/dS through nwm_align_backward with no score term (the
    alignment is not involved)."""

    @staticmethod
    def forward(ctx, w, miner: Miner):
        miner.score_pairs(w, want_raw=True)
        P = miner.plan.S_elems
        S = miner.S[:P].clone()
        ctx.save_for_backward(S, miner.S_raw[:P].clone())
        ctx.miner = miner
        ctx.w = w.detach().cpu()
        ctx.w_dtype, ctx.w_device = w.dtype, w.device
        return S

    @staticmethod
    def backward(ctx, gS):
        if not ctx.needs_input_grad[0]:
            return None, None
        mn = ctx.miner
        S, S_raw = ctx.saved_tensors
        gwb = torch.zeros(3, dtype=torch.float64, device=mn.ctx.device)
        align_backward(mn.plan, mn.batch, None, None, None, grad_S_extra=gS.contiguous().float(), S=S, S_raw=S_raw,
                       scorer=ctx.w, grad_wb=gwb, ws=mn.ws)
        return gwb.to(dtype=ctx.w_dtype, device=ctx.w_device), None


class NWAlign(torch.autograd.Function):
    """Score_b = NW score of pair b (Sec. 5.1) for similarity S (flat, the
    plan's layout) and gap.  Backward: dL/dS = a_b times the traced path's
    indicator (dense) and dL/dgap = sum_b a_b (n_b + m_b - 2 k_b).  The
    traceback is saved, so later alignments on the same miner do not change
    the gradient."""

    @staticmethod
    def forward(ctx, S, gap, miner: Miner, threshold: float = 0.5):
        Sc = S.detach().contiguous()
        if Sc.dtype != torch.float32 or Sc.numel() < miner.plan.S_elems:
            raise ValueError("S must be float32 with at least S_elems elements")
        miner.align(float(gap), threshold, S=Sc)
        ctx.miner = miner
        ctx.S_numel, ctx.S_shape = S.numel(), S.shape
        _save_gap(ctx, gap)
        ctx.save_for_backward(miner.tb.clone(), miner.n_diag.clone())
        return miner.score[:miner.batch.B].clone()

    @staticmethod
    def backward(ctx, g):
        mn = ctx.miner
        dev = mn.ctx.device
        tb, n_diag = ctx.saved_tensors
        need_S = ctx.needs_input_grad[0]
        need_gap = ctx.needs_input_grad[1] and ctx.gap_tensor
        if not (need_S or need_gap):
            return None, None, None, None
        gS = torch.zeros(max(ctx.S_numel, 1), dtype=torch.float32, device=dev) if need_S else None
        gg = torch.zeros(1, dtype=torch.float64, device=dev) if need_gap else None
        align_backward(mn.plan, mn.batch, tb, n_diag, g.contiguous().float(), grad_S=gS, grad_gap=gg, ws=mn.ws)
        gS = gS[:ctx.S_numel].reshape(ctx.S_shape) if need_S else None
        return gS, _gap_grad(ctx, gg), None, None


class MineScore(torch.autograd.Function):
    """Fused forward (score + align) with the path-sparse backward to the
    scorer weights and the gap (FP64 batch reduction), for the tuning of
    Sec. 5.2.  grad_S_extra (flat, S layout) is an extra dense dL/dS added
    in the backward."""

    @staticmethod
    def forward(ctx, w, gap, miner: Miner, threshold: float = 0.5, grad_S_extra=None):
        miner.mine(w, float(gap), threshold, want_raw=True)
        P = miner.plan.S_elems
        ctx.save_for_backward(miner.S[:P].clone(), miner.S_raw[:P].clone(), miner.tb.clone(), miner.n_diag.clone())
        ctx.miner = miner
        ctx.w = w.detach().cpu()
        ctx.w_dtype, ctx.w_device = w.dtype, w.device
        _save_gap(ctx, gap)
        ctx.extra = None if grad_S_extra is None else grad_S_extra.detach().contiguous().float()
        return miner.score[:miner.batch.B].clone()

    @staticmethod
    def backward(ctx, g):
        mn = ctx.miner
        dev = mn.ctx.device
        S, S_raw, tb, n_diag = ctx.saved_tensors
        need_w = ctx.needs_input_grad[0]
        need_gap = ctx.needs_input_grad[1] and ctx.gap_tensor
        if not (need_w or need_gap):
            return None, None, None, None, None
        gwb = torch.zeros(3, dtype=torch.float64, device=dev) if need_w else None
        gg = torch.zeros(1, dtype=torch.float64, device=dev) if need_gap else None
        align_backward(mn.plan, mn.batch, tb, n_diag, g.contiguous().float(),
                       grad_S_extra=ctx.extra if need_w else None, grad_gap=gg, S=S, S_raw=S_raw, scorer=ctx.w,
                       grad_wb=gwb, ws=mn.ws)
        gw = gwb.to(dtype=ctx.w_dtype, device=ctx.w_device) if need_w else None
        return gw, _gap_grad(ctx, gg), None, None, None
