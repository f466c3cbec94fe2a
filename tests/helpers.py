"""Shared helpers of the test suite: run the HIP path and the oracle on the
same seeded batch and compare."""
from __future__ import annotations

import numpy as np

import oracle

FLT_MIN = np.float32(np.finfo(np.float32).tiny)


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def run_gpu(batch, prec=0, scorer=None, gap=None, threshold=None, device="cuda:0", want_raw=True, params=None,
            timing=False):
    """Score + align a synth batch on the GPU; returns host numpy results.
    `params`: launch parameters set on the plan first ({name: value});
    `timing`: also return the launches per kernel class ("launches")."""
    import paper_1512_01641_amd as nw
    ctx = nw.Context(0)
    db = nw.DeviceBatch.from_host(batch, device)
    dd = nw.DeviceDict.from_host(batch, device)
    mn = nw.Miner(ctx, db, dd, prec)
    for k, v in (params or {}).items():
        mn.plan.set_param(k, v)
    w = batch.scorer if scorer is None else np.asarray(scorer, np.float32)
    if timing:
        mn.plan.set_timing(True)
    mn.score_pairs(w, want_raw=want_raw)
    mn.align(batch.gap if gap is None else gap, batch.threshold if threshold is None else threshold)
    import torch
    torch.cuda.synchronize()
    P = mn.plan.S_elems
    out = dict(S=mn.S[:P].cpu().numpy(), S_raw=mn.S_raw[:P].cpu().numpy() if want_raw else None,
               score=mn.score[:batch.B].cpu().numpy(), n_diag=mn.n_diag[:batch.B].cpu().numpy(),
               n_kept=mn.n_kept[:batch.B].cpu().numpy(), kept=mn.kept.cpu().numpy(), p_off=mn.p_off,
               miner=mn, ctx=ctx)
    if timing:
        out["launches"] = {k: v[1] for k, v in mn.plan.kernel_ms(reset=True).items()}
        mn.plan.set_timing(False)
    return out


def gpu_align_only(n, m, S32, gap, threshold, device="cuda:0", params=None):
    """GPU NW + keep on a given packed S (host FP32).  `params`: launch
    parameters set on the plan first ({name: value})."""
    import torch
    import paper_1512_01641_amd as nw
    n = np.asarray(n, np.int32)
    m = np.asarray(m, np.int32)
    ctx = nw.Context(0)
    z = np.zeros(len(n) + 0, np.int64)
    so = np.zeros(int(n.sum()) + 1, np.int64)
    to = np.zeros(int(m.sum()) + 1, np.int64)
    db = nw.DeviceBatch(n, m, so, np.zeros(0, np.int32), to, np.zeros(0, np.int32), 64, device, max_sent_tokens=0)
    plan = nw.Plan(ctx, db, 1, 0)
    for k, v in (params or {}).items():
        plan.set_param(k, v)
    dev = torch.device(device)
    S = torch.as_tensor(np.ascontiguousarray(S32, np.float32)).to(dev)
    B = len(n)
    score = torch.empty(max(B, 1), dtype=torch.float32, device=dev)
    n_diag = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    n_kept = torch.empty(max(B, 1), dtype=torch.int32, device=dev)
    kept = torch.empty((max(plan.kept_cap, 1), 2), dtype=torch.int32, device=dev)
    tb = torch.empty(max(plan.tb_bytes, 1), dtype=torch.uint8, device=dev)
    ws = plan.workspace()
    nw.align_batch(plan, S if S.numel() else None, gap, threshold, score, n_diag, kept, n_kept, tb, ws)
    torch.cuda.synchronize()
    del z
    return dict(score=score[:B].cpu().numpy(), n_diag=n_diag[:B].cpu().numpy(), n_kept=n_kept[:B].cpu().numpy(),
                kept=kept.cpu().numpy(), p_off=oracle.path_offsets(n, m), plan=plan, ctx=ctx,
                tb=tb, S=S, ws=ws, n_diag_t=n_diag, db=db)


def assert_align_equal(gpu, ora, n, m, check_path_as_kept=False):
    """Bit-exact comparison of GPU and oracle alignment results."""
    B = len(n)
    np.testing.assert_array_equal(gpu["score"].view(np.uint32), ora["score"].view(np.uint32))
    np.testing.assert_array_equal(gpu["n_diag"], ora["n_diag"])
    np.testing.assert_array_equal(gpu["n_kept"], ora["n_kept"])
    po = ora["path_off"]
    for b in range(B):
        o = int(po[b])
        k = int(ora["n_kept"][b])
        np.testing.assert_array_equal(gpu["kept"][o:o + k], ora["kept"][o:o + k], err_msg="pair %d" % b)
        if check_path_as_kept:
            kd = int(ora["n_diag"][b])
            np.testing.assert_array_equal(gpu["kept"][o:o + kd], ora["path"][o:o + kd], err_msg="path %d" % b)


def s_rel_err(S, S64):
    return np.abs(S.astype(np.float64) - S64) / np.maximum(np.abs(S64), float(FLT_MIN))


class GpuRun:
    """The batched HIP path on a whole synth batch, results kept on the GPU;
    accessors copy one pair at a time."""

    def __init__(self, batch, prec=0, scorer=None, gap=None, threshold=None, want_raw=True):
        import torch
        import paper_1512_01641_amd as nw
        self.batch = batch
        self.ctx = nw.Context(0)
        self.db = nw.DeviceBatch.from_host(batch, "cuda:0")
        self.dd = nw.DeviceDict.from_host(batch, "cuda:0")
        self.mn = nw.Miner(self.ctx, self.db, self.dd, prec)
        self.w = np.asarray(batch.scorer if scorer is None else scorer, np.float32)
        self.gap = batch.gap if gap is None else gap
        self.threshold = batch.threshold if threshold is None else threshold
        self.mn.score_pairs(self.w, want_raw=want_raw)
        self.mn.align(self.gap, self.threshold)
        torch.cuda.synchronize()
        B = batch.B
        self.s_off = oracle.s_offsets(batch.n, batch.m)
        self.p_off = oracle.path_offsets(batch.n, batch.m)
        self.score = self.mn.score[:B].cpu().numpy()
        self.n_diag = self.mn.n_diag[:B].cpu().numpy()
        self.n_kept = self.mn.n_kept[:B].cpu().numpy()

    def S(self, b):
        o0, o1 = int(self.s_off[b]), int(self.s_off[b + 1])
        return self.mn.S[o0:o1].cpu().numpy()

    def S_raw(self, b):
        o0, o1 = int(self.s_off[b]), int(self.s_off[b + 1])
        return self.mn.S_raw[o0:o1].cpu().numpy()

    def S_all(self):
        return self.mn.S[:int(self.s_off[-1])].cpu().numpy()

    def kept(self, b):
        o = int(self.p_off[b])
        return self.mn.kept[o:o + int(self.n_kept[b])].cpu().numpy()

    def kept_all(self):
        return self.mn.kept.cpu().numpy()


def load_oriented(cfg):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oriented_scorer.json")
    with open(path) as f:
        return np.asarray(json.load(f)[str(cfg)]["w"], np.float32)


def sample_pairs(batch, k, seed=0):
    """k pairs: the largest, the smallest non-empty, empty ones, and random."""
    cells = batch.n.astype(np.int64) * batch.m
    order = np.argsort(-cells, kind="stable")
    pick = [int(order[0])]
    nz = np.nonzero(cells > 0)[0]
    if len(nz):
        pick.append(int(nz[np.argmin(cells[nz])]))
    empty = np.nonzero(cells == 0)[0]
    pick += [int(x) for x in empty[:3]]
    rng = np.random.default_rng(seed)
    rest = rng.choice(batch.B, size=min(batch.B, k), replace=False)
    for x in rest:
        if len(pick) >= k:
            break
        if int(x) not in pick:
            pick.append(int(x))
    return sorted(set(pick))
