"""Benchmark of the mining hot path on one MI355X.

One step = one pass of the whole hot path over the batch: similarity of every
sentence pair (dictionary expansion, contraction + logistic scorer), NW fill,
traceback and threshold filter.  Inputs are resident in HBM before timing.

Workload of the JSON line's `value` (default): 4096 seeded synthetic document
pairs, sentence counts lognormal (median 60, clipped 20..2000, +-30 % target
skew), V = 4096, contraction operands BF16 with FP32 accumulation, DP in FP32.
Also measured on the same pairs: the batched path with FP32 operands and the
plain path (the same library called once per pair, FP32, no batching).  Two
more workloads are measured beside it (under `workloads`): 256 pairs of
5000 x 5000 sentences (V = 16384) and 100k pairs with lognormal counts
(median 60, up to 4000, 8 % empty-or-tiny sides, V = 16384, Zipf 1.05), both
BF16, the latter with the plain per-pair FP32 path on a seeded subsample.

Prints ONE JSON line.  Only one GPU is used; --gpus N > 1 exits with a
message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}
WORKLOADS = {
    2: "%d document pairs, sentence counts lognormal median 60 clipped 20-2000 (+-30%% skew), V=%d hashed vocab, "
       "Zipf(1.1) tokens, %s contraction operands, FP32 DP, gap -0.2, threshold 0.5",
    3: "%d document pairs of 5000x5000 sentences, V=%d hashed vocab, Zipf(1.1) tokens, %s contraction "
       "operands, FP32 DP, gap -0.2, threshold 0.5",
    5: "%d document pairs, sentence counts lognormal median 60 clipped 1-4000, 8%% empty-or-tiny sides, V=%d "
       "hashed vocab, Zipf(1.05) tokens, %s contraction operands, FP32 DP, gap -0.2, threshold 0.5",
}
EXTRA = {3: "256x5000x5000_V16384", 5: "100k_lognormal_V16384"}
TUNED = os.path.join(ROOT, "paper_1512_01641_amd", "tuned_params.json")


def _log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1000.0 / max(steps, 1)


def profiled_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None once the kernel's source differs from the profiled one."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["bytes_per_launch"]


# ---- algorithmic work per launch -------------------------------------------------

def compacted_chunks(batch):
    """Sum over contraction tiles (64 source x 64 target sentences of a pair)
    of the compacted K chunks the tile multiplies: ceil(K / 32), K = distinct
    words of the tile's target sentences."""
    tfirst = np.concatenate([[0], np.cumsum(batch.m, dtype=np.int64)])
    total = 0
    for p in range(batch.B):
        n, m = int(batch.n[p]), int(batch.m[p])
        if n == 0 or m == 0:
            continue
        rts = (n + 63) // 64
        for c0 in range(0, m, 64):
            a = batch.tgt_off[tfirst[p] + c0]
            b = batch.tgt_off[tfirst[p] + min(m, c0 + 64)]
            k = len(np.unique(batch.tgt_tok[a:b]))
            total += rts * ((k + 31) // 32)
    return total


def work_model(batch):
    """Algorithmic work of one launch of each kernel class over the batch,
    with its roofline bound and the definition used."""
    B, V = batch.B, batch.V
    n = batch.n.astype(np.int64)
    m = batch.m.astype(np.int64)
    cells = int(np.dot(n, m))
    n_src, n_tgt = int(n.sum()), int(m.sum())
    T_src, T_tgt = int(batch.src_tok.size), int(batch.tgt_tok.size)
    deg = np.diff(batch.d_row_off.astype(np.int64))
    E = int(deg[batch.src_tok].sum()) if T_src else 0
    nch = (V + 31) // 32
    ok = (n > 0) & (m > 0)
    n_rt = int(((n + 63) // 64)[ok].sum())
    n_ct = int(((m + 63) // 64)[ok].sum())
    n_kc = compacted_chunks(batch)
    path = int(np.minimum(n, m).sum())
    return {
        "merge": ("hbm", 4 * T_src + 8 * T_src + 8 * E + 16 * n_src + 8 * E + 4 * n_src,
                  "read: 4 B token + 8 B dictionary row offsets per source token, 8 B per dictionary entry, 16 B "
                  "per sentence; write: 8 B per merged entry (at most one per dictionary entry) + 4 B count per "
                  "sentence"),
        "build_a": ("hbm", 8 * E + 4 * n_src + 8 * E + 4 * n_rt * (nch + 1),
                    "read: 8 B per merged entry + 4 B count per sentence; write: 8 B per list entry (at most one "
                    "per merged entry) + 4 B chunk offsets per row tile and 32-word chunk"),
        "expand_a": ("hbm", 4 * T_src + 8 * T_src + 8 * E + 16 * n_src + 8 * E + 4 * n_rt * (nch + 1),
                     "fused merge + row-tile lists: read 4 B token + 8 B dictionary row offsets per source token, "
                     "8 B per dictionary entry, 16 B per sentence; write 8 B per list entry (at most one per "
                     "dictionary entry) + 4 B chunk offsets per row tile and 32-word chunk"),
        "build_b": ("hbm", 4 * T_tgt + 8 * n_tgt + 4 * T_tgt + n_ct * (4 * (nch + 1) + 16 * nch) + 4 * B * nch,
                    "read: 4 B token + 8 B offset per target token / sentence; write: 4 B list entry per token, "
                    "per column tile its chunk offsets, word masks and chunk ranges (20 B per 32-word chunk), per "
                    "pair a V-bit vocabulary"),
        "score": ("mfma", 2.0 * 64 * 64 * 32 * n_kc,
                  "2*64*64*32 flop per compacted K chunk of a 64x64 tile, %d chunks; the whole-vocabulary "
                  "definition would be 2*V*cells = %.4g flop" % (n_kc, 2.0 * V * cells)),
        "nw_fill": ("hbm", 4.25 * cells, "4.25 B/cell (4 B S read + 2-bit traceback)"),
        "walk": ("hbm", 16.0 * int((n + m)[ok].sum()) + 8 * path,
                 "16 B of direction codes per traceback step (n+m steps per pair) + 8 B per aligned pair"),
        "keep": ("hbm", 20.0 * path, "8 B aligned pair + 4 B S read + 8 B kept pair per aligned pair"),
    }, cells, n_kc


def rooflines(model, kernel_ms, prec_name):
    """Roofline object per timed kernel class (achieved = algorithmic work
    per launch / average launch duration)."""
    out = {}
    for k, (bound, work, definition) in model.items():
        ms = kernel_ms.get(k)
        if not ms or ms <= 0:
            continue
        if bound == "mfma":
            ach = work / (ms / 1000.0) / 1e12
            peak, unit = MFMA_PEAK_TFLOPS[prec_name], "TFLOP/s"
        else:
            ach = work / (ms / 1000.0) / 1e9
            peak, unit = HBM_PEAK_GBS, "GB/s"
        out[k] = {"bound": bound, "achieved": round(ach, 2), "peak": peak, "unit": unit,
                  "frac": round(ach / peak, 4), "kernel_ms": round(ms, 4), "algorithmic": definition}
    return out


KERNEL_NAMES = {"merge": "k_merge_src", "build_a": "k_build_a", "expand_a": "k_expand_a", "build_b": "k_build_b",
                "score": "k_score_c<%s>", "nw_fill": "k_nw_fill", "walk": "k_nw_walk", "keep": "k_keep"}


# ---- GPU measurements --------------------------------------------------------------

def batched(nw, torch, ctx, batch, prec_name, prec, args, db=None, dd=None):
    """Graph-replayed and eager (per-kernel events) times of the batched path."""
    db = nw.DeviceBatch.from_host(batch) if db is None else db
    dd = nw.DeviceDict.from_host(batch) if dd is None else dd
    mn = nw.Miner(ctx, db, dd, prec)
    w, gap, thr = batch.scorer, batch.gap, batch.threshold
    params = "defaults"
    for kv in args.param:
        k, v = kv.split("=")
        mn.plan.set_param(k, int(v))
        params = dict(p.split("=") for p in args.param)
    if not args.no_autotune and not args.param:
        from paper_1512_01641_amd import autotune
        r = autotune.autotune(mn, w, gap, thr, reps=5, cache_path=TUNED)
        params = dict(r["params"], source="cache" if r["cached"] else "tuned in this run")
        _log("launch parameters %s: %s" % (prec_name, params))
    step = lambda: mn.mine(w, gap, thr)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # eager launches, every kernel bracketed by HIP events on its stream
    mn.plan.set_timing(True)
    eager_ms = _time_steps(step, args.steps, 0, torch)
    km = mn.plan.kernel_ms(reset=True)
    mn.plan.set_timing(False)
    kernel = {k: v[0] / max(v[1], 1) for k, v in km.items() if v[1]}
    launches = {k: v[1] / args.steps for k, v in km.items() if v[1]}
    ms = eager_ms
    if not args.no_graph:
        gstep = lambda: mn.mine(w, gap, thr, graph=True)
        ms = _time_steps(gstep, args.steps, max(args.warmup, 1), torch)
    _log("%s: eager %.4f ms/step, %s %.4f ms/step" % (prec_name, eager_ms, "eager" if args.no_graph else "graph",
                                                      ms))
    return dict(ms=ms, eager_ms=eager_ms, kernel=kernel, launches=launches, params=params, miner=mn)


def plain(nw, torch, ctx, batch, idx, dd):
    """The same library called once per document pair (B = 1 plans, FP32,
    eager), over pairs `idx`; returns ms for the whole pass."""
    miners = []
    for k, b in enumerate(idx):
        sub = batch.subset([b])
        miners.append(nw.Miner(ctx, nw.DeviceBatch.from_host(sub), dd, nw.NWM_FP32))
        if (k + 1) % 1024 == 0:
            _log("plain setup %d/%d" % (k + 1, len(idx)))
    w, gap, thr = batch.scorer, batch.gap, batch.threshold

    def one_pass():
        for mnb in miners:
            mnb.mine(w, gap, thr)
    ms = _time_steps(one_pass, 1, 1, torch)
    del miners
    return ms


def summarize(batch, res, prec_name, counted):
    """`counted`: the committed counter traffic was taken on this workload
    (the full 4096-pair one); elsewhere traffic is null."""
    model, cells, n_kc = work_model(batch)
    rl = rooflines(model, res["kernel"], prec_name)
    for k, r in rl.items():
        name = KERNEL_NAMES[k] % prec_name if "%" in KERNEL_NAMES[k] else KERNEL_NAMES[k]
        r["kernel"] = name
        r["traffic"] = profiled_traffic(name) if counted else None
    dom = max(rl, key=lambda k: rl[k]["kernel_ms"])
    fill = res["kernel"].get("nw_fill")
    return dict(pairs_per_s=round(batch.B / (res["ms"] / 1000.0), 2), ms_per_step=round(res["ms"], 4),
                ms_per_step_eager=round(res["eager_ms"], 4),
                gcups=round(cells / (fill / 1000.0) / 1e9, 3) if fill else None,
                kernel_ms_per_step={k: round(v, 4) for k, v in res["kernel"].items()},
                launches_per_step=res["launches"], launch_params=res["params"],
                rooflines=rl, dominant=dom)


# ---- CPU baseline (the oracle) -----------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_pass(oracle, sub, nthreads):
    t0 = time.perf_counter()
    sc = oracle.score(sub, nthreads=nthreads)
    t1 = time.perf_counter()
    oracle.align(sub.n, sub.m, sc["S32"], sub.gap, sub.threshold, nthreads=nthreads)
    t2 = time.perf_counter()
    return sc, t1 - t0, t2 - t1


def cpu_baseline(nw, torch, ctx, batch, head_miner, head_prec, dd):
    """The CPU oracle (FP64 scores, FP32 DP + keep) timed on the host cores,
    on all of them and on one thread, with the S and DP phases separately;
    then the parity figures of the GPU path against it on the same workload."""
    import oracle
    from synth import corpus
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cores = max(1, min(avail, oracle.max_threads(), int(os.environ.get("OMP_NUM_THREADS", avail))))
    # all cores: leading pairs worth about 10 s at a conservative 1e8 cells/s (the
    # whole benchmark workload takes about a second)
    cum = np.cumsum(batch.n.astype(np.int64) * batch.m)
    k = max(1, min(batch.B, int(np.searchsorted(cum, 10.0 * 1e8)) + 1))
    sub = batch.subset(range(k)) if k < batch.B else batch
    sc, ts, td = _oracle_pass(oracle, sub, cores)
    dt = ts + td
    # one thread: leading pairs sized to about 8 s at the rate just measured
    rate1 = sub.cells() / dt / cores
    k1 = max(1, min(batch.B, int(np.searchsorted(cum, 8.0 * rate1)) + 1))
    sub1 = batch.subset(range(k1))
    _, ts1, td1 = _oracle_pass(oracle, sub1, 1)
    out = {"value": round(sub.B / dt, 3), "unit": "doc-pairs/s", "cores": cores, "kind": "oracle",
           "sample": "first %d of %d pairs (%d cells): score FP64 + NW FP32 + keep, %.2f s on %d threads" % (
               sub.B, batch.B, sub.cells(), dt, cores),
           "cpu_model": cpu_model(),
           "phase_s": {"score": round(ts, 3), "nw_and_keep": round(td, 3)},
           "single_thread": {"value": round(sub1.B / (ts1 + td1), 3), "unit": "doc-pairs/s", "cores": 1,
                             "sample": "first %d pairs (%d cells)" % (sub1.B, sub1.cells()),
                             "phase_s": {"score": round(ts1, 3), "nw_and_keep": round(td1, 3)}}}
    # parity of the GPU's batched run (head precision) on the same pairs
    s_off = oracle.s_offsets(batch.n, batch.m)
    S_gpu = head_miner.S[:int(s_off[sub.B])].cpu().numpy()
    dS = np.abs(S_gpu.astype(np.float64) - sc["S64"])
    al = oracle.align(sub.n, sub.m, S_gpu, batch.gap, batch.threshold, nthreads=cores)
    score = head_miner.score[:sub.B].cpu().numpy()
    n_kept = head_miner.n_kept[:sub.B].cpu().numpy()
    kept = head_miner.kept.cpu().numpy()
    exact = (score.view(np.uint32) == al["score"].view(np.uint32)) & (n_kept == al["n_kept"]) & (
        head_miner.n_diag[:sub.B].cpu().numpy() == al["n_diag"])
    p_off = al["path_off"]
    for b in np.nonzero(exact)[0]:
        o, kk = int(p_off[b]), int(n_kept[b])
        exact[b] = np.array_equal(kept[o:o + kk], al["kept"][o:o + kk])
    # planted-alignment F1 with the oriented scorer (FP64 oracle vs the GPU)
    with open(os.path.join(ROOT, "tests", "golden", "oriented_scorer.json")) as f:
        wo = np.asarray(json.load(f)[str(batch.cfg)]["w"], np.float32)
    fs = batch.subset(range(min(batch.B, 512)))
    so = oracle.score(fs, scorer=wo, nthreads=cores)
    ao = oracle.align(fs.n, fs.m, so["S32"], fs.gap, fs.threshold, nthreads=cores)
    gold = [fs.gold[fs.gold_off[q]:fs.gold_off[q + 1]] for q in range(fs.B)]
    f64 = oracle.f1([oracle.pair_kept(ao, q) for q in range(fs.B)], gold)
    fm = nw.Miner(ctx, nw.DeviceBatch.from_host(fs), dd, head_prec)
    fm.mine(wo, fs.gap, fs.threshold)
    torch.cuda.synchronize()
    fg = oracle.f1([fm.kept_pairs(q) for q in range(fs.B)], gold)
    out["parity"] = {
        "pairs": sub.B,
        "max_abs_dS_vs_fp64": float(dS.max()) if dS.size else 0.0,
        "dp_bitexact_rate": round(float(exact.mean()) if exact.size else 1.0, 6),
        "dp_definition": "oracle NW + keep on the GPU's S vs the GPU's score bits, path length and kept pairs",
        "f1_planted_fp64": round(f64, 3), "f1_planted_gpu": round(fg, 3), "f1_delta_points": round(fg - f64, 3),
        "f1_definition": "oriented scorer, first %d pairs, kept pairs vs the planted alignment" % fs.B}
    return out


# ---- main -------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pairs", type=int, default=None, help="fewer pairs of the same workload (testing)")
    ap.add_argument("--workload", type=int, choices=(2, 3, 5), default=2,
                    help="2: 4096 pairs, lognormal median 60, V=4096 (the benchmark line); 3: 256 pairs of "
                         "5000x5000, V=16384; 5: 100k pairs, lognormal median 60, V=16384")
    ap.add_argument("--no-extra", action="store_true", help="skip the 256x5000x5000 and 100k-pair workloads")
    ap.add_argument("--extra-steps", type=int, default=3)
    ap.add_argument("--plain-sample", type=int, default=1000,
                    help="pairs of the 100k-pair workload timed on the plain per-pair path (seeded sample)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-bidir", action="store_true", help="skip the bi-directional mining measurement")
    ap.add_argument("--no-search", action="store_true", help="skip the random-search tuning measurement")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="time eager launches only")
    ap.add_argument("--prec", choices=("both", "bf16", "f32"), default="both")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    ap.add_argument("--param", action="append", default=[], metavar="NAME=VALUE",
                    help="set a launch parameter on every plan (implies --no-autotune)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="run a plain device copy of MIB MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU only: the document pairs are independent, so N GPUs would each run "
              "the one-GPU path on a shard of the batch (see the design notes); no multi-GPU figure is made.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1512_01641_amd as nw
    from synth import corpus

    cfg = args.workload
    _log("generating workload %d" % cfg)
    batch = corpus.make_batch(cfg, pairs=args.pairs)
    B, V = batch.B, batch.V
    cells = batch.cells()
    ctx = nw.Context(0)
    db = nw.DeviceBatch.from_host(batch)
    dd = nw.DeviceDict.from_host(batch)
    w, gap, thr = batch.scorer, batch.gap, batch.threshold
    torch.cuda.synchronize()

    if args.copy_probe:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # give the factor that turns counter readings into bytes
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        _log("copy probe: %d bytes read, %d bytes written per copy" % (nbytes, nbytes))
        del src, dst

    precs = [p for p in (("bf16", nw.NWM_BF16), ("f32", nw.NWM_FP32)) if args.prec in ("both", p[0])]
    head, head_prec = precs[0]
    runs = {}
    for prec_name, prec in precs:
        _log("batched %s" % prec_name)
        runs[prec_name] = batched(nw, torch, ctx, batch, prec_name, prec, args, db, dd)
        if prec_name != head:
            runs[prec_name].pop("miner")
    head_sum = summarize(batch, runs[head], head, counted=cfg == 2 and args.pairs is None)

    bidir = None
    if not args.no_bidir:
        # bi-directional mining (Sec. 5.4, Table 3 "BI"): forward + reverse
        # direction (target side as the source, reverse dictionary) + union
        _log("bi-directional %s" % head)
        rbatch = corpus.reverse_batch(batch)
        bm = nw.BiMiner(ctx, db, dd, nw.DeviceDict.from_host(rbatch), head_prec)
        gb = not args.no_graph
        bstep = lambda: bm.mine(w, rbatch.scorer, gap, thr, graph=gb)
        bi_ms = _time_steps(bstep, args.steps, max(args.warmup, 1), torch)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            bm.union()
        ev1.record()
        torch.cuda.synchronize()
        bidir = {"pairs_per_s": round(B / (bi_ms / 1000.0), 2), "ms_per_step": round(bi_ms, 4),
                 "union_ms": round(ev0.elapsed_time(ev1) / args.steps, 4),
                 "kept_pairs_forward": int(bm.fwd.n_kept[:B].sum().item()),
                 "kept_pairs_bidirectional": int(bm.n_kept[:B].sum().item()),
                 "launch": "two graph replays + union kernel" if gb else "eager"}
        del bm

    search = None
    if not args.no_search:
        # the tuning script (Sec. 5.2): random search over (threshold, gap) on
        # a 100-pair tuning set (the paper tunes on 100 human-aligned pairs;
        # planted alignments stand in)
        from paper_1512_01641_amd import tune
        tb_ = batch.subset(range(min(100, B)))
        smn = nw.Miner(ctx, nw.DeviceBatch.from_host(tb_), dd, head_prec)
        tune.random_search(smn, w, tb_.gold_off, tb_.gold, trials=2, seed=1)   # warm-up
        torch.cuda.synchronize()
        trials = 64
        t0 = time.perf_counter()
        res = tune.random_search(smn, w, tb_.gold_off, tb_.gold, trials=trials, seed=0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        search = {"trials_per_s": round(trials / dt, 2), "pairs": tb_.B, "trials": trials,
                  "best": {"threshold": res["threshold"], "gap": res["gap"], "similarity": round(res["similarity"], 3)},
                  "note": "per trial: NW fill + traceback + keep on the GPU, similarity on the host"}
        del smn

    plain_ms = None
    if not args.no_plain:
        _log("plain per-pair FP32 (%d pairs)" % B)
        plain_ms = plain(nw, torch, ctx, batch, range(B), dd)

    cpu = None
    if not args.no_cpu:
        _log("cpu baseline")
        cpu = cpu_baseline(nw, torch, ctx, batch, runs[head]["miner"], head_prec, dd)
    runs[head].pop("miner")
    del db

    extra = {}
    if not args.no_extra:
        for xc in (3, 5):
            if xc == cfg:
                continue
            _log("workload %d: generating" % xc)
            xb = corpus.make_batch(xc)
            xd = nw.DeviceDict.from_host(xb)
            xa = argparse.Namespace(**vars(args))
            xa.steps, xa.warmup = args.extra_steps, 1
            r = batched(nw, torch, ctx, xb, "bf16", nw.NWM_BF16, xa, dd=xd)
            r.pop("miner")
            s = summarize(xb, r, "bf16", counted=False)
            s.update(pairs=xb.B, cells=xb.cells(), V=xb.V, workload=WORKLOADS[xc] % (xb.B, xb.V, "BF16"))
            if xc == 5 and not args.no_plain:
                rng = np.random.default_rng(1512)
                idx = np.sort(rng.choice(xb.B, size=min(args.plain_sample, xb.B), replace=False))
                _log("workload 5: plain per-pair FP32 on %d sampled pairs" % len(idx))
                pms = plain(nw, torch, ctx, xb, idx, xd)
                pps = len(idx) / (pms / 1000.0)
                s["pairs_per_s_plain_fp32"] = round(pps, 2)
                s["plain_sample"] = "%d pairs drawn by numpy default_rng(1512) without replacement" % len(idx)
                s["ratio_batched_bf16_vs_plain_fp32"] = round(s["pairs_per_s"] / pps, 2)
            extra[EXTRA[xc]] = s
            del xb, xd
            torch.cuda.empty_cache()

    hs = head_sum
    dom = hs["dominant"]
    out = {
        "metric": "NW GCUPS + aligned doc-pairs/s, batched BF16 vs plain FP32, same GPU",
        "value": hs["pairs_per_s"],
        "unit": "doc-pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hs["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic (seeded comparable-corpus generator with planted alignments)",
        "config": {"workload": WORKLOADS[cfg] % (B, V, head.upper()), "pairs": B, "cells": cells, "V": V},
        "gcups": hs["gcups"],
        "launch": "eager" if args.no_graph else "hipGraph replay of the whole path per step",
        "launch_params": {p: r["params"] for p, r in runs.items()},
        "ms_per_step_eager": {p: round(r["eager_ms"], 4) for p, r in runs.items()},
        "pairs_per_s_batched_fp32": round(B / (runs["f32"]["ms"] / 1000.0), 2) if "f32" in runs else None,
        "pairs_per_s_plain_fp32": round(B / (plain_ms / 1000.0), 2) if plain_ms else None,
        "ratio_batched_bf16_vs_plain_fp32": round(plain_ms / hs["ms_per_step"], 2) if plain_ms else None,
        "kernel_ms_per_step": {p: {k: round(v, 4) for k, v in r["kernel"].items()} for p, r in runs.items()},
        "rooflines": hs["rooflines"],
        "contraction_roofline": hs["rooflines"].get("score"),
        "dp_roofline": hs["rooflines"].get("nw_fill"),
    }
    # `roofline`: the kernel that took longest per step in the eager timed
    # region (every kernel class is a candidate; all are in `rooflines`)
    out["roofline"] = dict(hs["rooflines"][dom], dominant_class=dom)
    if extra:
        out["workloads"] = extra
    if bidir is not None:
        out["bidirectional"] = bidir
    if search is not None:
        out["random_search"] = search
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
