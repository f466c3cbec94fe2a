// C ABI of libnwmine: context, plan and the hot-path entry points.
// Host code only; every step of the path runs in the HIP kernels of k_*.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "libnwmine.h"
#include "nwm_internal.h"

namespace nwm {
hipError_t launch_merge_src(int64_t, const int64_t *, int64_t, const int64_t *, const int32_t *, const int32_t *,
                            const int32_t *, const float *, int, int, int, uint2 *, int32_t *, int, hipStream_t);
hipError_t launch_build_a(const PlanDev &, const int64_t *, const uint2 *, const int32_t *, uint2 *, int32_t *,
                          int, int, int, int64_t *, const uint32_t *, int, int, hipStream_t);
hipError_t launch_build_b(const PlanDev &, const int64_t *, const int32_t *, uint32_t *, int32_t *, int, int, int,
                          uint2 *, int32_t *, int2 *, int64_t *, uint32_t *, int, int, hipStream_t);
hipError_t launch_clear_u32(uint32_t *, int64_t, hipStream_t);
hipError_t launch_expand_a(const PlanDev &, const int64_t *, const int32_t *, const uint2 *, int, int, uint2 *,
                           int32_t *, int, int, int, int64_t *, int, int, hipStream_t);
bool expand_a_fits(int max_sent_tokens, int max_deg, int nch);
hipError_t launch_pack_dict(const int32_t *, const int32_t *, const float *, int, int, uint2 *, hipStream_t);
hipError_t build_set_attrs(int nch, int V);
hipError_t launch_score(const PlanDev &, bool, const int64_t *, const int64_t *, const uint2 *, const int32_t *,
                        const uint32_t *, const int32_t *, nwm_scorer, float *, float *, int, int, int, const uint2 *,
                        const int32_t *, const int2 *, const int64_t *, const int64_t *, int, int, hipStream_t);
size_t score_lds_bytes(int nch, bool bf16);
hipError_t score_set_attrs(int nch_max);
hipError_t launch_nw_fill(const PlanDev &, const float *, float, float *, char *, uint64_t *, int64_t, int32_t *,
                          int, int, int, int, hipStream_t);
hipError_t fill_set_attrs(int);
hipError_t launch_nw_reset(const PlanDev &, float, float *, uint64_t *, int64_t, int32_t *, hipStream_t);
hipError_t launch_nw_fill_items(const PlanDev &, const float *, float, float *, char *, uint64_t *, int64_t,
                                int32_t *, int32_t *, int, int, int, int, int, int, int, int, hipStream_t);
hipError_t launch_nw_walk(const PlanDev &, const char *, const float *, int2 *, int32_t *, int, int, hipStream_t);
hipError_t launch_keep(const PlanDev &, const float *, float, const int2 *, const int32_t *, int2 *, int32_t *, int,
                       int, hipStream_t);
hipError_t merge_set_attrs(int max_entries);
hipError_t launch_union_kept(int, const int64_t *, const int2 *, const int32_t *, const int2 *, const int32_t *,
                             int2 *, int32_t *, hipStream_t);
hipError_t launch_backward(const PlanDev &, const int64_t *, const int64_t *, const int2 *, const int32_t *,
                           const float *, const float *, float *, double *, const float *, const float *,
                           double *, float *, float *, hipStream_t);
}  // namespace nwm

using namespace nwm;

struct nwm_ctx {
  int device = 0;
  size_t lds_max = 0;
};

namespace {

// kernel classes of the per-kernel timing (nwm_kclass)
enum {
  K_MERGE = NWM_K_MERGE,
  K_BUILD_A = NWM_K_BUILD_A,
  K_BUILD_B = NWM_K_BUILD_B,
  K_SCORE = NWM_K_SCORE,
  K_FILL = NWM_K_FILL,
  K_WALK = NWM_K_WALK,
  K_KEEP = NWM_K_KEEP,
  K_BWD = NWM_K_BACKWARD,
  K_EXPAND_A = NWM_K_EXPAND_A,
  K_CLASSES = NWM_N_KCLASSES
};

struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (class, index of start event)
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void clear() {
    used = 0;
    marks.clear();
  }
  ~Timer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// Device scratch of nwm_align_batch_noalloc: the DP's queue heads and error
// flag (first 256 bytes), then the published boundary rows between strips.
// Every GPU the library runs on holds its own
// copy until the process ends; the host reaches it only through the address
// hipGetSymbolAddress gives on that device (the array's name in host code is
// not a device address).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_BYTES / 8];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Once per device, with that device current: the device address of `scratch`.
hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[dev] = ptr;
  return hipSuccess;
}

void *scratch_ptr(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}
}  // namespace

struct nwm_plan {
  nwm_ctx *ctx = nullptr;
  int device = 0;   // the context's device (kept here: a plan may outlive its context's handle)
  int B = 0, V = 0, max_deg = 0;
  nwm_prec prec = NWM_FP32;
  int64_t n_src = 0, n_tgt = 0, src_tokens = 0, tgt_tokens = 0;
  int64_t n_bnd = 0;   // uint64 entries of the published-row region
  int max_entries = 1; // dictionary entries of the longest source sentence (tokens x max_deg)
  // launch parameters (nwm_param) and what re-deriving the DP priority flags needs
  int32_t param[NWM_N_PARAMS] = {0, 0, 1, 50, 1, 0, 0, 1, 0, 1};
  int max_sent_tokens = 0;   // the batch's bound on tokens per sentence
  uint64_t param_version = 0;
  std::vector<int32_t> it_strip;   // strip index per DP item (no flags)
  std::vector<int64_t> it_chain;   // dependency chain of the item's pair
  std::vector<int32_t> tk_slot;    // strip index and link flags per task slot (no priority flag)
  std::vector<int64_t> tk_chain;   // dependency chain of the slot's pair (0: empty slot)
  int64_t max_chain = 0;
  int max_m = 0;
  // the pairs whose DP dependency chain is at least LONG_CHAIN_PERCENT of
  // the longest come first in every order (sentences, tiles, DP items,
  // pairs); nwm_mine prepares and scores them first and runs their DP on a
  // stream of its own while the main stream prepares, scores and aligns the
  // others
  int n_gt_long = 0, n_items_long = 0, n_pairs_long = 0, n_rt_long = 0, n_ct_long = 0;
  int64_t n_sent_long = 0;
  // the first of the long pairs (chain >= TOP_CHAIN_PERCENT of the longest):
  // their contraction tiles, DP items and pairs lead the long pairs' ranges
  int n_gt_top = 0, n_items_top = 0, n_pairs_top = 0, n_rt_top = 0, n_ct_top = 0;
  int n_tasks_top = 0, n_tasks_long = 0;   // the same ranges in tasks
  int64_t n_sent_top = 0;
  hipStream_t lane_stream = nullptr;   // the top pairs' DP
  hipEvent_t ev_top = nullptr, ev_top_done = nullptr;
  hipStream_t exp_stream = nullptr;    // the other pairs' source-side expansion
  hipEvent_t ev_long = nullptr, ev_long_done = nullptr, ev_b_long = nullptr, ev_b_rest = nullptr, ev_b_top = nullptr;
  hipEvent_t ev_a_rest = nullptr;
  std::vector<int32_t> n, m;
  void *dmeta = nullptr;
  PlanDev dev{};
  WsLayout ws{};
  nwm_sizes sizes{};
  Timer timer;
  // graph replay of nwm_mine: captured on cap_stream, keyed by the arguments
  bool graph_on = false;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  // second stream for the target-side tile lists (fork / join by events)
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::vector<uint64_t> graph_key;
};

namespace {

// The HIP error behind the last NWM_EDEVICE of this thread (nwm_last_device_error).
thread_local hipError_t g_last_hip_error = hipSuccess;

nwm_status dev_err(hipError_t e) {
  if (e == hipSuccess) return NWM_OK;
  g_last_hip_error = e;
  return NWM_EDEVICE;
}

// Launch checks read hipGetLastError, which also returns an error left by an
// earlier, unrelated HIP call of this thread (another library's, or a failed
// destroy): entry points clear it first, so a failure they report is their
// own.
void clear_stale_error() { (void)hipGetLastError(); }

// DP item words: strip index, plus ITEM_HOT for pairs whose dependency chain
// is at least NWM_PARAM_DP_HOT_PERCENT of the longest
void hot_flags(const nwm_plan *p, std::vector<int32_t> &out, std::vector<int32_t> &tasks) {
  const int64_t pct = p->param[NWM_PARAM_DP_HOT_PERCENT];
  auto hot = [&](int64_t chain) { return pct > 0 && chain > 0 && chain * 100 >= pct * p->max_chain; };
  out.resize(p->it_strip.size());
  for (size_t k = 0; k < out.size(); ++k) out[k] = p->it_strip[k] | (hot(p->it_chain[k]) ? ITEM_HOT : 0);
  tasks.resize(p->tk_slot.size());
  for (size_t k = 0; k < tasks.size(); ++k) tasks[k] = p->tk_slot[k] | (hot(p->tk_chain[k]) ? ITEM_HOT : 0);
}

struct Mark {
  nwm_plan *p;
  int cls;
  hipStream_t st;
  size_t idx = 0;
  bool active = false;
  Mark(nwm_plan *p_, int c, hipStream_t s) : p(p_), cls(c), st(s) {
    if (p->timer.on && !p->capturing) {
      hipEvent_t a = p->timer.get(), b = p->timer.get();
      if (a && b && hipEventRecord(a, st) == hipSuccess) {
        idx = p->timer.used - 2;
        active = true;
      }
    }
  }
  void done() {
    if (active) {
      if (hipEventRecord(p->timer.pool[idx + 1], st) == hipSuccess) p->timer.marks.push_back({cls, idx});
      active = false;
    }
  }
};

bool finite(float x) { return std::isfinite(x); }


}  // namespace

extern "C" {

const char *nwm_last_device_error(void) {
  return g_last_hip_error == hipSuccess ? "none" : hipGetErrorName(g_last_hip_error);
}

const char *nwm_strerror(nwm_status s) {
  switch (s) {
    case NWM_OK: return "ok";
    case NWM_EINVAL: return "invalid argument";
    case NWM_ESHAPE: return "inconsistent shapes";
    case NWM_ENOMEM: return "out of memory";
    case NWM_EDEVICE: return "HIP device error";
    case NWM_EUNSUPPORTED: return "size limit exceeded";
  }
  return "unknown status";
}

nwm_status nwm_create(nwm_ctx **ctx, int hip_device) {
  if (!ctx) return NWM_EINVAL;
  *ctx = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count) return NWM_EDEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) return NWM_EDEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return NWM_EDEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return NWM_EDEVICE;
  // the device address of the no-allocation entry point's scratch
  if (scratch_init(hip_device) != hipSuccess) return NWM_EDEVICE;
  nwm_ctx *c = new (std::nothrow) nwm_ctx();
  if (!c) return NWM_ENOMEM;
  c->device = hip_device;
  c->lds_max = prop.sharedMemPerBlock;
  *ctx = c;
  return NWM_OK;
}

void nwm_destroy(nwm_ctx *ctx) { delete ctx; }

nwm_status nwm_plan_create(nwm_ctx *ctx, const nwm_batch *batch, int32_t max_deg, nwm_prec prec,
                           nwm_plan **plan_out) {
  if (!ctx || !batch || !plan_out) return NWM_EINVAL;
  *plan_out = nullptr;
  if (prec != NWM_FP32 && prec != NWM_BF16) return NWM_EINVAL;
  const int B = batch->B;
  if (B < 0 || batch->V <= 0 || max_deg <= 0 || batch->src_tokens < 0 || batch->tgt_tokens < 0 ||
      batch->max_sent_tokens < 0)
    return NWM_EINVAL;
  if (B > 0 && (!batch->n_host || !batch->m_host)) return NWM_EINVAL;
  if (batch->V > MAX_V || max_deg > MAX_DEG || (int64_t)batch->max_sent_tokens * max_deg > MERGE_SLOTS)
    return NWM_EUNSUPPORTED;
  nwm_plan *p = new (std::nothrow) nwm_plan();
  if (!p) return NWM_ENOMEM;
  p->ctx = ctx;
  p->device = ctx->device;
  p->B = B;
  p->V = batch->V;
  p->max_deg = max_deg;
  p->prec = prec;
  p->src_tokens = batch->src_tokens;
  p->tgt_tokens = batch->tgt_tokens;
  p->max_entries = std::max(1, batch->max_sent_tokens * max_deg);
  p->max_sent_tokens = batch->max_sent_tokens;
  p->n.assign(batch->n_host, batch->n_host + B);
  p->m.assign(batch->m_host, batch->m_host + B);
  for (int b = 0; b < B; ++b) {
    if (p->n[b] < 0 || p->m[b] < 0) {
      delete p;
      return NWM_EINVAL;
    }
    if (p->m[b] > MAX_M) {
      delete p;
      return NWM_EUNSUPPORTED;
    }
    p->max_m = std::max(p->max_m, p->m[b]);
  }
  const int nch = (p->V + KC - 1) / KC;
  // ---- host metadata ---------------------------------------------------------
  std::vector<int64_t> sfirst(B + 1, 0), tfirst(B + 1, 0), s_off(B + 1, 0), p_off(B + 1, 0), tb_off(B + 1, 0);
  std::vector<int32_t> rt_pair, rt_row0, rt_rows, ct_pair, ct_col0, ct_cols, gt_rt, gt_ct;
  for (int b = 0; b < B; ++b) {
    const int64_t nb = p->n[b], mb = p->m[b];
    sfirst[b + 1] = sfirst[b] + nb;
    tfirst[b + 1] = tfirst[b] + mb;
    s_off[b + 1] = s_off[b] + nb * mb;
    p_off[b + 1] = p_off[b] + std::min(nb, mb);
    int64_t bits = 0;
    if (nb > 0 && mb > 0) bits = ((nb + 63) / 64) * ((mb + 63 + 63) / 64) * 1024;
    tb_off[b + 1] = tb_off[b] + bits;
  }
  // dependency chain of a pair's DP: one hand-off of ~80 steps per strip
  // plus the m + 63 steps of the last strip
  auto chain = [&](int b) { return (int64_t)((p->n[b] + 63) / 64 - 1) * 80 + p->m[b] + 63; };
  p->max_chain = 0;
  for (int b = 0; b < B; ++b)
    if (p->n[b] > 0 && p->m[b] > 0) p->max_chain = std::max(p->max_chain, chain(b));
  // the long pairs: dependency chain at least LONG_CHAIN_PERCENT of the longest
  std::vector<char> is_long(B, 0);
  for (int b = 0; b < B; ++b)
    is_long[b] = p->n[b] > 0 && p->m[b] > 0 && p->max_chain > 0 &&
                 100 * chain(b) >= (int64_t)LONG_CHAIN_PERCENT * p->max_chain;
  std::vector<char> is_top(B, 0);
  for (int b = 0; b < B; ++b)
    is_top[b] = is_long[b] && 100 * chain(b) >= (int64_t)TOP_CHAIN_PERCENT * p->max_chain;
  // tiles and source sentences in lane order: the long pairs first (longest
  // chain first, so the top pairs lead), then the others in pair order
  std::vector<int32_t> lane_pairs;
  for (int b = 0; b < B; ++b)
    if (is_long[b]) lane_pairs.push_back(b);
  std::stable_sort(lane_pairs.begin(), lane_pairs.end(), [&](int a, int c) { return chain(a) > chain(c); });
  const size_t n_long_pairs = lane_pairs.size();
  for (int b = 0; b < B; ++b)
    if (!is_long[b]) lane_pairs.push_back(b);
  std::vector<int64_t> sent_ids;
  sent_ids.reserve((size_t)sfirst[B]);
  p->n_rt_long = p->n_ct_long = p->n_gt_long = 0;
  p->n_sent_long = 0;
  p->n_gt_top = p->n_rt_top = p->n_ct_top = 0;
  p->n_sent_top = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const size_t q0 = pass == 0 ? 0 : n_long_pairs, q1 = pass == 0 ? n_long_pairs : lane_pairs.size();
    for (size_t q = q0; q < q1; ++q) {
      const int b = lane_pairs[q];
      const int64_t nb = p->n[b], mb = p->m[b];
      for (int64_t i = sfirst[b]; i < sfirst[b + 1]; ++i) sent_ids.push_back(i);
      const int rt0 = (int)rt_pair.size(), ct0 = (int)ct_pair.size();
      for (int r = 0; r < nb; r += TM) {
        rt_pair.push_back(b);
        rt_row0.push_back(r);
        rt_rows.push_back((int)std::min<int64_t>(TM, nb - r));
      }
      for (int c = 0; c < mb; c += TN) {
        ct_pair.push_back(b);
        ct_col0.push_back(c);
        ct_cols.push_back((int)std::min<int64_t>(TN, mb - c));
      }
      const int nrt = (int)rt_pair.size() - rt0, nct = (int)ct_pair.size() - ct0;
      for (int ri = 0; ri < nrt; ++ri)
        for (int ci = 0; ci < nct; ++ci) {
          gt_rt.push_back(rt0 + ri);
          gt_ct.push_back(ct0 + ci);
        }
      if (is_top[b]) {
        p->n_gt_top = (int)gt_rt.size();
        p->n_rt_top = (int)rt_pair.size();
        p->n_ct_top = (int)ct_pair.size();
        p->n_sent_top = (int64_t)sent_ids.size();
      }
    }
    if (pass == 0) {
      p->n_rt_long = (int)rt_pair.size();
      p->n_ct_long = (int)ct_pair.size();
      p->n_gt_long = (int)gt_rt.size();
      p->n_sent_long = (int64_t)sent_ids.size();
    }
  }
  p->n_src = sfirst[B];
  p->n_tgt = tfirst[B];
  std::vector<TileMeta> rt_meta(rt_pair.size()), ct_meta(ct_pair.size());
  for (size_t k = 0; k < rt_pair.size(); ++k)
    rt_meta[k] = TileMeta{sfirst[rt_pair[k]] + rt_row0[k], rt_rows[k], rt_pair[k]};
  for (size_t k = 0; k < ct_pair.size(); ++k)
    ct_meta[k] = TileMeta{tfirst[ct_pair[k]] + ct_col0[k], ct_cols[k], ct_pair[k]};
  std::vector<GtMeta> gt_meta(gt_rt.size());
  for (size_t g = 0; g < gt_rt.size(); ++g) {
    GtMeta &x = gt_meta[g];
    x.rt = gt_rt[g];
    x.ct = gt_ct[g];
    x.pair = rt_pair[x.rt];
    x.m = p->m[x.pair];
    x.row0 = rt_row0[x.rt];
    x.rows = rt_rows[x.rt];
    x.col0 = ct_col0[x.ct];
    x.cols = ct_cols[x.ct];
    x.s_first = sfirst[x.pair] + x.row0;
    x.t_first = tfirst[x.pair] + x.col0;
    x.s_off = s_off[x.pair];
    x.pad = 0;
  }
  // pair order of the DP, the walk and the keep: long pairs first (longest
  // chain first), then the others by cells, largest first
  std::vector<int32_t> order(B);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    if (is_long[a] != is_long[c]) return is_long[a] > is_long[c];
    if (is_long[a]) return chain(a) > chain(c);
    return (int64_t)p->n[a] * p->m[a] > (int64_t)p->n[c] * p->m[c];
  });
  p->n_pairs_long = p->n_pairs_top = 0;
  for (int b = 0; b < B; ++b) {
    p->n_pairs_long += is_long[b] ? 1 : 0;
    p->n_pairs_top += is_top[b] ? 1 : 0;
  }
  // DP work items: every strip of every non-empty pair, longest pair first;
  // boundary rows between consecutive strips
  std::vector<int32_t> it_pair, it_strip;
  std::vector<int64_t> bnd_off(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    const int64_t ns = (p->n[b] > 0 && p->m[b] > 0) ? (p->n[b] + 63) / 64 : 0;
    const int64_t links = ns > 0 ? ns - 1 : 0;
    bnd_off[b + 1] = bnd_off[b] + links * bnd_stride(p->m[b]);
  }
  // DP items in pair order (so the long pairs' strips come first); strips
  // of pairs on the longest chains run at raised wave priority (hot_flags)
  for (int q = 0; q < B; ++q) {
    const int b = order[q];
    if (p->n[b] <= 0 || p->m[b] <= 0) continue;
    for (int s = 0; s < (p->n[b] + 63) / 64; ++s) {
      it_pair.push_back(b);
      p->it_strip.push_back(s);
      p->it_chain.push_back(chain(b));
    }
    if (is_long[b]) p->n_items_long = (int)it_pair.size();
    if (is_top[b]) p->n_items_top = (int)it_pair.size();
  }
  // Queue order inside each launch (top pairs, other long pairs, the rest):
  // by the latest step at which a strip can start without lengthening the
  // longest chain, max_chain - chain(pair) + STRIP_LAG * strip.  A strip can
  // start about STRIP_LAG steps after the one above it; popping a pair's
  // strips one after another instead would leave most of them waiting for
  // their predecessors while holding a wave (on 256 pairs of 5000 x 5000
  // sentences about half of all wave time).  Strips of one pair keep their
  // order (a strip's predecessor is always popped first), and among equal
  // keys the pair order above (longest chain first) is kept.
  {
    const size_t N = it_pair.size();
    std::vector<int64_t> key(N);
    for (size_t k = 0; k < N; ++k)
      key[k] = (p->max_chain - p->it_chain[k]) + (int64_t)STRIP_LAG * p->it_strip[k];
    const size_t cut[4] = {0, (size_t)p->n_items_top, (size_t)p->n_items_long, N};
    std::vector<size_t> idx(N);
    std::iota(idx.begin(), idx.end(), (size_t)0);
    for (int r = 0; r < 3; ++r)
      std::stable_sort(idx.begin() + cut[r], idx.begin() + cut[r + 1],
                       [&](size_t a, size_t c) { return key[a] < key[c]; });
    std::vector<int32_t> ip(N), is(N);
    std::vector<int64_t> ic(N);
    for (size_t k = 0; k < N; ++k) {
      ip[k] = it_pair[idx[k]];
      is[k] = p->it_strip[idx[k]];
      ic[k] = p->it_chain[idx[k]];
    }
    it_pair.swap(ip);
    p->it_strip.swap(is);
    p->it_chain.swap(ic);
  }
  // Tasks of the LDS-ring fill, FILL_SLOTS strips each, in the same queue
  // order and the same three ranges.  Strips 4g .. 4g + 3 of a pair (fewer
  // at its end) form one linked group, placed where strip 4g stands in the
  // queue into consecutive slots of one task, each handing its last row to
  // the next through LDS; strips of one-strip pairs take single slots.  A
  // group that does not fit in the open task's free slots closes it (its
  // empty slots, pair -1, wait for the task's end).
  std::vector<int32_t> tk_pair;
  {
    const size_t cut[4] = {0, (size_t)p->n_items_top, (size_t)p->n_items_long, it_pair.size()};
    for (int r = 0; r < 3; ++r) {
      int fill = 0;   // used slots of the open task
      auto push_slot = [&](int32_t pb, int32_t word, int64_t chain) {
        tk_pair.push_back(pb);
        p->tk_slot.push_back(word);
        p->tk_chain.push_back(chain);
        if (++fill == FILL_SLOTS) fill = 0;
      };
      auto close_task = [&]() {
        while (fill > 0) push_slot(-1, 0, 0);
      };
      for (size_t k = cut[r]; k < cut[r + 1]; ++k) {
        const int32_t pb = it_pair[k], st = p->it_strip[k];
        const int32_t ns = (p->n[pb] + 63) / 64;
        if (st % FILL_SLOTS != 0) continue;   // placed with strip st - st % FILL_SLOTS
        const int cnt = std::min(FILL_SLOTS, ns - st);
        if (fill + cnt > FILL_SLOTS) close_task();
        for (int q = 0; q < cnt; ++q)
          push_slot(pb, (st + q) | (q > 0 ? ITEM_LINK_IN : 0) | (q + 1 < cnt ? ITEM_LINK_OUT : 0), p->it_chain[k]);
      }
      close_task();
      if (r == 0) p->n_tasks_top = (int)(tk_pair.size() / FILL_SLOTS);
      if (r == 1) p->n_tasks_long = (int)(tk_pair.size() / FILL_SLOTS);
    }
  }
  std::vector<int32_t> tk_words;
  hot_flags(p, it_strip, tk_words);
  // ---- device metadata: one allocation -----------------------------------------
  struct Piece {
    const void *src;
    size_t bytes;
    size_t off;
  };
  std::vector<Piece> pieces;
  size_t tot = 0;
  auto add = [&](const void *src, size_t bytes) {
    pieces.push_back({src, bytes, tot});
    tot = align_up(tot + std::max<size_t>(bytes, 1), 256);
    return pieces.size() - 1;
  };
  size_t i_n = add(p->n.data(), 4 * (size_t)B), i_m = add(p->m.data(), 4 * (size_t)B);
  size_t i_sf = add(sfirst.data(), 8 * (size_t)(B + 1)), i_tf = add(tfirst.data(), 8 * (size_t)(B + 1));
  size_t i_so = add(s_off.data(), 8 * (size_t)(B + 1)), i_po = add(p_off.data(), 8 * (size_t)(B + 1));
  size_t i_to = add(tb_off.data(), 8 * (size_t)(B + 1));
  size_t i_rp = add(rt_pair.data(), 4 * rt_pair.size()), i_rr = add(rt_row0.data(), 4 * rt_row0.size());
  size_t i_rn = add(rt_rows.data(), 4 * rt_rows.size());
  size_t i_cp = add(ct_pair.data(), 4 * ct_pair.size()), i_cc = add(ct_col0.data(), 4 * ct_col0.size());
  size_t i_cn = add(ct_cols.data(), 4 * ct_cols.size());
  size_t i_gr = add(gt_rt.data(), 4 * gt_rt.size()), i_gc = add(gt_ct.data(), 4 * gt_ct.size());
  size_t i_gm = add(gt_meta.data(), sizeof(GtMeta) * gt_meta.size());
  size_t i_rm = add(rt_meta.data(), sizeof(TileMeta) * rt_meta.size());
  size_t i_cm = add(ct_meta.data(), sizeof(TileMeta) * ct_meta.size());
  size_t i_do = add(order.data(), 4 * order.size());
  size_t i_si = add(sent_ids.data(), 8 * sent_ids.size());
  size_t i_ip = add(it_pair.data(), 4 * it_pair.size()), i_is = add(it_strip.data(), 4 * it_strip.size());
  size_t i_tp = add(tk_pair.data(), 4 * tk_pair.size()), i_ts = add(tk_words.data(), 4 * tk_words.size());
  size_t i_bo = add(bnd_off.data(), 8 * (size_t)(B + 1));
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete p;
    return NWM_EDEVICE;
  }
  if (hipMalloc(&p->dmeta, tot) != hipSuccess) {
    delete p;
    return NWM_ENOMEM;
  }
  std::vector<char> host(tot, 0);
  for (auto &pc : pieces)
    if (pc.bytes) std::memcpy(host.data() + pc.off, pc.src, pc.bytes);
  if (hipMemcpy(p->dmeta, host.data(), tot, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p->dmeta);
    delete p;
    return NWM_EDEVICE;
  }
  char *d = static_cast<char *>(p->dmeta);
  auto at = [&](size_t i) { return (void *)(d + pieces[i].off); };
  PlanDev &D = p->dev;
  D.B = B;
  D.V = p->V;
  D.max_deg = max_deg;
  D.nch = nch;
  D.n = (const int32_t *)at(i_n);
  D.m = (const int32_t *)at(i_m);
  D.sfirst = (const int64_t *)at(i_sf);
  D.tfirst = (const int64_t *)at(i_tf);
  D.s_off = (const int64_t *)at(i_so);
  D.p_off = (const int64_t *)at(i_po);
  D.tb_off = (const int64_t *)at(i_to);
  D.n_rt = (int)rt_pair.size();
  D.n_ct = (int)ct_pair.size();
  D.rt_pair = (const int32_t *)at(i_rp);
  D.rt_row0 = (const int32_t *)at(i_rr);
  D.rt_rows = (const int32_t *)at(i_rn);
  D.ct_pair = (const int32_t *)at(i_cp);
  D.ct_col0 = (const int32_t *)at(i_cc);
  D.ct_cols = (const int32_t *)at(i_cn);
  D.n_gt = (int)gt_rt.size();
  D.gt_rt = (const int32_t *)at(i_gr);
  D.gt_ct = (const int32_t *)at(i_gc);
  D.gt_meta = (const GtMeta *)at(i_gm);
  D.rt_meta = (const TileMeta *)at(i_rm);
  D.ct_meta = (const TileMeta *)at(i_cm);
  D.dp_order = (const int32_t *)at(i_do);
  D.sent_ids = (const int64_t *)at(i_si);
  D.n_items = (int)it_pair.size();
  D.it_pair = (const int32_t *)at(i_ip);
  D.it_strip = (const int32_t *)at(i_is);
  D.n_tasks = (int)(tk_pair.size() / FILL_SLOTS);
  D.tk_pair = (const int32_t *)at(i_tp);
  D.tk_slot = (const int32_t *)at(i_ts);
  D.bnd_off = (const int64_t *)at(i_bo);
  D.path_base = (int64_t)align_up((size_t)tb_off[B], 256);
  // ---- workspace layout ------------------------------------------------------------
  WsLayout &W = p->ws;
  size_t o = 0;
  auto carve = [&](size_t bytes) {
    size_t r = o;
    o = align_up(o + std::max<size_t>(bytes, 1), 256);
    return r;
  };
  const size_t a_ent = (size_t)p->src_tokens * (size_t)max_deg;
  W.a_merged = carve(8 * a_ent);
  W.d_pack = carve(8 * 4 * (size_t)p->V);
  W.a_cnt = carve(4 * (size_t)p->n_src);
  W.a_list = carve(8 * (a_ent + LIST_SLACK_A));
  W.a_choff = carve(4 * (size_t)D.n_rt * (size_t)(nch + 1));
  W.b_list = carve(4 * ((size_t)p->tgt_tokens + LIST_SLACK_B));
  W.b_choff = carve(4 * (size_t)D.n_ct * (size_t)(nch + 1));
  W.b_mt = carve(8 * (size_t)D.n_ct * (size_t)nch);
  W.b_kcn = carve(4 * (size_t)D.n_ct);
  W.b_rng = carve(8 * (size_t)D.n_ct * (size_t)nch);
  W.a_base = carve(8 * (size_t)D.n_rt);
  W.b_base = carve(8 * (size_t)D.n_ct);
  W.p_voc = carve(4 * (size_t)B * (size_t)nch);
  W.bwd = carve(16 * ((size_t)B + (size_t)D.n_rt));
  // published rows, + 2 entries (cleared in 16-byte units)
  W.bnd = carve(8 * ((size_t)bnd_off[B] + 2));
  p->n_bnd = bnd_off[B] + 2;
  W.ctl = carve(16);
  W.total = o;
  p->sizes.S_elems = (size_t)s_off[B];
  p->sizes.kept_cap = (size_t)p_off[B];
  p->sizes.tb_bytes = (size_t)D.path_base + 8 * (size_t)p_off[B];
  p->sizes.ws_bytes = W.total;
  // ---- kernel attributes (dynamic LDS above the default) ---------------------------
  if (merge_set_attrs(p->max_entries) != hipSuccess || score_set_attrs(nch) != hipSuccess ||
      build_set_attrs(nch, p->V) != hipSuccess || fill_set_attrs(0) != hipSuccess) {
    (void)hipFree(p->dmeta);
    delete p;
    return NWM_EDEVICE;
  }
  *plan_out = p;
  return NWM_OK;
}

nwm_status nwm_plan_sizes(const nwm_plan *plan, nwm_sizes *sizes) {
  if (!plan || !sizes) return NWM_EINVAL;
  *sizes = plan->sizes;
  return NWM_OK;
}

void nwm_plan_destroy(nwm_plan *plan) {
  if (!plan) return;
  (void)hipSetDevice(plan->device);
  if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
  if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
  if (plan->aux_stream) (void)hipStreamDestroy(plan->aux_stream);
  if (plan->ev_fork) (void)hipEventDestroy(plan->ev_fork);
  if (plan->ev_join) (void)hipEventDestroy(plan->ev_join);
  if (plan->ev_long) (void)hipEventDestroy(plan->ev_long);
  if (plan->ev_b_long) (void)hipEventDestroy(plan->ev_b_long);
  if (plan->ev_b_top) (void)hipEventDestroy(plan->ev_b_top);
  if (plan->ev_b_rest) (void)hipEventDestroy(plan->ev_b_rest);
  if (plan->lane_stream) (void)hipStreamDestroy(plan->lane_stream);
  if (plan->exp_stream) (void)hipStreamDestroy(plan->exp_stream);
  if (plan->ev_a_rest) (void)hipEventDestroy(plan->ev_a_rest);
  if (plan->ev_long_done) (void)hipEventDestroy(plan->ev_long_done);
  if (plan->ev_top) (void)hipEventDestroy(plan->ev_top);
  if (plan->ev_top_done) (void)hipEventDestroy(plan->ev_top_done);
  if (plan->dmeta) (void)hipFree(plan->dmeta);
  delete plan;
}

static nwm_status check_batch(const nwm_plan *p, const nwm_batch *b) {
  if (!b) return NWM_EINVAL;
  if (b->B != p->B || b->V != p->V || b->src_tokens != p->src_tokens || b->tgt_tokens != p->tgt_tokens)
    return NWM_ESHAPE;
  if (p->n_src > 0 && (!b->src_off || (p->src_tokens > 0 && !b->src_tok))) return NWM_EINVAL;
  if (p->n_tgt > 0 && (!b->tgt_off || (p->tgt_tokens > 0 && !b->tgt_tok))) return NWM_EINVAL;
  return NWM_OK;
}

// Merged dictionary rows and tile lists of a batch (the expansion), then the
// contraction of tiles [g0, g0 + G).
static nwm_status check_score_args(const nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, nwm_scorer sc,
                                   const float *S, const void *ws) {
  if (!p || !dict) return NWM_EINVAL;
  nwm_status s = check_batch(p, batch);
  if (s != NWM_OK) return s;
  if (dict->V != p->V || dict->max_deg > p->max_deg || dict->max_deg <= 0) return NWM_ESHAPE;
  if (!finite(sc.w0) || !finite(sc.w1) || !finite(sc.b)) return NWM_EINVAL;
  if (p->sizes.S_elems == 0) return NWM_OK;
  if (!S || !ws || !dict->row_off || !dict->col || !dict->val) return NWM_EINVAL;
  return NWM_OK;
}

// The two-kernel source path of the compacted contraction leaves out source
// entries whose word no target sentence of the pair holds: the column-tile
// builders form each pair's vocabulary, the row-tile builders of a pair wait
// for them.  The fused path keeps those entries (the contraction never finds
// their words in a tile's vocabulary) and waits for nothing.
// The source side runs as one fused kernel per row tile.
static bool fused_a(const nwm_plan *p) {
  return p->param[NWM_PARAM_EXPAND_FUSED] && expand_a_fits(p->max_sent_tokens, p->max_deg, p->dev.nch);
}

static uint32_t *pair_vocab(nwm_plan *p, void *ws) {
  // only the two-kernel source path filters by the pair's target vocabulary
  return p->param[NWM_PARAM_SCORE_COMPACT] && !fused_a(p) ? (uint32_t *)(static_cast<char *>(ws) + p->ws.p_voc)
                                                          : nullptr;
}

// The source-side expansion of part of the batch on `st`: merged dictionary
// rows of source sentences sent_ids[k0, k0 + ns), then (once `tgt_done` has
// been reached, when given: the column tiles of the same pairs are built) the
// lists of row tiles [r0, r0 + nr), which hold exactly those sentences.
static hipError_t expand_src(nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, void *ws, int64_t k0,
                             int64_t ns, int r0, int nr, hipEvent_t tgt_done, hipStream_t st) {
  char *w = static_cast<char *>(ws);
  uint2 *merged = (uint2 *)(w + p->ws.a_merged);
  int32_t *cnt = (int32_t *)(w + p->ws.a_cnt);
  const bool bf16 = p->prec == NWM_BF16;
  // list entries of the dense contraction are LDS byte offsets inside the
  // operand tiles
  const int pitch = bf16 ? PITCH_BF16 : PITCH_F32;
  const int esize = bf16 ? 2 : 4;
  if (fused_a(p)) {
    // no dependency on the target side; the wait keeps the contract that the
    // contraction queued after this on `st` finds both sides built
    Mark mx(p, K_EXPAND_A, st);
    hipError_t e = launch_expand_a(p->dev, batch->src_off, batch->src_tok, (const uint2 *)(w + p->ws.d_pack), p->V,
                                   p->max_entries, (uint2 *)(w + p->ws.a_list), (int32_t *)(w + p->ws.a_choff),
                                   pitch, esize, p->param[NWM_PARAM_SCORE_COMPACT], (int64_t *)(w + p->ws.a_base),
                                   r0, nr, st);
    mx.done();
    if (e == hipSuccess && tgt_done) e = hipStreamWaitEvent(st, tgt_done, 0);
    return e;
  }
  Mark mk(p, K_MERGE, st);
  hipError_t e = launch_merge_src(ns, p->dev.sent_ids, k0, batch->src_off, batch->src_tok, dict->row_off, dict->col,
                                  dict->val, p->V, p->max_deg, p->max_entries, merged, cnt,
                                  p->param[NWM_PARAM_MERGE_WAVES_PER_CU], st);
  mk.done();
  if (e == hipSuccess && tgt_done) e = hipStreamWaitEvent(st, tgt_done, 0);
  Mark ma(p, K_BUILD_A, st);
  if (e == hipSuccess)
    e = launch_build_a(p->dev, batch->src_off, merged, cnt, (uint2 *)(w + p->ws.a_list),
                       (int32_t *)(w + p->ws.a_choff), pitch, esize, p->param[NWM_PARAM_SCORE_COMPACT],
                       (int64_t *)(w + p->ws.a_base), pair_vocab(p, ws), r0, nr, st);
  ma.done();
  return e;
}

// The lists of column tiles [c0, c0 + nc) on `st`; `first` clears the pair
// vocabularies beforehand (once per pass over the batch).
static hipError_t expand_tgt(nwm_plan *p, const nwm_batch *batch, void *ws, int c0, int nc, bool first,
                             hipStream_t st) {
  char *w = static_cast<char *>(ws);
  const bool bf16 = p->prec == NWM_BF16;
  uint32_t *voc = pair_vocab(p, ws);
  Mark mk(p, K_BUILD_B, st);
  hipError_t e = hipSuccess;
  if (first && voc) e = launch_clear_u32(voc, (int64_t)p->B * p->dev.nch, st);
  if (e == hipSuccess)
    e = launch_build_b(p->dev, batch->tgt_off, batch->tgt_tok, (uint32_t *)(w + p->ws.b_list),
                       (int32_t *)(w + p->ws.b_choff), bf16 ? PITCH_BF16 : PITCH_F32, bf16 ? 2 : 4,
                       p->param[NWM_PARAM_SCORE_COMPACT], (uint2 *)(w + p->ws.b_mt), (int32_t *)(w + p->ws.b_kcn),
                       (int2 *)(w + p->ws.b_rng), (int64_t *)(w + p->ws.b_base), voc, c0, nc, st);
  mk.done();
  return e;
}

// The whole expansion.  The target-side lists do not depend on the source
// side: they are built on the plan's second stream, forked from `st` by an
// event, while `st` merges the source rows; the row-tile lists wait for them
// (under graph capture: a parallel branch of the graph joined there).
// The fused source path reads the dictionary padded to four entries per row
// (one 8-byte load per entry): packed on `st` before any expansion forks off.
// (untimed: a few microseconds, kept out of the per-launch averages of the
// kernel classes)
static hipError_t pack_dict(nwm_plan *p, const nwm_dict *dict, void *ws, hipStream_t st) {
  if (!fused_a(p)) return hipSuccess;
  return launch_pack_dict(dict->row_off, dict->col, dict->val, p->V, p->max_deg,
                          (uint2 *)(static_cast<char *>(ws) + p->ws.d_pack), st);
}

static hipError_t expand_lists(nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, void *ws, hipStream_t st) {
  hipError_t e = pack_dict(p, dict, ws, st);
  if (e == hipSuccess) e = hipEventRecord(p->ev_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->aux_stream, p->ev_fork, 0);
  if (e == hipSuccess) e = expand_tgt(p, batch, ws, 0, p->dev.n_ct, true, p->aux_stream);
  if (e == hipSuccess) e = hipEventRecord(p->ev_join, p->aux_stream);
  if (e == hipSuccess) e = expand_src(p, batch, dict, ws, 0, p->n_src, 0, p->dev.n_rt, p->ev_join, st);
  return e;
}

static hipError_t score_tiles(nwm_plan *p, const nwm_batch *batch, nwm_scorer sc, float *S, float *S_raw, void *ws,
                              int g0, int G, hipStream_t st) {
  char *w = static_cast<char *>(ws);
  Mark mk(p, K_SCORE, st);
  hipError_t e = launch_score(p->dev, p->prec == NWM_BF16, batch->src_off, batch->tgt_off, (uint2 *)(w + p->ws.a_list),
                              (int32_t *)(w + p->ws.a_choff), (uint32_t *)(w + p->ws.b_list),
                              (int32_t *)(w + p->ws.b_choff), sc, S, S_raw, p->param[NWM_PARAM_SCORE_XCD_MAP],
                              p->param[NWM_PARAM_SCORE_COMPACT], p->param[NWM_PARAM_SCORE_KGROUP],
                              (uint2 *)(w + p->ws.b_mt),
                              (int32_t *)(w + p->ws.b_kcn), (int2 *)(w + p->ws.b_rng), (int64_t *)(w + p->ws.a_base),
                              (int64_t *)(w + p->ws.b_base), g0, G, st);
  mk.done();
  return e;
}

static hipError_t ensure_streams(nwm_plan *p) {
  if (p->aux_stream) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&p->aux_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->lane_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->exp_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_a_rest, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_long, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_long_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_b_long, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_b_top, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_b_rest, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_top, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_top_done, hipEventDisableTiming);
  return e;
}

nwm_status nwm_score_pairs(nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, nwm_scorer sc, float *S,
                           float *S_raw, void *ws, void *stream) {
  clear_stale_error();
  nwm_status s = check_score_args(p, batch, dict, sc, S, ws);
  if (s != NWM_OK || p->sizes.S_elems == 0) return s;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = ensure_streams(p);
  if (e == hipSuccess) e = expand_lists(p, batch, dict, ws, st);
  if (e == hipSuccess) e = score_tiles(p, batch, sc, S, S_raw, ws, 0, p->dev.n_gt, st);
  return dev_err(e);
}

nwm_status nwm_align_batch(nwm_plan *p, const float *S, float gap, float threshold, float *score,
                           int32_t *n_diag, int32_t *kept, int32_t *n_kept, void *tb, void *ws, void *stream) {
  clear_stale_error();
  if (!p) return NWM_EINVAL;
  if (!finite(gap) || !finite(threshold)) return NWM_EINVAL;
  if (p->B == 0) return NWM_OK;
  if (!score || !n_diag || !n_kept) return NWM_EINVAL;
  if (p->sizes.S_elems > 0 && !S) return NWM_EINVAL;
  if (p->sizes.kept_cap > 0 && (!kept || !tb)) return NWM_EINVAL;
  if (!ws) return NWM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  char *w = static_cast<char *>(ws);
  char *tbc = static_cast<char *>(tb);
  int2 *path = tbc ? (int2 *)(tbc + p->dev.path_base) : nullptr;
  hipError_t e;
  {
    Mark mk(p, K_FILL, st);
    e = launch_nw_fill(p->dev, S, gap, score, tbc, (uint64_t *)(w + p->ws.bnd), p->n_bnd,
                       (int32_t *)(w + p->ws.ctl), p->param[NWM_PARAM_FILL_WAVES_PER_CU],
                       p->param[NWM_PARAM_DP_SPIN_LIMIT], p->param[NWM_PARAM_DP_TEST_HOLD],
                       p->param[NWM_PARAM_FILL_STAGING], st);
    mk.done();
  }
  if (e != hipSuccess) return dev_err(e);
  {
    Mark mk(p, K_WALK, st);
    e = launch_nw_walk(p->dev, tbc, score, path, n_diag, 0, p->B, st);
    mk.done();
  }
  if (e == hipSuccess) {
    Mark mk(p, K_KEEP, st);
    e = launch_keep(p->dev, S, threshold, path, n_diag, (int2 *)kept, n_kept, 0, p->B, st);
    mk.done();
  }
  return dev_err(e);
}

nwm_status nwm_align_check(const nwm_plan *p, const void *ws, int32_t *failed, void *stream) {
  if (failed) *failed = 0;
  if (!p) return NWM_EINVAL;
  if (p->B == 0) return NWM_OK;
  if (!ws) return NWM_EINVAL;
  int32_t flag = 0;
  const char *w = static_cast<const char *>(ws);
  hipStream_t st = (hipStream_t)stream;
  if (hipMemcpyAsync(&flag, w + p->ws.ctl + 4, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return NWM_EDEVICE;
  if (failed) *failed = flag != 0;
  return flag != 0 ? NWM_EDEVICE : NWM_OK;
}

nwm_status nwm_align_batch_noalloc(nwm_plan *p, const float *S, float gap, float threshold, float *score,
                                   int32_t *n_diag, int32_t *kept, int32_t *n_kept, void *tb, void *stream) {
  if (!p) return NWM_EINVAL;
  if (!finite(gap) || !finite(threshold)) return NWM_EINVAL;
  if (p->B == 0) return NWM_OK;
  if (!score || !n_diag || !n_kept) return NWM_EINVAL;
  if (p->sizes.S_elems > 0 && !S) return NWM_EINVAL;
  if (p->sizes.kept_cap > 0 && (!kept || !tb)) return NWM_EINVAL;
  // [256 B: queue heads, error flag][published rows]
  const size_t need = 256 + 8 * (size_t)p->n_bnd;
  if (need > NOALLOC_SCRATCH_BYTES) return NWM_EUNSUPPORTED;
  char *base = static_cast<char *>(scratch_ptr(p->device));
  if (!base) return NWM_EDEVICE;
  clear_stale_error();
  hipStream_t st = (hipStream_t)stream;
  char *tbc = static_cast<char *>(tb);
  int2 *path = tbc ? (int2 *)(tbc + p->dev.path_base) : nullptr;
  int32_t *ctl = reinterpret_cast<int32_t *>(base);
  uint64_t *bnd = reinterpret_cast<uint64_t *>(base + 256);
  // the reset kernel clears the queue heads, the error flag and the published
  // rows' tags left by the previous call (no memset node, no allocation)
  hipError_t e = launch_nw_fill(p->dev, S, gap, score, tbc, bnd, p->n_bnd, ctl, p->param[NWM_PARAM_FILL_WAVES_PER_CU],
                                p->param[NWM_PARAM_DP_SPIN_LIMIT], p->param[NWM_PARAM_DP_TEST_HOLD],
                                p->param[NWM_PARAM_FILL_STAGING], st);
  if (e == hipSuccess) e = launch_nw_walk(p->dev, tbc, score, path, n_diag, 0, p->B, st);
  if (e == hipSuccess) e = launch_keep(p->dev, S, threshold, path, n_diag, (int2 *)kept, n_kept, 0, p->B, st);
  return dev_err(e);
}

nwm_status nwm_align_backward(nwm_plan *p, const nwm_batch *batch, const void *tb, const int32_t *n_diag,
                              const float *grad_score, const float *grad_S_extra, float *grad_S, double *grad_gap,
                              const float *S, const float *S_raw, nwm_scorer sc, double *grad_wb, void *ws,
                              void *stream) {
  (void)sc;
  if (!p) return NWM_EINVAL;
  clear_stale_error();
  nwm_status s = check_batch(p, batch);
  if (s != NWM_OK) return s;
  if (p->B == 0) return NWM_OK;
  if (!ws) return NWM_EINVAL;
  // the path term needs the traceback of nwm_align_batch; without a score
  // gradient only the dense term runs and tb / n_diag are not read
  if (grad_score && (!n_diag || (p->sizes.kept_cap > 0 && !tb))) return NWM_EINVAL;
  if (grad_wb && p->sizes.S_elems > 0 && (!S || !S_raw)) return NWM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const char *tbc = static_cast<const char *>(tb);
  const int2 *path = tbc ? (const int2 *)(tbc + p->dev.path_base) : nullptr;
  char *w = static_cast<char *>(ws);
  float *part_path = (float *)(w + p->ws.bwd);
  float *part_dense = part_path + 4 * (size_t)p->B;
  Mark mk(p, K_BWD, st);
  hipError_t e = launch_backward(p->dev, batch->src_off, batch->tgt_off, path, n_diag, grad_score, grad_S_extra,
                                 grad_S, grad_gap, S, S_raw, grad_wb, part_path, part_dense, st);
  mk.done();
  return dev_err(e);
}

nwm_status nwm_plan_set_param(nwm_plan *p, nwm_param param, int32_t value) {
  if (!p) return NWM_EINVAL;
  switch (param) {
    case NWM_PARAM_FILL_WAVES_PER_CU:
    case NWM_PARAM_MERGE_WAVES_PER_CU:
      if (value < 0 || value > 32) return NWM_EINVAL;
      break;
    case NWM_PARAM_SCORE_XCD_MAP:
    case NWM_PARAM_SCORE_COMPACT:
      if (value != 0 && value != 1) return NWM_EINVAL;
      break;
    case NWM_PARAM_DP_HOT_PERCENT:
      if (value < 0 || value > 100) return NWM_EINVAL;
      break;
    case NWM_PARAM_DP_SPIN_LIMIT:
      if (value < 0 || value > (1 << 30)) return NWM_EINVAL;
      break;
    case NWM_PARAM_DP_TEST_HOLD:
      if (value != 0 && value != 1) return NWM_EINVAL;
      break;
    case NWM_PARAM_SCORE_KGROUP:
      if (value != 1 && value != 2) return NWM_EINVAL;
      break;
    case NWM_PARAM_FILL_STAGING:
      if (value < 0 || value > 2) return NWM_EINVAL;
      break;
    case NWM_PARAM_EXPAND_FUSED:
      if (value != 0 && value != 1) return NWM_EINVAL;
      break;
    default:
      return NWM_EINVAL;
  }
  if (p->param[param] == value) return NWM_OK;
  p->param[param] = value;
  ++p->param_version;
  if (param == NWM_PARAM_DP_HOT_PERCENT && !p->it_strip.empty()) {
    std::vector<int32_t> words, tasks;
    hot_flags(p, words, tasks);
    if (hipSetDevice(p->device) != hipSuccess ||
        hipMemcpy(const_cast<int32_t *>(p->dev.it_strip), words.data(), 4 * words.size(), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(const_cast<int32_t *>(p->dev.tk_slot), tasks.data(), 4 * tasks.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
      return NWM_EDEVICE;
  }
  return NWM_OK;
}

nwm_status nwm_plan_get_param(const nwm_plan *p, nwm_param param, int32_t *value) {
  if (!p || !value || (int)param < 0 || (int)param >= NWM_N_PARAMS) return NWM_EINVAL;
  *value = p->param[param];
  return NWM_OK;
}

nwm_status nwm_union_kept(const nwm_plan *p, const int32_t *kept_fwd, const int32_t *n_kept_fwd,
                          const int32_t *kept_rev, const int32_t *n_kept_rev, int32_t *kept_out, int32_t *n_out,
                          void *stream) {
  if (!p) return NWM_EINVAL;
  if (p->B == 0) return NWM_OK;
  if (!n_kept_fwd || !n_kept_rev || !n_out) return NWM_EINVAL;
  clear_stale_error();
  if (p->sizes.kept_cap > 0 && (!kept_fwd || !kept_rev || !kept_out)) return NWM_EINVAL;
  return dev_err(launch_union_kept(p->B, p->dev.p_off, (const int2 *)kept_fwd, n_kept_fwd, (const int2 *)kept_rev,
                                   n_kept_rev, (int2 *)kept_out, n_out, (hipStream_t)stream));
}

nwm_status nwm_plan_set_graph(nwm_plan *p, int on) {
  if (!p) return NWM_EINVAL;
  p->graph_on = on != 0;
  if (!p->graph_on && p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
    p->graph_key.clear();
  }
  return NWM_OK;
}

// The whole path for nwm_mine.  The pairs with the longest DP dependency
// chains (first in every order of the plan) are scored first; their fill,
// walk and keep then run on the plan's second stream while the main stream
// scores and aligns the other pairs, so the long chains overlap the rest of
// the batch instead of running alone at the end.  Every kernel computes the
// same values as in nwm_score_pairs + nwm_align_batch.
static nwm_status mine_path(nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, nwm_scorer sc, float gap,
                            float threshold, float *S, float *S_raw, float *score, int32_t *n_diag, int32_t *kept,
                            int32_t *n_kept, void *tb, void *ws, hipStream_t st) {
  nwm_status s = check_score_args(p, batch, dict, sc, S, ws);
  if (s != NWM_OK) return s;
  if (!finite(gap) || !finite(threshold)) return NWM_EINVAL;
  if (p->B == 0) return NWM_OK;
  if (!score || !n_diag || !n_kept || !ws) return NWM_EINVAL;
  if (p->sizes.kept_cap > 0 && (!kept || !tb)) return NWM_EINVAL;
  char *w = static_cast<char *>(ws);
  char *tbc = static_cast<char *>(tb);
  int2 *path = tbc ? (int2 *)(tbc + p->dev.path_base) : nullptr;
  uint64_t *bnd = (uint64_t *)(w + p->ws.bnd);
  int32_t *ctl = (int32_t *)(w + p->ws.ctl);
  const int wpc = p->param[NWM_PARAM_FILL_WAVES_PER_CU];
  const int spin = p->param[NWM_PARAM_DP_SPIN_LIMIT], hold = p->param[NWM_PARAM_DP_TEST_HOLD];
  const int stg = p->param[NWM_PARAM_FILL_STAGING];
  const PlanDev &D = p->dev;
  const bool scored = p->sizes.S_elems > 0;
  const int gl = p->n_gt_long, il = p->n_items_long, ol = p->n_pairs_long;
  const int rl = p->n_rt_long, cl = p->n_ct_long, rtop = p->n_rt_top, ctop = p->n_ct_top;
  const int64_t kl = p->n_sent_long, ktop = p->n_sent_top;
  hipError_t e = ensure_streams(p);
  hipStream_t aux = p->aux_stream, lane = p->lane_stream, xs = p->exp_stream;
  if (e == hipSuccess && scored) e = pack_dict(p, dict, ws, st);
  // target-side lists on one side stream (the long pairs' first, each part
  // announced by an event), the other pairs' source-side expansion on a
  // second one, both from the start
  if (e == hipSuccess) e = hipEventRecord(p->ev_fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(aux, p->ev_fork, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(xs, p->ev_fork, 0);
  if (scored) {
    if (e == hipSuccess) e = expand_tgt(p, batch, ws, 0, ctop, true, aux);
    if (e == hipSuccess) e = hipEventRecord(p->ev_b_top, aux);
    if (e == hipSuccess) e = expand_tgt(p, batch, ws, ctop, cl - ctop, false, aux);
    if (e == hipSuccess) e = hipEventRecord(p->ev_b_long, aux);
    if (e == hipSuccess) e = expand_tgt(p, batch, ws, cl, D.n_ct - cl, false, aux);
  }
  if (e == hipSuccess) e = hipEventRecord(p->ev_b_rest, aux);
  // the other pairs' source-side expansion on the second side stream, issued
  // before any DP so that it does not queue behind one; with top pairs, only
  // once their tiles are scored (a replayed graph may put it on the main
  // stream's hardware queue, where the top pairs' contraction would wait
  // behind it)
  auto rest_src = [&]() {
    if (e == hipSuccess && scored)
      e = expand_src(p, batch, dict, ws, kl, p->n_src - kl, rl, D.n_rt - rl, p->ev_b_rest, xs);
    if (e == hipSuccess) e = hipEventRecord(p->ev_a_rest, xs);
  };
  const int gtop = p->n_gt_top, itop = p->n_items_top, otop = p->n_pairs_top;
  const int ttop = p->n_tasks_top, tl = p->n_tasks_long;
  const bool rest_after_top = ol > 0 && gtop > 0;
  if (!rest_after_top) rest_src();
  if (e == hipSuccess) e = launch_nw_reset(D, gap, score, bnd, p->n_bnd, ctl, st);
  if (ol > 0) {
    // the long pairs: expand and score on the main stream, the top pairs
    // first (their lists, then their tiles); the top pairs' DP on the lane
    // stream as soon as their tiles are scored, the other long pairs' DP
    // after theirs on the side stream that built the column tiles (four
    // streams in all, one hardware queue each), while the main stream goes
    // on with the rest
    if (scored) {
      if (e == hipSuccess) e = expand_src(p, batch, dict, ws, 0, ktop, 0, rtop, p->ev_b_top, st);
      if (e == hipSuccess) e = score_tiles(p, batch, sc, S, S_raw, ws, 0, gtop, st);
    }
    if (e == hipSuccess) e = hipEventRecord(p->ev_top, st);
    if (scored) {
      if (e == hipSuccess) e = expand_src(p, batch, dict, ws, ktop, kl - ktop, rtop, rl - rtop, p->ev_b_long, st);
      if (e == hipSuccess) e = score_tiles(p, batch, sc, S, S_raw, ws, gtop, gl - gtop, st);
    }
    if (e == hipSuccess) e = hipEventRecord(p->ev_long, st);
    if (otop > 0) {
      if (e == hipSuccess) e = hipStreamWaitEvent(lane, p->ev_top, 0);
      if (e == hipSuccess)
        e = launch_nw_fill_items(D, S, gap, score, tbc, bnd, p->n_bnd, ctl + 2, ctl + 1, 0, itop, 0, ttop, wpc, spin,
                                 hold, stg, lane);
      if (e == hipSuccess) e = launch_nw_walk(D, tbc, score, path, n_diag, 0, otop, lane);
      if (e == hipSuccess) e = launch_keep(D, S, threshold, path, n_diag, (int2 *)kept, n_kept, 0, otop, lane);
      if (e == hipSuccess) e = hipEventRecord(p->ev_top_done, lane);
    }
    if (ol > otop) {
      if (e == hipSuccess) e = hipStreamWaitEvent(aux, p->ev_long, 0);
      if (e == hipSuccess)
        e = launch_nw_fill_items(D, S, gap, score, tbc, bnd, p->n_bnd, ctl + 3, ctl + 1, itop, il - itop, ttop,
                                 tl - ttop, wpc, spin, hold, stg, aux);
      if (e == hipSuccess) e = launch_nw_walk(D, tbc, score, path, n_diag, otop, ol - otop, aux);
      if (e == hipSuccess)
        e = launch_keep(D, S, threshold, path, n_diag, (int2 *)kept, n_kept, otop, ol - otop, aux);
      if (e == hipSuccess) e = hipEventRecord(p->ev_long_done, aux);
    }
    if (rest_after_top) {   // issued last: the long pairs' work is queued first
      if (e == hipSuccess) e = hipStreamWaitEvent(xs, p->ev_top, 0);
      rest_src();
    }
  }
  if (e == hipSuccess) e = hipStreamWaitEvent(st, p->ev_a_rest, 0);
  if (e == hipSuccess) e = hipStreamWaitEvent(st, p->ev_b_rest, 0);
  if (e == hipSuccess && scored) e = score_tiles(p, batch, sc, S, S_raw, ws, gl, D.n_gt - gl, st);
  if (e == hipSuccess)
    e = launch_nw_fill_items(D, S, gap, score, tbc, bnd, p->n_bnd, ctl, ctl + 1, il, D.n_items - il, tl,
                             D.n_tasks - tl, wpc, spin, hold, stg, st);
  if (e == hipSuccess) e = launch_nw_walk(D, tbc, score, path, n_diag, ol, p->B - ol, st);
  if (e == hipSuccess) e = launch_keep(D, S, threshold, path, n_diag, (int2 *)kept, n_kept, ol, p->B - ol, st);
  if (e == hipSuccess && ol > 0 && otop > 0) e = hipStreamWaitEvent(st, p->ev_top_done, 0);
  if (e == hipSuccess && ol > otop) e = hipStreamWaitEvent(st, p->ev_long_done, 0);
  return dev_err(e);
}

nwm_status nwm_mine(nwm_plan *p, const nwm_batch *batch, const nwm_dict *dict, nwm_scorer sc, float gap,
                    float threshold, float *S, float *S_raw, float *score, int32_t *n_diag, int32_t *kept,
                    int32_t *n_kept, void *tb, void *ws, void *stream) {
  if (!p) return NWM_EINVAL;
  clear_stale_error();
  if (!p->graph_on) {
    if (p->timer.on) {
      // per-kernel timing: one kernel at a time on the caller's stream
      nwm_status s = nwm_score_pairs(p, batch, dict, sc, S, S_raw, ws, stream);
      if (s != NWM_OK) return s;
      return nwm_align_batch(p, S, gap, threshold, score, n_diag, kept, n_kept, tb, ws, stream);
    }
    return mine_path(p, batch, dict, sc, gap, threshold, S, S_raw, score, n_diag, kept, n_kept, tb, ws,
                     (hipStream_t)stream);
  }
  if (!batch || !dict) return NWM_EINVAL;
  uint32_t w0b, w1b, bb, gb, tb_;
  std::memcpy(&w0b, &sc.w0, 4);
  std::memcpy(&w1b, &sc.w1, 4);
  std::memcpy(&bb, &sc.b, 4);
  std::memcpy(&gb, &gap, 4);
  std::memcpy(&tb_, &threshold, 4);
  std::vector<uint64_t> key = {
      (uint64_t)(uintptr_t)batch->src_off, (uint64_t)(uintptr_t)batch->src_tok, (uint64_t)(uintptr_t)batch->tgt_off,
      (uint64_t)(uintptr_t)batch->tgt_tok, (uint64_t)(uintptr_t)dict->row_off,  (uint64_t)(uintptr_t)dict->col,
      (uint64_t)(uintptr_t)dict->val,      (uint64_t)dict->max_deg,             ((uint64_t)w0b << 32) | w1b,
      ((uint64_t)bb << 32) | gb,           (uint64_t)tb_,                       (uint64_t)(uintptr_t)S,
      (uint64_t)(uintptr_t)S_raw,          (uint64_t)(uintptr_t)score,          (uint64_t)(uintptr_t)n_diag,
      (uint64_t)(uintptr_t)kept,           (uint64_t)(uintptr_t)n_kept,         (uint64_t)(uintptr_t)tb,
      (uint64_t)(uintptr_t)ws,             p->param_version};
  if (!p->graph_exec || key != p->graph_key) {
    if (p->graph_exec) {
      (void)hipGraphExecDestroy(p->graph_exec);
      p->graph_exec = nullptr;
    }
    hipError_t e = hipSuccess;
    if (!p->cap_stream) e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = ensure_streams(p);
    if (e == hipSuccess) e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return dev_err(e);
    p->capturing = true;
    nwm_status s = mine_path(p, batch, dict, sc, gap, threshold, S, S_raw, score, n_diag, kept, n_kept, tb, ws,
                             p->cap_stream);
    p->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (s != NWM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess || !g) return dev_err(e != hipSuccess ? e : hipErrorUnknown);
    e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      p->graph_exec = nullptr;
      return dev_err(e);
    }
    p->graph_key = key;
  }
  return dev_err(hipGraphLaunch(p->graph_exec, (hipStream_t)stream));
}

nwm_status nwm_plan_set_timing(nwm_plan *p, int on) {
  if (!p) return NWM_EINVAL;
  p->timer.on = on != 0;
  p->timer.clear();
  return NWM_OK;
}

nwm_status nwm_plan_kernel_ms(nwm_plan *p, double ms[NWM_N_KCLASSES], int32_t counts[NWM_N_KCLASSES], int reset) {
  if (!p || !ms) return NWM_EINVAL;
  for (int k = 0; k < K_CLASSES; ++k) {
    ms[k] = 0.0;
    if (counts) counts[k] = 0;
  }
  for (auto &mk : p->timer.marks) {
    hipEvent_t a = p->timer.pool[mk.second], b = p->timer.pool[mk.second + 1];
    if (hipEventSynchronize(b) != hipSuccess) return NWM_EDEVICE;
    float t = 0.f;
    if (hipEventElapsedTime(&t, a, b) != hipSuccess) return NWM_EDEVICE;
    ms[mk.first] += t;
    if (counts) counts[mk.first] += 1;
  }
  if (reset) p->timer.clear();
  return NWM_OK;
}

}  // extern "C"
