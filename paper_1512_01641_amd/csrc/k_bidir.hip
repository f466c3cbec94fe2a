// Bi-directional mining (Sec. 5.4, Table 3 "BI"): a second classifier scores
// the same document pairs in the reverse direction (target sentences as the
// source side, a target-to-source dictionary) and the aligned pairs both
// directions keep are merged.  The merge is the union of the two kept sets,
// each sentence pair once, in ascending (i, j) order.
//
// k_union_kept  one wave per document pair.  Both inputs are strictly
//               increasing in i and in j (kept pairs lie on a monotone NW
//               path), so as 64-bit keys (i << 32 | j) both are sorted.  The
//               wave merges them 64 + 64 keys at a time: every key not above
//               the smaller of the two blocks' last keys (or every key, once
//               a block holds the rest of its list) is final in this round.
//               A key's output position is its rank in its own block plus
//               the number of final keys of the other block below it (binary
//               search over that block in LDS); a reverse key equal to a
//               forward key is dropped.  Every round retires at least one
//               whole block.
#include "nwm_internal.h"

namespace nwm {

static __device__ __forceinline__ void wave_sync_b() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Number of keys in blk[0..64) below x (blk ascending, padded with ~0).
static __device__ __forceinline__ int count_below(const uint64_t *blk, uint64_t x) {
  int lo = 0;
#pragma unroll
  for (int step = 32; step >= 1; step >>= 1)
    if (blk[lo + step - 1] < x) lo += step;
  return lo + (blk[lo] < x ? 1 : 0);   // lo <= 63 here
}

__global__ __launch_bounds__(64) void k_union_kept(int B, const int64_t *__restrict__ p_off,
                                                   const int2 *__restrict__ kept_f, const int32_t *__restrict__ n_f,
                                                   const int2 *__restrict__ kept_r, const int32_t *__restrict__ n_r,
                                                   int2 *__restrict__ out, int32_t *__restrict__ n_out) {
  __shared__ uint64_t fb[64], rb[64];
  const int b = blockIdx.x;
  if (b >= B) return;
  const int lane = threadIdx.x;
  const int64_t o = p_off[b];
  const int cap = (int)(p_off[b + 1] - o);   // min(n, m): each list holds at most this many
  const int nf = min(max(n_f[b], 0), cap), nr = min(max(n_r[b], 0), cap);
  const int2 *F = kept_f + o;
  const int2 *R = kept_r + o;     // (target index, source index): swapped on the way in
  int2 *Out = out + 2 * o;        // capacity 2 min(n, m)
  constexpr uint64_t INF = ~0ull;
  auto key = [](int i, int j) -> uint64_t { return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j; };
  int pf = 0, pr = 0, no = 0;
  while (pf < nf || pr < nr) {
    const int2 fv = pf + lane < nf ? F[pf + lane] : make_int2(0, 0);
    const int2 rv = pr + lane < nr ? R[pr + lane] : make_int2(0, 0);
    const uint64_t fk = pf + lane < nf ? key(fv.x, fv.y) : INF;
    const uint64_t rk = pr + lane < nr ? key(rv.y, rv.x) : INF;
    fb[lane] = fk;
    rb[lane] = rk;
    wave_sync_b();
    // a block that does not reach the end of its list bounds what is final
    const uint64_t flast = pf + 64 < nf ? fb[63] : INF;
    const uint64_t rlast = pr + 64 < nr ? rb[63] : INF;
    const uint64_t lim = flast < rlast ? flast : rlast;
    const bool fin_f = fk != INF && fk <= lim;
    const bool fin_r = rk != INF && rk <= lim;
    const int below_r = count_below(rb, fk);   // reverse keys < fk (all final when fk is)
    const int below_f = count_below(fb, rk);   // forward keys < rk (all final when rk is)
    const bool dup = fin_r && below_f < 64 && fb[below_f] == rk;
    const bool emit_r = fin_r && !dup;
    const uint64_t mask_r = __ballot(emit_r);
    const uint64_t mask_f = __ballot(fin_f);
    const uint64_t mask_rc = __ballot(fin_r);   // consumed reverse keys (emitted or duplicate)
    // (the bound checks only matter for inputs that are not sorted)
    if (fin_f) {
      const uint64_t m = below_r >= 64 ? mask_r : (mask_r & ((1ull << below_r) - 1ull));
      const int pos = no + lane + __popcll(m);
      if (pos < 2 * cap) Out[pos] = fv;
    }
    if (emit_r) {
      const int pos = no + below_f + __popcll(mask_r & ((1ull << lane) - 1ull));
      if (pos < 2 * cap) Out[pos] = make_int2(rv.y, rv.x);
    }
    const int cf = __popcll(mask_f), cr = __popcll(mask_rc);
    no += cf + __popcll(mask_r);
    pf += cf;
    pr += cr;
    wave_sync_b();   // the blocks are rewritten next round
  }
  if (lane == 0) n_out[b] = min(no, 2 * cap);
}

hipError_t launch_union_kept(int B, const int64_t *p_off, const int2 *kept_f, const int32_t *n_f, const int2 *kept_r,
                             const int32_t *n_r, int2 *out, int32_t *n_out, hipStream_t st) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_union_kept, dim3(B), dim3(64), 0, st, B, p_off, kept_f, n_f, kept_r, n_r, out, n_out);
  return hipGetLastError();
}

}  // namespace nwm
