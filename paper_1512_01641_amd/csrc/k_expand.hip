// Operand preparation for the similarity contraction S_raw = (X.D).Y^T
// (Sec. 4: dictionary with translation probabilities; the features are read as
// the dictionary coverage of a target sentence by a source sentence).
//
// 1. k_merge_src   one wave per source sentence: T'[i][u] = sum over the
//                  sentence's token occurrences t of D[t][u].  Duplicated
//                  targets u are merged through an LDS owner table; the sums
//                  are FP64 atomics of FP32 terms, exact (and hence independent
//                  of the order of the atomics) while the terms of one sum
//                  span fewer than 2^29 in magnitude, then rounded to FP32 once.
// 2. k_build_a     one workgroup per row tile (TM source sentences of a pair):
//                  the tile's merged entries regrouped chunk-major (K chunks of
//                  KC words), each entry pre-encoded as its LDS offset in the
//                  dense operand tile.
// 3. k_build_b     one workgroup per column tile: the distinct tokens of each
//                  target sentence (binary presence Y), regrouped the same way.
// Positions inside a chunk come from LDS atomics and vary run to run; every
// (row, word) pair occurs once per chunk, so the dense tiles built from the
// lists -- and the contraction -- do not depend on that order.
#include "nwm_internal.h"

namespace nwm {

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__global__ __launch_bounds__(64) void k_merge_src(int64_t n_sent, const int64_t *__restrict__ src_off,
                                                  const int32_t *__restrict__ src_tok,
                                                  const int32_t *__restrict__ d_row_off,
                                                  const int32_t *__restrict__ d_col,
                                                  const float *__restrict__ d_val, int V, int max_deg,
                                                  uint2 *__restrict__ merged, int32_t *__restrict__ cnt) {
  extern __shared__ __align__(16) char smem[];
  double *acc = reinterpret_cast<double *>(smem);                       // [MERGE_SLOTS]
  uint32_t *su = reinterpret_cast<uint32_t *>(acc + MERGE_SLOTS);       // [MERGE_SLOTS]
  volatile uint16_t *owner = reinterpret_cast<uint16_t *>(su + MERGE_SLOTS);  // [V]
  const int lane = threadIdx.x;
  const uint16_t EMPTY = 0xFFFF;
  for (int u = lane; u < V; u += 64) owner[u] = EMPTY;
  for (int s = lane; s < MERGE_SLOTS; s += 64) acc[s] = 0.0;
  __syncthreads();
  for (int64_t sent = blockIdx.x; sent < n_sent; sent += gridDim.x) {
    const int64_t t0 = src_off[sent], t1 = src_off[sent + 1];
    int nuniq = 0;
    for (int64_t p0 = t0; p0 < t1; p0 += 64) {
      const int64_t p = p0 + lane;
      int tok = (p < t1) ? src_tok[p] : -1;
      if ((uint32_t)tok >= (uint32_t)V) tok = -1;
      const int e0 = (tok >= 0) ? d_row_off[tok] : 0;
      int deg = (tok >= 0) ? d_row_off[tok + 1] - e0 : 0;
      if (deg > max_deg) deg = max_deg;
      for (int q = 0; q < max_deg; ++q) {
        bool act = q < deg;
        if (__ballot(act) == 0) break;
        uint32_t u = act ? (uint32_t)d_col[e0 + q] : 0u;
        const float v = act ? d_val[e0 + q] : 0.0f;
        if (u >= (uint32_t)V) act = false;
        uint16_t o = act ? owner[u] : EMPTY;
        const bool claim = act && o == EMPTY;
        const uint16_t tag = (uint16_t)(0x8000 | lane);
        if (claim) owner[u] = tag;
        wave_sync();
        const bool winner = claim && owner[u] == tag;
        const uint64_t wm = __ballot(winner);
        const int slot_w = nuniq + __popcll(wm & ((1ull << lane) - 1ull));
        const bool ok = winner && slot_w < MERGE_SLOTS;
        if (winner) owner[u] = ok ? (uint16_t)slot_w : (uint16_t)0x7FFF;
        if (ok) su[slot_w] = u;
        wave_sync();
        const uint16_t slot = act ? owner[u] : EMPTY;
        if (act && slot < MERGE_SLOTS) atomicAdd(&acc[slot], (double)v);
        nuniq += __popcll(wm);
        if (nuniq > MERGE_SLOTS) nuniq = MERGE_SLOTS;
        wave_sync();
      }
    }
    wave_sync();
    const int64_t base = t0 * (int64_t)max_deg;
    for (int s = lane; s < nuniq; s += 64) {
      merged[base + s] = make_uint2(su[s], __float_as_uint((float)acc[s]));
      acc[s] = 0.0;
      owner[su[s]] = EMPTY;
    }
    if (lane == 0) cnt[sent] = nuniq;
    wave_sync();
  }
}

// Exclusive scan of cnt[0..len) into off[0..len] by one 256-thread block.
// `tmp` holds 256 ints of LDS.
static __device__ void block_exclusive_scan(int *vals, int len, int *tmp) {
  const int tid = threadIdx.x;
  const int per = (len + 255) / 256;
  const int lo = tid * per;
  const int hi = min(lo + per, len);
  int s = 0;
  for (int k = lo; k < hi; ++k) s += vals[k];
  tmp[tid] = s;
  __syncthreads();
  for (int d = 1; d < 256; d <<= 1) {
    int x = (tid >= d) ? tmp[tid - d] : 0;
    __syncthreads();
    tmp[tid] += x;
    __syncthreads();
  }
  int run = tmp[tid] - s;
  __syncthreads();
  for (int k = lo; k < hi; ++k) {
    int c = vals[k];
    vals[k] = run;
    run += c;
  }
  if (tid == 255) vals[len] = tmp[255];
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_build_a(PlanDev P, const int64_t *__restrict__ src_off,
                                                 const uint2 *__restrict__ merged,
                                                 const int32_t *__restrict__ cnt, uint2 *__restrict__ a_list,
                                                 int32_t *__restrict__ a_choff, int pitch) {
  extern __shared__ __align__(16) char smem[];
  int *off = reinterpret_cast<int *>(smem);  // [nch + 1]
  int *tmp = off + P.nch + 1;                // [256]
  const int rt = blockIdx.x;
  const int pair = P.rt_pair[rt];
  const int rows = P.rt_rows[rt];
  const int64_t s0 = P.sfirst[pair] + P.rt_row0[rt];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = threadIdx.x; c <= P.nch; c += 256) off[c] = 0;
  __syncthreads();
  for (int r = wave; r < rows; r += 4) {
    const int64_t base = src_off[s0 + r] * (int64_t)P.max_deg;
    const int c = cnt[s0 + r];
    for (int e = lane; e < c; e += 64) atomicAdd(&off[merged[base + e].x / KC], 1);
  }
  __syncthreads();
  block_exclusive_scan(off, P.nch, tmp);
  int32_t *choff = a_choff + (int64_t)rt * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 256) choff[c] = off[c];
  __syncthreads();
  const int64_t tile_base = src_off[s0] * (int64_t)P.max_deg;
  for (int r = wave; r < rows; r += 4) {
    const int64_t base = src_off[s0 + r] * (int64_t)P.max_deg;
    const int c = cnt[s0 + r];
    for (int e = lane; e < c; e += 64) {
      const uint2 ent = merged[base + e];
      const int pos = atomicAdd(&off[ent.x / KC], 1);
      a_list[tile_base + pos] = make_uint2((uint32_t)(r * pitch + (int)(ent.x % KC)), ent.y);
    }
  }
}

__global__ __launch_bounds__(256) void k_build_b(PlanDev P, const int64_t *__restrict__ tgt_off,
                                                 const int32_t *__restrict__ tgt_tok,
                                                 uint32_t *__restrict__ b_list, int32_t *__restrict__ b_choff,
                                                 int pitch) {
  extern __shared__ __align__(16) char smem[];
  int *off = reinterpret_cast<int *>(smem);        // [nch + 1]
  int *tmp = off + P.nch + 1;                      // [256]
  uint32_t *bits = reinterpret_cast<uint32_t *>(tmp + 256);  // 4 waves x [V/32]
  const int words = (P.V + 31) / 32;
  const int ct = blockIdx.x;
  const int pair = P.ct_pair[ct];
  const int cols = P.ct_cols[ct];
  const int64_t t0 = P.tfirst[pair] + P.ct_col0[ct];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t *mybits = bits + wave * words;
  for (int c = threadIdx.x; c <= P.nch; c += 256) off[c] = 0;
  for (int w = lane; w < words; w += 64) mybits[w] = 0u;
  __syncthreads();
  // pass 1: count distinct tokens of every sentence by chunk
  for (int r = wave; r < cols; r += 4) {
    const int64_t q0 = tgt_off[t0 + r], q1 = tgt_off[t0 + r + 1];
    for (int64_t q = q0 + lane; q < q1; q += 64) {
      const uint32_t u = (uint32_t)tgt_tok[q];
      if (u < (uint32_t)P.V) {
        const uint32_t bit = 1u << (u & 31);
        if (!(atomicOr(&mybits[u >> 5], bit) & bit)) atomicAdd(&off[u / KC], 1);
      }
    }
    wave_sync();
    for (int64_t q = q0 + lane; q < q1; q += 64) {
      const uint32_t u = (uint32_t)tgt_tok[q];
      if (u < (uint32_t)P.V) mybits[u >> 5] = 0u;
    }
    wave_sync();
  }
  __syncthreads();
  block_exclusive_scan(off, P.nch, tmp);
  int32_t *choff = b_choff + (int64_t)ct * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 256) choff[c] = off[c];
  __syncthreads();
  const int64_t tile_base = tgt_off[t0];
  for (int r = wave; r < cols; r += 4) {
    const int64_t q0 = tgt_off[t0 + r], q1 = tgt_off[t0 + r + 1];
    for (int64_t q = q0 + lane; q < q1; q += 64) {
      const uint32_t u = (uint32_t)tgt_tok[q];
      if (u < (uint32_t)P.V) {
        const uint32_t bit = 1u << (u & 31);
        if (!(atomicOr(&mybits[u >> 5], bit) & bit)) {
          const int pos = atomicAdd(&off[u / KC], 1);
          b_list[tile_base + pos] = (uint32_t)(r * pitch + (int)(u % KC));
        }
      }
    }
    wave_sync();
    for (int64_t q = q0 + lane; q < q1; q += 64) {
      const uint32_t u = (uint32_t)tgt_tok[q];
      if (u < (uint32_t)P.V) mybits[u >> 5] = 0u;
    }
    wave_sync();
  }
}

// ---- launchers ----------------------------------------------------------------
hipError_t launch_merge_src(int64_t n_sent, const int64_t *src_off, const int32_t *src_tok,
                            const int32_t *d_row_off, const int32_t *d_col, const float *d_val, int V,
                            int max_deg, uint2 *merged, int32_t *cnt, hipStream_t st) {
  if (n_sent <= 0) return hipSuccess;
  const size_t lds = MERGE_SLOTS * (sizeof(double) + sizeof(uint32_t)) + sizeof(uint16_t) * (size_t)V;
  const int grid = (int)(n_sent < 65536 ? n_sent : 65536);
  hipLaunchKernelGGL(k_merge_src, dim3(grid), dim3(64), lds, st, n_sent, src_off, src_tok, d_row_off,
                     d_col, d_val, V, max_deg, merged, cnt);
  return hipGetLastError();
}

hipError_t launch_build_a(const PlanDev &P, const int64_t *src_off, const uint2 *merged, const int32_t *cnt,
                          uint2 *a_list, int32_t *a_choff, int pitch, hipStream_t st) {
  if (P.n_rt <= 0) return hipSuccess;
  const size_t lds = sizeof(int) * (size_t)(P.nch + 1 + 256);
  hipLaunchKernelGGL(k_build_a, dim3(P.n_rt), dim3(256), lds, st, P, src_off, merged, cnt, a_list, a_choff,
                     pitch);
  return hipGetLastError();
}

hipError_t launch_build_b(const PlanDev &P, const int64_t *tgt_off, const int32_t *tgt_tok, uint32_t *b_list,
                          int32_t *b_choff, int pitch, hipStream_t st) {
  if (P.n_ct <= 0) return hipSuccess;
  const size_t lds = sizeof(int) * (size_t)(P.nch + 1 + 256) + sizeof(uint32_t) * 4 * (size_t)((P.V + 31) / 32);
  hipLaunchKernelGGL(k_build_b, dim3(P.n_ct), dim3(256), lds, st, P, tgt_off, tgt_tok, b_list, b_choff, pitch);
  return hipGetLastError();
}

hipError_t merge_set_attrs(int V) {
  const size_t lds = MERGE_SLOTS * (sizeof(double) + sizeof(uint32_t)) + sizeof(uint16_t) * (size_t)V;
  return hipFuncSetAttribute((const void *)k_merge_src, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace nwm
