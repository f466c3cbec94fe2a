// Operand preparation for the similarity contraction S_raw = (X.D).Y^T
// (Sec. 4: dictionary with translation probabilities; the features are read as
// the dictionary coverage of a target sentence by a source sentence).
//
// 1. k_expand_tok  one thread per source token: its dictionary row.
//    k_merge_src   one wave per source sentence: T'[i][u] = sum over the
//                  sentence's token occurrences t of D[t][u].  Duplicated
//                  targets u are merged through an LDS owner table; the sums
//                  are FP64 atomics of FP32 terms, exact (and hence independent
//                  of the order of the atomics) while the terms of one sum
//                  span fewer than 2^29 in magnitude, then rounded to FP32 once.
// 2. k_build_a     one workgroup per row tile (TM source sentences of a pair):
//                  the tile's merged entries regrouped chunk-major (K chunks of
//                  KC words), each entry pre-encoded as its LDS byte offset in
//                  the dense operand tile.
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

// One thread per source token occurrence: its dictionary row, written at a
// fixed stride of max_deg entries {target word, weight bits} (empty slots get
// word 0xFFFFFFFF).  Fully parallel, so the token -> row -> entries chain of
// dependent loads is hidden by occupancy rather than paid per sentence.
__global__ __launch_bounds__(256) void k_expand_tok(int64_t n_tok, const int32_t *__restrict__ src_tok,
                                                    const int32_t *__restrict__ d_row_off,
                                                    const int32_t *__restrict__ d_col,
                                                    const float *__restrict__ d_val, int V, int max_deg,
                                                    uint2 *__restrict__ raw) {
  for (int64_t p = blockIdx.x * (int64_t)256 + threadIdx.x; p < n_tok; p += (int64_t)gridDim.x * 256) {
    const int tok = src_tok[p];
    int e0 = 0, deg = 0;
    if ((uint32_t)tok < (uint32_t)V) {
      e0 = d_row_off[tok];
      deg = min(d_row_off[tok + 1] - e0, max_deg);
    }
    uint2 *out = raw + p * max_deg;
    for (int q = 0; q < max_deg; ++q) {
      uint2 e = make_uint2(0xFFFFFFFFu, 0u);
      if (q < deg) {
        const uint32_t u = (uint32_t)d_col[e0 + q];
        if (u < (uint32_t)V) e = make_uint2(u, __float_as_uint(d_val[e0 + q]));
      }
      out[q] = e;
    }
  }
}

// One wave per source sentence (grid-stride): merge the sentence's
// contiguous block of dictionary entries by target word.  The first 128
// entries of the next sentence are loaded while the current one merges.
__global__ __launch_bounds__(64) void k_merge_src(int64_t n_sent, const int64_t *__restrict__ src_off,
                                                  const uint2 *__restrict__ raw, int V, int max_deg,
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

  auto fetch = [&](int64_t sent, uint2 &e0, uint2 &e1, int &ne, int64_t &base) {
    const int64_t t0 = src_off[sent], t1 = src_off[sent + 1];
    base = t0 * (int64_t)max_deg;
    ne = (int)((t1 - t0) * max_deg);
    e0 = lane < ne ? raw[base + lane] : make_uint2(0xFFFFFFFFu, 0u);
    e1 = 64 + lane < ne ? raw[base + 64 + lane] : make_uint2(0xFFFFFFFFu, 0u);
  };

  int64_t sent = blockIdx.x;
  uint2 n0 = make_uint2(0xFFFFFFFFu, 0u), n1 = n0;
  int nne = 0;
  int64_t nbase = 0;
  if (sent < n_sent) fetch(sent, n0, n1, nne, nbase);
  for (; sent < n_sent; sent += gridDim.x) {
    const uint2 c0 = n0, c1 = n1;
    const int ne = nne;
    const int64_t base = nbase;
    if (sent + gridDim.x < n_sent) fetch(sent + gridDim.x, n0, n1, nne, nbase);
    int nuniq = 0;
    for (int r0 = 0; r0 < ne; r0 += 64) {
      const uint2 e = r0 == 0 ? c0 : r0 == 64 ? c1 : (r0 + lane < ne ? raw[base + r0 + lane] : make_uint2(0xFFFFFFFFu, 0u));
      uint32_t u = e.x;
      bool act = u < (uint32_t)V;
      const float v = __uint_as_float(e.y);
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

// Rows handled by one wave of a 256-thread tile builder: w, w+4, ... (<= 16).
constexpr int ROWS_PER_WAVE = TM / 4;

__global__ __launch_bounds__(256) void k_build_a(PlanDev P, const int64_t *__restrict__ src_off,
                                                 const uint2 *__restrict__ merged,
                                                 const int32_t *__restrict__ cnt, uint2 *__restrict__ a_list,
                                                 int32_t *__restrict__ a_choff, int pitch, int esize) {
  extern __shared__ __align__(16) char smem[];
  int *off = reinterpret_cast<int *>(smem);  // [nch + 1]
  int *tmp = off + P.nch + 1;                // [256]
  const int rt = blockIdx.x;
  const int pair = P.rt_pair[rt];
  const int rows = P.rt_rows[rt];
  const int64_t s0 = P.sfirst[pair] + P.rt_row0[rt];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = threadIdx.x; c <= P.nch; c += 256) off[c] = 0;
  // every row of this wave at once: lane k fetches row wave + 4k's count and
  // base, then the first 128 entries of every row are loaded together
  const int myrow = wave + 4 * lane;
  const int rc = (lane < ROWS_PER_WAVE && myrow < rows) ? cnt[s0 + myrow] : 0;
  const int64_t rb = (lane < ROWS_PER_WAVE && myrow < rows) ? src_off[s0 + myrow] * (int64_t)P.max_deg : 0;
  uint2 e[ROWS_PER_WAVE][2];
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int c = __shfl(rc, k, 64);
    const int64_t base = __shfl(rb, k, 64);
    e[k][0] = lane < c ? merged[base + lane] : make_uint2(0xFFFFFFFFu, 0u);
    e[k][1] = 64 + lane < c ? merged[base + 64 + lane] : make_uint2(0xFFFFFFFFu, 0u);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (e[k][q].x != 0xFFFFFFFFu) atomicAdd(&off[e[k][q].x / KC], 1);
    const int c = __shfl(rc, k, 64);
    const int64_t base = __shfl(rb, k, 64);
    for (int x = 128 + lane; x < c; x += 64) atomicAdd(&off[merged[base + x].x / KC], 1);
  }
  __syncthreads();
  block_exclusive_scan(off, P.nch, tmp);
  int32_t *choff = a_choff + (int64_t)rt * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 256) choff[c] = off[c];
  __syncthreads();
  const int64_t tile_base = src_off[s0] * (int64_t)P.max_deg;
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int r = wave + 4 * k;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint2 ent = e[k][q];
      if (ent.x != 0xFFFFFFFFu) {
        const int pos = atomicAdd(&off[ent.x / KC], 1);
        a_list[tile_base + pos] = make_uint2((uint32_t)((r * pitch + (int)(ent.x % KC)) * esize), ent.y);
      }
    }
    const int c = __shfl(rc, k, 64);
    const int64_t base = __shfl(rb, k, 64);
    for (int x = 128 + lane; x < c; x += 64) {
      const uint2 ent = merged[base + x];
      const int pos = atomicAdd(&off[ent.x / KC], 1);
      a_list[tile_base + pos] = make_uint2((uint32_t)((r * pitch + (int)(ent.x % KC)) * esize), ent.y);
    }
  }
}

__global__ __launch_bounds__(256) void k_build_b(PlanDev P, const int64_t *__restrict__ tgt_off,
                                                 const int32_t *__restrict__ tgt_tok,
                                                 uint32_t *__restrict__ b_list, int32_t *__restrict__ b_choff,
                                                 int pitch, int esize) {
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
  // sentences of this wave: lane k fetches sentence wave + 4k's token range,
  // then the first 64 tokens of every sentence are loaded together
  const int mycol = wave + 4 * lane;
  const bool vk = lane < ROWS_PER_WAVE && mycol < cols;
  const int64_t q0 = vk ? tgt_off[t0 + mycol] : 0;
  const int ql = vk ? (int)(tgt_off[t0 + mycol + 1] - q0) : 0;
  uint32_t tok[ROWS_PER_WAVE];
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int64_t a = __shfl(q0, k, 64);
    const int l = __shfl(ql, k, 64);
    tok[k] = lane < l ? (uint32_t)tgt_tok[a + lane] : 0xFFFFFFFFu;
  }
  __syncthreads();
  // pass 1: distinct tokens of each sentence (first occurrence per word),
  // counted by chunk; first occurrences are remembered for pass 2
  uint32_t first = 0u;   // bit k: this lane's token of sentence k is a first occurrence
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const uint32_t u = tok[k];
    if (u < (uint32_t)P.V) {
      const uint32_t bit = 1u << (u & 31);
      if (!(atomicOr(&mybits[u >> 5], bit) & bit)) {
        first |= 1u << k;
        atomicAdd(&off[u / KC], 1);
      }
    }
    const int64_t a = __shfl(q0, k, 64);
    const int l = __shfl(ql, k, 64);
    for (int x = 64 + lane; x < l; x += 64) {   // long sentences
      const uint32_t v = (uint32_t)tgt_tok[a + x];
      if (v < (uint32_t)P.V) {
        const uint32_t bit = 1u << (v & 31);
        if (!(atomicOr(&mybits[v >> 5], bit) & bit)) atomicAdd(&off[v / KC], 1);
      }
    }
    wave_sync();
    if (u < (uint32_t)P.V) mybits[u >> 5] = 0u;
    for (int x = 64 + lane; x < l; x += 64) {
      const uint32_t v = (uint32_t)tgt_tok[a + x];
      if (v < (uint32_t)P.V) mybits[v >> 5] = 0u;
    }
    wave_sync();
  }
  __syncthreads();
  block_exclusive_scan(off, P.nch, tmp);
  int32_t *choff = b_choff + (int64_t)ct * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 256) choff[c] = off[c];
  __syncthreads();
  const int64_t tile_base = tgt_off[t0];
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int r = wave + 4 * k;
    if (first & (1u << k)) {
      const uint32_t u = tok[k];
      const int pos = atomicAdd(&off[u / KC], 1);
      b_list[tile_base + pos] = (uint32_t)((r * pitch + (int)(u % KC)) * esize);
    }
    const int64_t a = __shfl(q0, k, 64);
    const int l = __shfl(ql, k, 64);
    if (l > 64) {   // long sentences: redo the first-occurrence test
      const uint32_t u = tok[k];
      if (u < (uint32_t)P.V) atomicOr(&mybits[u >> 5], 1u << (u & 31));
      wave_sync();
      for (int x = 64 + lane; x < l; x += 64) {
        const uint32_t v = (uint32_t)tgt_tok[a + x];
        if (v < (uint32_t)P.V) {
          const uint32_t bit = 1u << (v & 31);
          if (!(atomicOr(&mybits[v >> 5], bit) & bit)) {
            const int pos = atomicAdd(&off[v / KC], 1);
            b_list[tile_base + pos] = (uint32_t)((r * pitch + (int)(v % KC)) * esize);
          }
        }
      }
      wave_sync();
      if (u < (uint32_t)P.V) mybits[u >> 5] = 0u;
      for (int x = 64 + lane; x < l; x += 64) {
        const uint32_t v = (uint32_t)tgt_tok[a + x];
        if (v < (uint32_t)P.V) mybits[v >> 5] = 0u;
      }
      wave_sync();
    }
  }
}

// ---- launchers ----------------------------------------------------------------
hipError_t launch_merge_src(int64_t n_sent, int64_t n_tok, const int64_t *src_off, const int32_t *src_tok,
                            const int32_t *d_row_off, const int32_t *d_col, const float *d_val, int V,
                            int max_deg, uint2 *raw, uint2 *merged, int32_t *cnt, hipStream_t st) {
  if (n_sent <= 0) return hipSuccess;
  if (n_tok > 0) {
    const int64_t blocks = (n_tok + 255) / 256;
    hipLaunchKernelGGL(k_expand_tok, dim3((unsigned)(blocks < 65536 ? blocks : 65536)), dim3(256), 0, st, n_tok,
                       src_tok, d_row_off, d_col, d_val, V, max_deg, raw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const size_t lds = MERGE_SLOTS * (sizeof(double) + sizeof(uint32_t)) + sizeof(uint16_t) * (size_t)V;
  const int grid = (int)(n_sent < 16384 ? n_sent : 16384);
  hipLaunchKernelGGL(k_merge_src, dim3(grid), dim3(64), lds, st, n_sent, src_off, raw, V, max_deg, merged, cnt);
  return hipGetLastError();
}

hipError_t launch_build_a(const PlanDev &P, const int64_t *src_off, const uint2 *merged, const int32_t *cnt,
                          uint2 *a_list, int32_t *a_choff, int pitch, int esize, hipStream_t st) {
  if (P.n_rt <= 0) return hipSuccess;
  const size_t lds = sizeof(int) * (size_t)(P.nch + 1 + 256);
  hipLaunchKernelGGL(k_build_a, dim3(P.n_rt), dim3(256), lds, st, P, src_off, merged, cnt, a_list, a_choff,
                     pitch, esize);
  return hipGetLastError();
}

hipError_t launch_build_b(const PlanDev &P, const int64_t *tgt_off, const int32_t *tgt_tok, uint32_t *b_list,
                          int32_t *b_choff, int pitch, int esize, hipStream_t st) {
  if (P.n_ct <= 0) return hipSuccess;
  const size_t lds = sizeof(int) * (size_t)(P.nch + 1 + 256) + sizeof(uint32_t) * 4 * (size_t)((P.V + 31) / 32);
  hipLaunchKernelGGL(k_build_b, dim3(P.n_ct), dim3(256), lds, st, P, tgt_off, tgt_tok, b_list, b_choff, pitch,
                     esize);
  return hipGetLastError();
}

hipError_t merge_set_attrs(int V) {
  const size_t lds = MERGE_SLOTS * (sizeof(double) + sizeof(uint32_t)) + sizeof(uint16_t) * (size_t)V;
  return hipFuncSetAttribute((const void *)k_merge_src, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace nwm
