// Operand preparation for the similarity contraction S_raw = (X.D).Y^T
// (Sec. 4: dictionary with translation probabilities; the features are read as
// the dictionary coverage of a target sentence by a source sentence).
//
// 1. k_merge_src   one wave per source sentence: T'[i][u] = sum over the
//                  sentence's token occurrences t of D[t][u].  Duplicated
//                  targets u are merged through a small LDS hash table; the
//                  sums are FP64 atomics of FP32 terms, exact (and hence
//                  independent of the order of the atomics) while the terms of
//                  one sum span fewer than 2^29 in magnitude, then rounded to
//                  FP32 once.
// 2. k_build_a     one workgroup per row tile (TM source sentences of a pair):
//                  the tile's merged entries regrouped chunk-major (K chunks of
//                  KC words), each entry pre-encoded as its LDS byte offset in
//                  the dense operand tile.
// 3. k_build_b     one workgroup per column tile: the distinct tokens of each
//                  target sentence (binary presence Y), regrouped the same way.
// 4. k_expand_a    1 and 2 fused (one workgroup per row tile, merged rows kept
//                  on chip), over the dictionary padded to four entries per row
//                  (k_pack_dict); used when sentences and dictionary rows are
//                  short enough (see expand_a_fits).
// Positions inside a chunk come from LDS atomics and vary run to run; every
// (row, word) pair occurs once per chunk, so the dense tiles built from the
// lists -- and the contraction -- do not depend on that order.
#include "nwm_internal.h"

#include <algorithm>

namespace nwm {

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

constexpr uint32_t HEMPTY = 0xFFFFFFFFu;

// Software pipeline of the merge over a wave's sentences.  A sentence's
// first 16 * MERGE_ROUNDS tokens are merged in rounds of 16 tokens x 4
// dictionary entries, one entry per lane: lane l of round q takes entry l % 4
// of the row of token 16 q + l / 4 (its four lanes load the same token and row
// offsets).  Every load is a vector load issued ahead of the sentence that
// needs it: the sentence id five sentences ahead, its token range four ahead,
// its tokens three ahead, their dictionary row offsets two ahead and the
// entries one ahead, so each load has a whole sentence of merging to land.  (Scalar loads would share their wait
// counter with the LDS atomics of the merge and be waited for at the first
// of them.)  The pipelined loads are unconditional: raw buffer loads with an
// offset past the buffer for lanes with nothing to load (they read 0), or
// loads at an in-range address, so the wait counts stay exact; validity is
// applied when a value is used.  A merged row leaves the LDS table into
// registers and is stored at the start of the next sentence by unconditional
// buffer stores whose range check drops the lanes past the row's end, so the
// next wait for the pipelined loads never waits for these stores.
constexpr int MERGE_OUT_REGS = 4;   // merged entries per lane held for the deferred store
constexpr int MERGE_ROUNDS = 3;     // pipelined rounds of 16 tokens
typedef unsigned int m_u32x2 __attribute__((ext_vector_type(2)));

struct MergeId {
  int64_t sent;   // sentence number within the launch (>= n_sent: none)
  m_u32x2 id;     // sent_ids[sent] as loaded
};
struct MergeOff {
  int64_t sent, id;
  m_u32x2 t0, t1;   // the sentence's token range, as loaded
};
struct MergeTok {
  int64_t id, t0;
  int len;
  int tok[MERGE_ROUNDS];   // the lane's token in each round
};
struct MergeRow {
  int64_t id, t0;
  int len;
  int e0[MERGE_ROUNDS], e1[MERGE_ROUNDS];   // its row [e0, e1) (e1 = e0 if none)
};
struct MergeEnt {
  int64_t id, t0;
  int len;
  int e0[MERGE_ROUNDS], deg[MERGE_ROUNDS];
  uint32_t u[MERGE_ROUNDS];   // the lane's entry (valid if lane % 4 < deg)
  float v[MERGE_ROUNDS];
};
struct MergeOut {
  int64_t base, id;
  int n;   // merged entries (-1: nothing to store)
  uint2 v[MERGE_OUT_REGS];
};
constexpr uint32_t BUF_OOB = 0xFFFFFFF0u;

static __device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

static __device__ __forceinline__ int64_t first_lane64(int64_t x) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A wave's merge table in LDS: 2^hbits slots of (word, FP64 sum), and the
// slots claimed by the current sentence in claim order (at most half the
// slots, which the plan's bound on tokens x degree never exceeds).
struct MergeTable {
  double *acc;
  uint32_t *key;
  int *slots;
  int hbits;
};

// One dictionary entry (u, v) per lane into the table (a lane with u >= V
// has none): open addressing with linear probing; the FP32 term is added to
// the slot's FP64 sum.  Words new to the table take the next slot numbers in
// lane order; nuniq counts them (wave-uniform).  A full table drops entries.
static __device__ __forceinline__ void table_insert(const MergeTable &T, int V, uint32_t u, float v, int lane,
                                                    int &nuniq) {
  const int HS = 1 << T.hbits, CAPU = HS >> 1;
  const bool act = u < (uint32_t)V;
  uint32_t h = act ? (u * 0x9E3779B1u) >> (32 - T.hbits) : 0u;
  bool pending = act, claimed = false, placed = false;
  int probes = 0;
  while (__ballot(pending) != 0) {
    if (pending) {
      const uint32_t old = atomicCAS(&T.key[h], HEMPTY, u);
      if (old == HEMPTY || old == u) {
        claimed = old == HEMPTY;
        placed = true;
        pending = false;
      } else if (++probes >= HS) {
        pending = false;   // table full: drop
      } else {
        h = (h + 1) & (uint32_t)(HS - 1);
      }
    }
  }
  if (placed) atomicAdd(&T.acc[h], (double)v);
  const uint64_t cm = __ballot(claimed);
  const int rank = nuniq + (int)__popcll(cm & ((1ull << lane) - 1ull));
  if (claimed && rank < CAPU) T.slots[rank] = (int)h;
  nuniq = min(nuniq + (int)__popcll(cm), CAPU);
}

// One wave per source sentence (grid-stride): T'[i][u] = sum over the
// sentence's tokens t of D[t][u], merged by target word u through an LDS
// hash table of 2^hbits slots (open addressing, linear probing, at most half
// full by the plan's bound on tokens x degree).  The sums are FP64 LDS atomics
// of FP32 terms -- exact, so independent of the order of the atomics --
// rounded to FP32 once on the way out.  A sentence longer than the caller's
// max_sent_tokens (a contract violation) cannot hang or write out of bounds:
// a full table or slot list drops entries.
__global__ __launch_bounds__(64) void k_merge_src(int64_t n_sent, const int64_t *__restrict__ sent_ids,
                                                  const int64_t *__restrict__ src_off,
                                                  const int32_t *__restrict__ src_tok,
                                                  const int32_t *__restrict__ d_row_off,
                                                  const int32_t *__restrict__ d_col, const float *__restrict__ d_val,
                                                  int V, int max_deg, int hbits, uint2 *__restrict__ merged,
                                                  int32_t *__restrict__ cnt) {
  extern __shared__ __align__(16) char smem[];
  const int HS = 1 << hbits;
  const int CAPU = HS >> 1;                                  // distinct words per sentence
  double *acc = reinterpret_cast<double *>(smem);            // [HS]
  uint32_t *key = reinterpret_cast<uint32_t *>(acc + HS);    // [HS]
  int *slots = reinterpret_cast<int *>(key + HS);            // [CAPU] claimed slots, claim order
  const int lane = threadIdx.x;
  for (int h = lane; h < HS; h += 64) {
    key[h] = HEMPTY;
    acc[h] = 0.0;
  }
  wave_sync();

  const int nnz = d_row_off[V];   // dictionary entries
  const __amdgpu_buffer_rsrc_t r_ids =
      __builtin_amdgcn_make_buffer_rsrc((void *)sent_ids, (short)0, (int)(n_sent * 8), 0x00020000);
  const __amdgpu_buffer_rsrc_t r_row =
      __builtin_amdgcn_make_buffer_rsrc((void *)d_row_off, (short)0, (V + 1) * 4, 0x00020000);
  const __amdgpu_buffer_rsrc_t r_col = __builtin_amdgcn_make_buffer_rsrc((void *)d_col, (short)0, nnz * 4, 0x00020000);
  const __amdgpu_buffer_rsrc_t r_val = __builtin_amdgcn_make_buffer_rsrc((void *)d_val, (short)0, nnz * 4, 0x00020000);

  // sentence number `sent` of this launch is sentence sent_ids[sent]
  auto load_id = [&](int64_t sent) {
    MergeId I;
    I.sent = sent;
    I.id = __builtin_amdgcn_raw_buffer_load_b64(r_ids, sent < n_sent ? (uint32_t)sent * 8u : BUF_OOB, 0, 0);
    return I;
  };
  // (a buffer load, not a plain one: the compiler would turn a load at a
  // wave-uniform address into a scalar load)
  auto load_off = [&](const MergeId &I) {
    MergeOff O;
    O.sent = I.sent;
    O.id = first_lane64((int64_t)(((uint64_t)I.id.y << 32) | I.id.x));   // 0 past the launch: a valid index
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)(src_off + O.id), (short)0, 16, 0x00020000);
    O.t0 = __builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0);
    O.t1 = __builtin_amdgcn_raw_buffer_load_b64(r, 8u, 0, 0);
    return O;
  };
  auto load_tok = [&](const MergeOff &O) {
    MergeTok T;
    T.id = O.id;
    T.t0 = first_lane64((int64_t)(((uint64_t)O.t0.y << 32) | O.t0.x));
    const int64_t t1 = first_lane64((int64_t)(((uint64_t)O.t1.y << 32) | O.t1.x));
    T.len = O.sent < n_sent ? (int)max(t1 - T.t0, (int64_t)0) : 0;
    // a buffer over this sentence's first 16 * MERGE_ROUNDS tokens
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(src_tok + T.t0), (short)0, min(T.len, 16 * MERGE_ROUNDS) * 4, 0x00020000);
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) T.tok[q] = (int)buf_u32(r, (uint32_t)(16 * q + (lane >> 2)) * 4u);
    return T;
  };
  auto load_row = [&](const MergeTok &T) {
    MergeRow R;
    R.id = T.id;
    R.t0 = T.t0;
    R.len = T.len;
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) {
      const bool ok = 16 * q + (lane >> 2) < T.len && (unsigned)T.tok[q] < (unsigned)V;
      const uint32_t off = ok ? (uint32_t)T.tok[q] * 4u : BUF_OOB;
      R.e0[q] = (int)buf_u32(r_row, off);
      R.e1[q] = (int)buf_u32(r_row, ok ? off + 4u : BUF_OOB);
    }
    return R;
  };
  auto load_ent = [&](const MergeRow &R) {
    MergeEnt E;
    E.id = R.id;
    E.t0 = R.t0;
    E.len = R.len;
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) {
      E.e0[q] = R.e0[q];
      E.deg[q] = max(0, min(R.e1[q] - R.e0[q], max_deg));
      const uint32_t off = (lane & 3) < E.deg[q] ? (uint32_t)(E.e0[q] + (lane & 3)) * 4u : BUF_OOB;
      E.u[q] = buf_u32(r_col, off);
      E.v[q] = __uint_as_float(buf_u32(r_val, off));
    }
    return E;
  };
  // the merged row held in registers and the count; lanes past the row's end
  // (and every lane of an empty record) fall outside the buffer ranges
  // (base, id and n are wave-uniform; stating it keeps the resources scalar)
  auto store_out = [&](const MergeOut &M) {
    const int n_rec = __builtin_amdgcn_readfirstlane(M.n);
    const int n = max(n_rec, 0);
    const int64_t id = first_lane64(M.id);
    const __amdgpu_buffer_rsrc_t r_m =
        __builtin_amdgcn_make_buffer_rsrc((void *)(merged + first_lane64(M.base)), (short)0, n * 8, 0x00020000);
#pragma unroll
    for (int r = 0; r < MERGE_OUT_REGS; ++r)
      __builtin_amdgcn_raw_buffer_store_b64((m_u32x2){M.v[r].x, M.v[r].y}, r_m, (uint32_t)(lane + 64 * r) * 8u, 0,
                                            0);
    const __amdgpu_buffer_rsrc_t r_c =
        __builtin_amdgcn_make_buffer_rsrc((void *)(cnt + id), (short)0, n_rec >= 0 ? 4 : 0, 0x00020000);
    __builtin_amdgcn_raw_buffer_store_b32(n_rec, r_c, (uint32_t)lane * 4u, 0, 0);
  };

  int nuniq = 0;
  const MergeTable tab{acc, key, slots, hbits};
  auto insert = [&](uint32_t u, float v) { table_insert(tab, V, u, v, lane, nuniq); };

  const int64_t G = gridDim.x;
  int64_t sent = blockIdx.x;
  MergeEnt E = load_ent(load_row(load_tok(load_off(load_id(sent)))));
  MergeRow R = load_row(load_tok(load_off(load_id(sent + G))));
  MergeTok T = load_tok(load_off(load_id(sent + 2 * G)));
  MergeOff O = load_off(load_id(sent + 3 * G));
  MergeId I = load_id(sent + 4 * G);
  MergeOut out;
  out.base = out.id = 0;
  out.n = -1;
#pragma unroll
  for (int r = 0; r < MERGE_OUT_REGS; ++r) out.v[r] = make_uint2(0u, 0u);
  for (; sent < n_sent; sent += G) {
    const MergeEnt cur = E;
    E = load_ent(R);
    R = load_row(T);
    T = load_tok(O);
    O = load_off(I);
    I = load_id(sent + 5 * G);
    store_out(out);   // the previous sentence's row

    nuniq = 0;
    // first 16 * MERGE_ROUNDS tokens: four entries of every row loaded ahead,
    // further entries (rows longer than four) here
    const int rounds = min((cur.len + 15) >> 4, MERGE_ROUNDS);
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) {
      if (q >= rounds) break;
      insert((lane & 3) < cur.deg[q] ? cur.u[q] : HEMPTY, cur.v[q]);
      if (max_deg > 4) {
        for (int d = 4 + (lane & 3);; d += 4) {
          if (__ballot(d < cur.deg[q]) == 0) break;
          uint32_t u = HEMPTY;
          float v = 0.0f;
          if (d < cur.deg[q]) {
            u = (uint32_t)d_col[cur.e0[q] + d];
            v = d_val[cur.e0[q] + d];
          }
          insert(u, v);
        }
      }
    }
    // tokens past those (long sentences), one per lane
    for (int c0 = 16 * MERGE_ROUNDS; c0 < cur.len; c0 += 64) {
      int e0 = 0, deg = 0;
      if (c0 + lane < cur.len) {
        const int tok = src_tok[cur.t0 + c0 + lane];
        if ((unsigned)tok < (unsigned)V) {
          e0 = d_row_off[tok];
          deg = min(d_row_off[tok + 1] - e0, max_deg);
        }
      }
      for (int q = 0; q < max_deg; ++q) {
        if (__ballot(q < deg) == 0) break;
        uint32_t u = HEMPTY;
        float v = 0.0f;
        if (q < deg) {
          u = (uint32_t)d_col[e0 + q];
          v = d_val[e0 + q];
        }
        insert(u, v);
      }
    }
    wave_sync();
    // take the merged row out of the table and clear every slot this
    // sentence claimed (a dropped entry claimed none); each claimed slot
    // belongs to one lane.  Entries past the registers' share are stored here.
    out.base = cur.t0 * (int64_t)max_deg;
    out.id = cur.id;
    out.n = nuniq;
#pragma unroll
    for (int r = 0; r < MERGE_OUT_REGS; ++r) {
      const int e = lane + 64 * r;
      uint2 v = make_uint2(0u, 0u);
      if (e < nuniq) {
        const int h = slots[e];
        v = make_uint2(key[h], __float_as_uint((float)acc[h]));
        key[h] = HEMPTY;
        acc[h] = 0.0;
      }
      out.v[r] = v;
    }
    for (int e = 64 * MERGE_OUT_REGS + lane; e < nuniq; e += 64) {
      const int h = slots[e];
      merged[out.base + e] = make_uint2(key[h], __float_as_uint((float)acc[h]));
      key[h] = HEMPTY;
      acc[h] = 0.0;
    }
    wave_sync();
  }
  store_out(out);
}

// Exclusive scan of vals[0..len) in place, total in vals[len], by the first
// wave of a 256-thread block (each lane sums a run of consecutive entries,
// a wave-wide scan of the run sums, each lane writes its run back); the
// caller has synchronised the block after writing vals.  `tmp` is unused.
static __device__ void block_exclusive_scan(int *vals, int len, int *tmp) {
  (void)tmp;
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    const int per = (len + 63) / 64;
    const int lo = min(lane * per, len);
    const int hi = min(lo + per, len);
    int sum = 0;
    for (int k = lo; k < hi; ++k) sum += vals[k];
    int incl = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int x = __shfl_up(incl, d, 64);
      if (lane >= d) incl += x;
    }
    int run = incl - sum;
    for (int k = lo; k < hi; ++k) {
      const int c = vals[k];
      vals[k] = run;
      run += c;
    }
    if (lane == 63) vals[len] = incl;
  }
  __syncthreads();
}

// Rows handled by one wave of a 256-thread tile builder: w, w+4, ... (<= 16).
constexpr int ROWS_PER_WAVE = TM / 4;

// Entry encoding: dense contraction -- the LDS byte offset of (row, word %
// KC) in the operand tile; compacted contraction (compact != 0) -- word << 6 |
// row, placed by the contraction once it knows the column tile's vocabulary.
static __device__ __forceinline__ uint32_t a_code(uint32_t u, int r, int pitch, int esize, int compact) {
  return compact ? (u << 6) | (uint32_t)r : (uint32_t)((r * pitch + (int)(u % KC)) * esize);
}

// Entry value: the FP32 term, except for the compacted BF16 contraction,
// which gets the row's byte offset in the operand tile in the high half and
// the BF16 operand (the same conversion the dense path does) in the low half.
static __device__ __forceinline__ uint32_t a_val(uint32_t v, int r, int pitch, int esize, int compact) {
  if (!(compact && esize == 2)) return v;
  const __bf16 h = (__bf16)__uint_as_float(v);
  return ((uint32_t)(r * pitch * 2) << 16) | (uint32_t)__builtin_bit_cast(uint16_t, h);
}

__global__ __launch_bounds__(256) void k_build_a(PlanDev P, const int64_t *__restrict__ src_off,
                                                 const uint2 *__restrict__ merged,
                                                 const int32_t *__restrict__ cnt, uint2 *__restrict__ a_list,
                                                 int32_t *__restrict__ a_choff, int pitch, int esize, int compact,
                                                 int64_t *__restrict__ a_base, const uint32_t *__restrict__ p_voc,
                                                 int r0) {
  extern __shared__ __align__(16) char smem[];
  int *off = reinterpret_cast<int *>(smem);  // [nch + 1]
  int *tmp = off + P.nch + 1;                // [256]
  uint32_t *voc = reinterpret_cast<uint32_t *>(tmp + 256);   // [nch] (with p_voc)
  const int rt = r0 + (int)blockIdx.x;
  const TileMeta tm = P.rt_meta[rt];
  const int rows = tm.count;
  const int64_t s0 = tm.first;
  // with p_voc: the pair's target vocabulary (one bit per word, KC words per
  // chunk); an entry whose word no target sentence of the pair holds meets a
  // zero in every column of every tile of the pair and is left out
  if (p_voc)
    for (int w = threadIdx.x; w < P.nch; w += 256) voc[w] = p_voc[(int64_t)tm.pair * P.nch + w];
  // issued with the rows' counts, used for the placement
  const int64_t tile_base = src_off[s0] * (int64_t)P.max_deg;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int c = threadIdx.x; c <= P.nch; c += 256) off[c] = 0;
  // every row of this wave at once: lane k fetches row wave + 4k's count and
  // base (rows past the tile read row 0 and count 0), then the first 128
  // entries of every row are loaded together by unconditional buffer loads
  // (entries past a row's count fall outside its buffer range)
  const int myrow = wave + 4 * lane;
  const bool vrow = lane < ROWS_PER_WAVE && myrow < rows;
  const int64_t srow = s0 + (vrow ? myrow : 0);
  const int rc_ld = cnt[srow];
  const int64_t rb = src_off[srow] * (int64_t)P.max_deg;
  const int rc = vrow ? rc_ld : 0;
  auto row_cnt = [&](int k) { return __builtin_amdgcn_readlane(rc, k); };
  auto row_base = [&](int k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)rb, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)rb >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  uint2 e[ROWS_PER_WAVE][2];
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(merged + row_base(k)), (short)0, min(row_cnt(k), 128) * 8, 0x00020000);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const m_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (uint32_t)(64 * q + lane) * 8u, 0, 0);
      e[k][q] = make_uint2(v.x, v.y);
    }
  }
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k)
#pragma unroll
    for (int q = 0; q < 2; ++q)
      if (64 * q + lane >= row_cnt(k)) e[k][q].x = 0xFFFFFFFFu;
  __syncthreads();
  auto in_voc = [&](uint32_t u) { return p_voc == nullptr || ((voc[u / KC] >> (u % KC)) & 1u) != 0u; };
  if (p_voc) {
#pragma unroll
    for (int k = 0; k < ROWS_PER_WAVE; ++k)
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint32_t u = e[k][q].x;
        if (u != 0xFFFFFFFFu && !in_voc(u)) e[k][q].x = 0xFFFFFFFFu;
      }
  }
  // masked-off entries count into the lane's own slot past the table
  // (tmp[lane]: never read), so the atomics need no branches
  const int junk = P.nch + 1 + lane;
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t u = e[k][q].x;
      atomicAdd(&off[u != 0xFFFFFFFFu ? (int)(u / KC) : junk], 1);
    }
    const int c = row_cnt(k);
    const int64_t base = row_base(k);
    for (int x = 128 + lane; x < c; x += 64) {
      const uint32_t u = merged[base + x].x;
      if (in_voc(u)) atomicAdd(&off[u / KC], 1);
    }
  }
  __syncthreads();
  block_exclusive_scan(off, P.nch, tmp);
  int32_t *choff = a_choff + (int64_t)rt * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 256) choff[c] = off[c];
  const int total = __builtin_amdgcn_readfirstlane(off[P.nch]);   // entries of the tile (wave-uniform)
  __syncthreads();
  if (threadIdx.x == 0) a_base[rt] = tile_base;
  // placement: every position is taken first, then every entry is stored by
  // an unconditional buffer store (masked-off entries at an offset past the
  // tile's range)
  const __amdgpu_buffer_rsrc_t r_out =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a_list + tile_base), (short)0, total * 8, 0x00020000);
  int pos[ROWS_PER_WAVE][2];
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t u = e[k][q].x;
      pos[k][q] = atomicAdd(&off[u != 0xFFFFFFFFu ? (int)(u / KC) : junk], 1);
    }
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int r = wave + 4 * k;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint2 ent = e[k][q];
      const bool ok = ent.x != 0xFFFFFFFFu;
      __builtin_amdgcn_raw_buffer_store_b64(
          (m_u32x2){a_code(ok ? ent.x : 0u, r, pitch, esize, compact), a_val(ent.y, r, pitch, esize, compact)}, r_out,
          ok ? (uint32_t)pos[k][q] * 8u : BUF_OOB, 0, 0);
    }
  }
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int r = wave + 4 * k;
    const int c = row_cnt(k);
    const int64_t base = row_base(k);
    for (int x = 128 + lane; x < c; x += 64) {
      const uint2 ent = merged[base + x];
      if (in_voc(ent.x)) {
        const int p = atomicAdd(&off[ent.x / KC], 1);
        a_list[tile_base + p] =
            make_uint2(a_code(ent.x, r, pitch, esize, compact), a_val(ent.y, r, pitch, esize, compact));
      }
    }
  }
}

// Fused source-side expansion: the merge and the row-tile list builder in one
// kernel, so merged rows never leave the chip.  One workgroup of EXA_WAVES
// waves per row tile; wave w merges the tile's rows w, w + EXA_WAVES, ...
// (EXA_SENT of them) in its own LDS table of (word, FP64 sum) slots: the same
// sums as k_merge_src's (exact FP64 sums of the FP32 terms, rounded to FP32
// once).  A row's entries sit three per lane (token 16 q + l / 4, entry l % 4
// of its dictionary row, for q < 3): the three compare-and-swaps of a probe go
// out together, the lane whose swap claimed a slot owns that word, every
// entry adds its term to its word's slot, and each owner reads its sum back
// and clears the slot -- about two LDS round trips per row, and the merged
// row stays where the owners are (an entry per owner, holes elsewhere).  The
// loads of all of a wave's rows go out stage by stage (token ranges, tokens,
// padded dictionary entries: three dependent rounds per wave).  Then
// the workgroup counts the entries per K chunk, scans the counts and places
// every entry, as k_build_a does.  Requires sentences of at most
// 16 * MERGE_ROUNDS tokens and dictionary rows of at most 4 entries (the plan
// checks); tokens past that bound (a broken contract) are ignored.  There is
// no pair-vocabulary filter: an entry whose word no column tile holds is
// skipped by the contraction's own lookup.
constexpr int EXA_WAVES = 8;
constexpr int EXA_SENT = TM / EXA_WAVES;   // rows per wave

// Per wave: acc [HS + 64] (FP64) and key [HS + 64]; slot HS + l is lane l's
// junk slot (never matched).  Only the keys need clearing: an owner writes
// its slot's sum before any other term is added.
static __host__ __device__ inline size_t expand_a_wave_bytes(int hbits) {
  return (((size_t)1 << hbits) + 64) * (sizeof(double) + sizeof(uint32_t));
}

// Merge state of one entry of a row, in one register: its probe slot (below
// HS) while it probes; HS + lane (the lane's junk slot) when it has no slot
// (no entry, or dropped by a full table); its final slot with EXA_OWN (it
// claimed the slot) or EXA_JOIN (the slot already held its word) set.
constexpr uint32_t EXA_OWN = 1u << 30, EXA_JOIN = 1u << 29, EXA_SLOT = EXA_JOIN - 1u;

// The NQ compare-and-swaps of one probe round (entry q: word w[q] into slot
// h[q] if it is free; an entry that is not probing swaps its lane's junk slot
// with itself), issued back to back and waited for together -- written as
// asm because the compiler waits for each before issuing the next.  old[q]
// is what the slot held.
template <int NQ>
static __device__ __forceinline__ void cas_round(uint32_t (&old)[NQ], uint32_t base, const uint32_t (&h)[NQ],
                                                 uint32_t HS, uint32_t junk, const uint32_t (&w)[MERGE_ROUNDS]) {
  uint32_t a[NQ], v[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const bool probing = h[q] < HS;
    a[q] = base + 4u * (probing ? h[q] : junk);
    v[q] = probing ? w[q] : HEMPTY;
  }
  if constexpr (NQ == 1) {
    asm volatile("ds_cmpst_rtn_b32 %0, %1, %2, %3\n\ts_waitcnt lgkmcnt(0)"
                 : "=&v"(old[0])
                 : "v"(a[0]), "v"(HEMPTY), "v"(v[0])
                 : "memory");
  } else if constexpr (NQ == 2) {
    asm volatile(
        "ds_cmpst_rtn_b32 %0, %2, %4, %5\n\t"
        "ds_cmpst_rtn_b32 %1, %3, %4, %6\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(old[0]), "=&v"(old[1])
        : "v"(a[0]), "v"(a[1]), "v"(HEMPTY), "v"(v[0]), "v"(v[1])
        : "memory");
  } else {
    static_assert(NQ == 3, "at most three entries per lane");
    asm volatile(
        "ds_cmpst_rtn_b32 %0, %3, %6, %7\n\t"
        "ds_cmpst_rtn_b32 %1, %4, %6, %8\n\t"
        "ds_cmpst_rtn_b32 %2, %5, %6, %9\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(old[0]), "=&v"(old[1]), "=&v"(old[2])
        : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(HEMPTY), "v"(v[0]), "v"(v[1]), "v"(v[2])
        : "memory");
  }
}

// Merge one row whose entries sit in the first NQ of the lane's registers
// (the others hold none) through the wave's table, which it leaves clear;
// out[q] = {word, FP32 sum} for the entries that own their word, word
// HEMPTY elsewhere.
template <int NQ>
static __device__ __forceinline__ void merge_row(uint32_t *key, double *acc, int hbits, int V, int lane,
                                                 const uint32_t (&u)[MERGE_ROUNDS], const float (&v)[MERGE_ROUNDS],
                                                 uint2 (&out)[MERGE_ROUNDS]) {
  const uint32_t HS = 1u << hbits, mask = HS - 1u, junk = HS + (uint32_t)lane;
  const uint32_t base = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void *)key;
  uint32_t h[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) h[q] = u[q] < (uint32_t)V ? (__umul24(u[q], 0x9E3779u) >> (24 - hbits)) & mask : junk;
  // probe rounds: a free slot is claimed, a slot holding the word is joined,
  // another word moves the entry on (linear probing); after HS rounds the
  // table is full and the entries still probing are dropped
  for (uint32_t round = 0;; ++round) {
    bool probing = false;
#pragma unroll
    for (int q = 0; q < NQ; ++q) probing = probing | (h[q] < HS);
    if (__ballot(probing) == 0) break;
    if (round >= HS) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) h[q] = h[q] < HS ? junk : h[q];
      break;
    }
    uint32_t old[NQ];
    cas_round<NQ>(old, base, h, HS, junk, u);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const bool free_slot = old[q] == HEMPTY;
      const bool hit = free_slot | (old[q] == u[q]);
      const uint32_t done = h[q] | (free_slot ? EXA_OWN : EXA_JOIN);
      const uint32_t next = (h[q] + 1u) & mask;
      h[q] = h[q] < HS ? (hit ? done : next) : h[q];
    }
  }
  // each owner starts its word's sum with its own term, then the entries
  // that joined add theirs (FP64 atomics, only where a word repeats); the
  // owners read the sums back (every term has landed: LDS operations of a
  // wave complete in order) and free their slots
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (h[q] & EXA_OWN) acc[h[q] & EXA_SLOT] = (double)v[q];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (h[q] & EXA_JOIN) atomicAdd(&acc[h[q] & EXA_SLOT], (double)v[q]);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    uint2 o = make_uint2(HEMPTY, 0u);
    if (h[q] & EXA_OWN) {
      const uint32_t sl = h[q] & EXA_SLOT;
      o = make_uint2(u[q], __float_as_uint((float)acc[sl]));
      key[sl] = HEMPTY;
    }
    out[q] = o;
  }
#pragma unroll
  for (int q = NQ; q < MERGE_ROUNDS; ++q) out[q] = make_uint2(HEMPTY, 0u);
}

size_t expand_a_lds_bytes(int hbits, int nch) {
  return EXA_WAVES * expand_a_wave_bytes(hbits) + sizeof(int) * (size_t)(nch + 1 + 64);
}

__global__ __launch_bounds__(64 * EXA_WAVES) void k_expand_a(PlanDev P, const int64_t *__restrict__ src_off,
                                                             const int32_t *__restrict__ src_tok,
                                                             const uint2 *__restrict__ dpk, int V, int hbits,
                                                             uint2 *__restrict__ a_list,
                                                             int32_t *__restrict__ a_choff, int pitch, int esize,
                                                             int compact, int64_t *__restrict__ a_base, int r0) {
  extern __shared__ __align__(16) char smem[];
  const int HS = 1 << hbits;
  const size_t per_wave = expand_a_wave_bytes(hbits);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *acc = reinterpret_cast<double *>(smem + wave * per_wave);   // [HS + 64]
  uint32_t *key = reinterpret_cast<uint32_t *>(acc + HS + 64);        // [HS + 64]
  int *off = reinterpret_cast<int *>(smem + EXA_WAVES * per_wave);    // [nch + 1], then 64 junk slots
  const int rt = r0 + (int)blockIdx.x;
  const TileMeta tm = P.rt_meta[rt];
  const int rows = tm.count;
  const int64_t s0 = tm.first;
  const int64_t tile_base = src_off[s0] * (int64_t)P.max_deg;
  for (int h = lane; h < HS + 64; h += 64) key[h] = HEMPTY;
  for (int c = threadIdx.x; c < P.nch + 1 + 64; c += 64 * EXA_WAVES) off[c] = 0;

  // stage 1: lane k (< EXA_SENT) holds row wave + EXA_WAVES k's token range
  const int myrow = wave + EXA_WAVES * lane;
  const bool vrow = lane < EXA_SENT && myrow < rows;
  const int64_t srow = s0 + (vrow ? myrow : 0);
  const int64_t q0 = src_off[srow];
  const int qlen = vrow ? (int)min(src_off[srow + 1] - q0, (int64_t)(16 * MERGE_ROUNDS)) : 0;
  const __amdgpu_buffer_rsrc_t r_dpk = __builtin_amdgcn_make_buffer_rsrc((void *)dpk, (short)0, V * 32, 0x00020000);
  int len[EXA_SENT];
  // stage 2: tokens (lane l of round q: token 16 q + l / 4 of the row)
  int tok[EXA_SENT][MERGE_ROUNDS];
#pragma unroll
  for (int k = 0; k < EXA_SENT; ++k) {
    len[k] = __builtin_amdgcn_readlane(qlen, k);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)q0, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)q0 >> 32), k);
    const int64_t t0 = (int64_t)(((uint64_t)hi << 32) | lo);
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc((void *)(src_tok + t0), (short)0, len[k] * 4, 0x00020000);
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) tok[k][q] = (int)buf_u32(r, (uint32_t)(16 * q + (lane >> 2)) * 4u);
  }
  // stage 3: the entries, from the padded dictionary (lane l: entry l % 4
  // of its token's row; padding and missing tokens read word HEMPTY)
  uint32_t eu[EXA_SENT][MERGE_ROUNDS];
  float ev[EXA_SENT][MERGE_ROUNDS];
#pragma unroll
  for (int k = 0; k < EXA_SENT; ++k)
#pragma unroll
    for (int q = 0; q < MERGE_ROUNDS; ++q) {
      const bool ok = 16 * q + (lane >> 2) < len[k] && (unsigned)tok[k][q] < (unsigned)V;
      const m_u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(
          r_dpk, ok ? ((uint32_t)tok[k][q] * 4u + (uint32_t)(lane & 3)) * 8u : BUF_OOB, 0, 0);
      eu[k][q] = ok ? x.x : HEMPTY;
      ev[k][q] = __uint_as_float(x.y);
    }
  wave_sync();   // the table is clear
  // merge row by row (a row of at most 16 q tokens needs only q of the
  // lane's entries); the merged row stays in registers
  uint2 out[EXA_SENT][MERGE_ROUNDS];
#pragma unroll
  for (int k = 0; k < EXA_SENT; ++k) {
    const int rounds = (len[k] + 15) >> 4;
    if (rounds <= 1) merge_row<1>(key, acc, hbits, V, lane, eu[k], ev[k], out[k]);
    else if (rounds == 2) merge_row<2>(key, acc, hbits, V, lane, eu[k], ev[k], out[k]);
    else merge_row<3>(key, acc, hbits, V, lane, eu[k], ev[k], out[k]);
  }

  // count per K chunk (lanes without an entry count into their own junk slot)
  __syncthreads();
  const int junk = P.nch + 1 + lane;
#pragma unroll
  for (int k = 0; k < EXA_SENT; ++k)
#pragma unroll
    for (int r = 0; r < MERGE_ROUNDS; ++r) {
      const uint32_t u = out[k][r].x;
      if (__ballot(u != HEMPTY) == 0) continue;   // (wave-uniform)
      atomicAdd(&off[u != HEMPTY ? (int)(u / KC) : junk], 1);
    }
  __syncthreads();
  block_exclusive_scan(off, P.nch, nullptr);
  int32_t *choff = a_choff + (int64_t)rt * (P.nch + 1);
  for (int c = threadIdx.x; c <= P.nch; c += 64 * EXA_WAVES) choff[c] = off[c];
  const int total = __builtin_amdgcn_readfirstlane(off[P.nch]);
  __syncthreads();
  if (threadIdx.x == 0) a_base[rt] = tile_base;
  // placement: unconditional buffer stores (no entry: an offset past the range)
  const __amdgpu_buffer_rsrc_t r_out =
      __builtin_amdgcn_make_buffer_rsrc((void *)(a_list + tile_base), (short)0, total * 8, 0x00020000);
#pragma unroll
  for (int k = 0; k < EXA_SENT; ++k) {
    const int row = wave + EXA_WAVES * k;
#pragma unroll
    for (int r = 0; r < MERGE_ROUNDS; ++r) {
      const uint2 ent = out[k][r];
      const bool ok = ent.x != HEMPTY;
      if (__ballot(ok) == 0) continue;   // (wave-uniform)
      const int pos = atomicAdd(&off[ok ? (int)(ent.x / KC) : junk], 1);
      __builtin_amdgcn_raw_buffer_store_b64(
          (m_u32x2){a_code(ok ? ent.x : 0u, row, pitch, esize, compact), a_val(ent.y, row, pitch, esize, compact)},
          r_out, ok ? (uint32_t)pos * 8u : BUF_OOB, 0, 0);
    }
  }
}

// Compacted contraction (compact != 0): the column tile's vocabulary W (the
// distinct words of its sentences, ascending) numbers the K positions, so the
// contraction only walks ceil(|W| / KC) chunks.  Per global chunk c of KC
// words the builder writes mt[c] = {bit mask of W's words in c, |W| words in
// chunks before c}: the compacted position of word u is then
// mt[u/KC].base + popcount(mt[u/KC].mask below bit u%KC).  The B entries are
// grouped by compacted chunk and encoded at their compacted position.
__global__ __launch_bounds__(256) void k_build_b(PlanDev P, const int64_t *__restrict__ tgt_off,
                                                 const int32_t *__restrict__ tgt_tok,
                                                 uint32_t *__restrict__ b_list, int32_t *__restrict__ b_choff,
                                                 int pitch, int esize, int compact, uint2 *__restrict__ mt,
                                                 int32_t *__restrict__ kcn, int2 *__restrict__ krng,
                                                 int64_t *__restrict__ b_base, uint32_t *__restrict__ p_voc,
                                                 int c0) {
  extern __shared__ __align__(16) char smem[];
  int *off = reinterpret_cast<int *>(smem);        // [nch + 1]
  int *tmp = off + P.nch + 1;                      // [256]
  uint32_t *bits = reinterpret_cast<uint32_t *>(tmp + 256);  // 4 waves x [V/32]
  const int words = (P.V + 31) / 32;
  int *ubase = reinterpret_cast<int *>(bits + 4 * words);    // [words + 1] (compact)
  uint32_t *ubits = reinterpret_cast<uint32_t *>(ubase + words + 1);   // [words] (compact)
  const int ct = c0 + (int)blockIdx.x;
  const TileMeta tm = P.ct_meta[ct];
  const int cols = tm.count;
  const int64_t t0 = tm.first;
  const int64_t tile_base = tgt_off[t0];   // issued with the sentences' ranges
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint32_t *mybits = bits + wave * words;
  for (int c = threadIdx.x; c <= P.nch; c += 256) off[c] = 0;
  for (int w = lane; w < words; w += 64) mybits[w] = 0u;
  // sentences of this wave: lane k fetches sentence wave + 4k's token range
  // (sentences past the tile read sentence 0 and length 0), then the first
  // 64 tokens of every sentence are loaded together by unconditional buffer
  // loads (tokens past a sentence's length fall outside its buffer range)
  const int mycol = wave + 4 * lane;
  const bool vk = lane < ROWS_PER_WAVE && mycol < cols;
  const int64_t tq = t0 + (vk ? mycol : 0);
  const int64_t q0 = tgt_off[tq];
  const int ql = vk ? (int)(tgt_off[tq + 1] - q0) : 0;
  auto sent_len = [&](int k) { return __builtin_amdgcn_readlane(ql, k); };
  auto sent_off = [&](int k) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)q0, k);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)q0 >> 32), k);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  };
  uint32_t tok[ROWS_PER_WAVE];
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(tgt_tok + sent_off(k)), (short)0,
        __builtin_amdgcn_readfirstlane(min(max(sent_len(k), 0), 64) * 4), 0x00020000);
    tok[k] = buf_u32(r, (uint32_t)lane * 4u);
  }
#pragma unroll
  for (int k = 0; k < ROWS_PER_WAVE; ++k)
    if (lane >= sent_len(k)) tok[k] = 0xFFFFFFFFu;
  __syncthreads();
  if (compact) {
    // the tile's vocabulary: union of its sentences' words (each wave ORs
    // its sentences into its own bitmap, then the four are combined), then
    // the compacted position base of every chunk
#pragma unroll
    for (int k = 0; k < ROWS_PER_WAVE; ++k) {
      const uint32_t u = tok[k];
      if (u < (uint32_t)P.V) atomicOr(&mybits[u >> 5], 1u << (u & 31));
      const int64_t a = sent_off(k);
      const int l = sent_len(k);
      for (int x = 64 + lane; x < l; x += 64) {
        const uint32_t v = (uint32_t)tgt_tok[a + x];
        if (v < (uint32_t)P.V) atomicOr(&mybits[v >> 5], 1u << (v & 31));
      }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < words; w += 256) {
      ubits[w] = bits[w] | bits[words + w] | bits[2 * words + w] | bits[3 * words + w];
      bits[w] = bits[words + w] = bits[2 * words + w] = bits[3 * words + w] = 0u;
    }
    __syncthreads();
    // the pair's vocabulary is the union of its tiles' (cleared beforehand)
    if (p_voc)
      for (int w = threadIdx.x; w < words; w += 256)
        if (ubits[w]) atomicOr(&p_voc[(int64_t)tm.pair * words + w], ubits[w]);
    for (int w = threadIdx.x; w < words; w += 256) ubase[w] = __popc(ubits[w]);
    __syncthreads();
    block_exclusive_scan(ubase, words, tmp);
    // compacted chunk kc covers positions KC kc .. min(KC kc + KC, K) - 1:
    // its first / last global chunk is the one holding the first / last of
    // these positions (each written by exactly one thread)
    const int K = ubase[words];
    int32_t *rng = reinterpret_cast<int32_t *>(krng + (int64_t)ct * words);
    for (int w = threadIdx.x; w < words; w += 256) {
      const uint32_t msk = ubits[w];
      mt[(int64_t)ct * words + w] = make_uint2(msk, (uint32_t)ubase[w]);
      if (msk) {
        const int b0 = ubase[w], b1 = b0 + __popc(msk);   // positions [b0, b1)
        for (int kc = b0 / KC; kc <= (b1 - 1) / KC; ++kc) {
          const int first = KC * kc, last = min(KC * kc + KC, K) - 1;
          if (first >= b0 && first < b1) rng[2 * kc] = w;
          if (last >= b0 && last < b1) rng[2 * kc + 1] = w;
        }
      }
    }
    if (threadIdx.x == 0) kcn[ct] = (K + KC - 1) / KC;
    __syncthreads();
  }
  if (threadIdx.x == 0) b_base[ct] = tile_base;
  // K chunk and position inside it of word u
  auto kchunk = [&](uint32_t u) -> int {
    if (!compact) return (int)(u / KC);
    const uint32_t w = u >> 5, bit = u & 31;
    return (ubase[w] + __popc(ubits[w] & ((1u << bit) - 1u))) / KC;
  };
  auto kcode = [&](uint32_t u, int r) -> uint32_t {
    if (!compact) return (uint32_t)((r * pitch + (int)(u % KC)) * esize);
    const uint32_t w = u >> 5, bit = u & 31;
    const int pos = ubase[w] + __popc(ubits[w] & ((1u << bit) - 1u));
    return (uint32_t)((r * pitch + pos % KC) * esize);
  };
  // pass 1: distinct tokens of each sentence (first occurrence per word),
  // counted by chunk; first occurrences are remembered for pass 2
  uint32_t first = 0u;   // bit k: this lane's token of sentence k is a first occurrence
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const uint32_t u = tok[k];
    if (u < (uint32_t)P.V) {
      const uint32_t bit = 1u << (u & 31);
      if (!(atomicOr(&mybits[u >> 5], bit) & bit)) {
        first |= 1u << k;
        atomicAdd(&off[kchunk(u)], 1);
      }
    }
    const int64_t a = sent_off(k);
    const int l = sent_len(k);
    for (int x = 64 + lane; x < l; x += 64) {   // long sentences
      const uint32_t v = (uint32_t)tgt_tok[a + x];
      if (v < (uint32_t)P.V) {
        const uint32_t bit = 1u << (v & 31);
        if (!(atomicOr(&mybits[v >> 5], bit) & bit)) atomicAdd(&off[kchunk(v)], 1);
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
  for (int k = 0; k < ROWS_PER_WAVE; ++k) {
    const int r = wave + 4 * k;
    if (first & (1u << k)) {
      const uint32_t u = tok[k];
      const int pos = atomicAdd(&off[kchunk(u)], 1);
      b_list[tile_base + pos] = kcode(u, r);
    }
    const int64_t a = sent_off(k);
    const int l = sent_len(k);
    if (l > 64) {   // long sentences: redo the first-occurrence test
      const uint32_t u = tok[k];
      if (u < (uint32_t)P.V) atomicOr(&mybits[u >> 5], 1u << (u & 31));
      wave_sync();
      for (int x = 64 + lane; x < l; x += 64) {
        const uint32_t v = (uint32_t)tgt_tok[a + x];
        if (v < (uint32_t)P.V) {
          const uint32_t bit = 1u << (v & 31);
          if (!(atomicOr(&mybits[v >> 5], bit) & bit)) {
            const int pos = atomicAdd(&off[kchunk(v)], 1);
            b_list[tile_base + pos] = kcode(v, r);
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
int merge_hbits(int max_entries) {
  int hb = 7;
  while ((1 << hb) < 2 * max_entries) ++hb;
  return hb;
}

size_t merge_lds_bytes(int hbits) {
  const size_t hs = (size_t)1 << hbits;
  return hs * (sizeof(double) + sizeof(uint32_t)) + (hs / 2) * sizeof(int);
}

// Sentences sent_ids[k0 .. k0 + n_sent).
hipError_t launch_merge_src(int64_t n_sent, const int64_t *sent_ids, int64_t k0, const int64_t *src_off,
                            const int32_t *src_tok, const int32_t *d_row_off, const int32_t *d_col,
                            const float *d_val, int V, int max_deg, int max_entries, uint2 *merged, int32_t *cnt,
                            int waves_per_cu, hipStream_t st) {
  if (n_sent <= 0) return hipSuccess;
  if (n_sent >= ((int64_t)1 << 28)) return hipErrorInvalidValue;   // byte offsets of sent_ids stay 32-bit
  const int hb = merge_hbits(max_entries);
  const size_t lds = merge_lds_bytes(hb);
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  // resident waves: LDS-bound (about 160 KiB per CU), at most 32 per CU
  int per = (int)((160u * 1024u) / lds);
  per = per < 1 ? 1 : (per > 32 ? 32 : per);
  if (waves_per_cu > 0 && waves_per_cu < per) per = waves_per_cu;
  const int64_t want = (int64_t)cus * per;
  const int grid = (int)(n_sent < want ? n_sent : want);
  hipLaunchKernelGGL(k_merge_src, dim3(grid), dim3(64), lds, st, n_sent, sent_ids + k0, src_off, src_tok, d_row_off,
                     d_col, d_val, V, max_deg, hb, merged, cnt);
  return hipGetLastError();
}

// Row tiles [r0, r0 + n).
hipError_t launch_build_a(const PlanDev &P, const int64_t *src_off, const uint2 *merged, const int32_t *cnt,
                          uint2 *a_list, int32_t *a_choff, int pitch, int esize, int compact, int64_t *a_base,
                          const uint32_t *p_voc, int r0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const size_t lds = sizeof(int) * (size_t)(2 * P.nch + 1 + 256);
  hipLaunchKernelGGL(k_build_a, dim3(n), dim3(256), lds, st, P, src_off, merged, cnt, a_list, a_choff, pitch, esize,
                     compact, a_base, p_voc, r0);
  return hipGetLastError();
}

// Row tiles [r0, r0 + n), fused merge and list build.
// Merge-table size of the fused expansion: at most half full.
static int expand_a_hbits(int max_entries) { return merge_hbits(max_entries); }

hipError_t launch_expand_a(const PlanDev &P, const int64_t *src_off, const int32_t *src_tok, const uint2 *dpk, int V,
                           int max_entries, uint2 *a_list, int32_t *a_choff, int pitch, int esize, int compact,
                           int64_t *a_base, int r0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int hb = expand_a_hbits(max_entries);
  hipLaunchKernelGGL(k_expand_a, dim3(n), dim3(64 * EXA_WAVES), expand_a_lds_bytes(hb, P.nch), st, P, src_off,
                     src_tok, dpk, V, hb, a_list, a_choff, pitch, esize, compact, a_base, r0);
  return hipGetLastError();
}

// The dictionary padded to four entries per row: dpk[4 t + e] = entry e of
// row t, or word HEMPTY past the row's end.  Rows are cut at max_deg (at most
// four: the fused path only runs for such plans), as the merge cuts them.
__global__ __launch_bounds__(256) void k_pack_dict(const int32_t *__restrict__ row_off, const int32_t *__restrict__ col,
                                                   const float *__restrict__ val, int V, int max_deg,
                                                   uint2 *__restrict__ dpk) {
  for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < 4 * (int64_t)V; k += (int64_t)gridDim.x * 256) {
    const int t = (int)(k >> 2), e = (int)(k & 3);
    const int e0 = row_off[t], deg = min(row_off[t + 1] - e0, max_deg);
    dpk[k] = e < deg ? make_uint2((uint32_t)col[e0 + e], __float_as_uint(val[e0 + e])) : make_uint2(HEMPTY, 0u);
  }
}

hipError_t launch_pack_dict(const int32_t *row_off, const int32_t *col, const float *val, int V, int max_deg,
                            uint2 *dpk, hipStream_t st) {
  if (V <= 0) return hipSuccess;
  const int64_t blocks = (4 * (int64_t)V + 255) / 256;
  hipLaunchKernelGGL(k_pack_dict, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, st, row_off, col, val,
                     V, max_deg, dpk);
  return hipGetLastError();
}

// Whether the fused expansion covers a plan: every sentence's tokens in the
// merge's rounds, every dictionary row within four entries, and its LDS
// within the default dynamic limit.
bool expand_a_fits(int max_sent_tokens, int max_deg, int nch) {
  if (max_sent_tokens > 16 * MERGE_ROUNDS || max_deg > 4) return false;
  return expand_a_lds_bytes(expand_a_hbits(std::max(1, max_sent_tokens * max_deg)), nch) <= 65536;
}

__global__ __launch_bounds__(256) void k_clear_u32(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) p[k] = 0u;
}

// A fill kernel, not a memset: the clear may be captured into a graph.
hipError_t launch_clear_u32(uint32_t *p, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_clear_u32, dim3((unsigned)(blocks < 2048 ? blocks : 2048)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

size_t build_b_lds_bytes(int nch, int V) {
  const size_t words = (size_t)((V + 31) / 32);
  return sizeof(int) * (size_t)(nch + 1 + 256) + sizeof(uint32_t) * (4 * words + 2 * words + 1);
}

// Column tiles [c0, c0 + n).
hipError_t launch_build_b(const PlanDev &P, const int64_t *tgt_off, const int32_t *tgt_tok, uint32_t *b_list,
                          int32_t *b_choff, int pitch, int esize, int compact, uint2 *mt, int32_t *kcn,
                          int2 *krng, int64_t *b_base, uint32_t *p_voc, int c0, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_b, dim3(n), dim3(256), build_b_lds_bytes(P.nch, P.V), st, P, tgt_off, tgt_tok, b_list,
                     b_choff, pitch, esize, compact, mt, kcn, krng, b_base, p_voc, c0);
  return hipGetLastError();
}

hipError_t build_set_attrs(int nch, int V) {
  return hipFuncSetAttribute((const void *)k_build_b, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)build_b_lds_bytes(nch, V));
}

hipError_t merge_set_attrs(int max_entries) {
  return hipFuncSetAttribute((const void *)k_merge_src, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)merge_lds_bytes(merge_hbits(max_entries)));
}

}  // namespace nwm
