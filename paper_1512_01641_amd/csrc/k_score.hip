// Similarity of every sentence pair (Sec. 4): the dictionary-coverage
// contraction S_raw = (1/l_i) (T'.Y^T) on MFMA, with the logistic scorer
// fused into the epilogue:
//   z = w0 * S_raw + w1 * rho + b,  rho = min(l_i, l'_j) / max(l_i, l'_j),
//   S = 1 / (1 + exp(-z)).
//
// One wave = one TM x TN tile of one document pair, over the whole
// vocabulary (no workgroup barriers, several independent waves per CU).  K is
// walked in chunks of KC words.  The operands of a chunk are dense LDS tiles
// built from the chunk-major lists of k_build_a / k_build_b: the list entries
// of a chunk are loaded into registers two chunks ahead, scattered into one of
// two LDS buffers, read as MFMA fragments, and the same entries clear the
// buffer again one chunk later -- so the scatter and the fragment reads of
// chunk c+1 overlap the MFMAs of chunk c.  Tiles are mapped so that the tiles
// of one pair (which share their lists) run on one XCD and share its L2.  The
// epilogue transposes the accumulators through LDS and stores S (and S_raw)
// with coalesced rows.
//
// Operands: BF16 (v_mfma_f32_16x16x32_bf16) or FP32 (v_mfma_f32_16x16x4_f32);
// accumulation is FP32 in both cases.  Y is 0/1 and exact in BF16; T' is
// rounded once to the operand type.
#include "nwm_internal.h"
#include "libnwmine.h"

namespace nwm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool BF16>
struct Op;
template <>
struct Op<true> {
  typedef __bf16 T;
  static constexpr int PITCH = PITCH_BF16;
};
template <>
struct Op<false> {
  typedef float T;
  static constexpr int PITCH = PITCH_F32;
};

constexpr int REG_A = 2;   // A entries per lane held in registers per chunk (128)
constexpr int REG_B = 4;   // B entries per lane (256; frequent target words crowd the first chunks)

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// List entries of one K chunk of one tile, as loaded: lane l holds entries
// l, 64 + l, ... of the chunk; entries at or past the chunk's count are junk
// and are recognised from the count at scatter time (so the loaded values are
// not touched before they are needed, and the loads stay in flight).
struct Chunk {
  uint2 a[REG_A];     // {LDS element offset in the A tile, FP32 value bits}
  uint32_t b[REG_B];  // LDS element offset in the B tile
  int a0, na, b0, nb; // list start and count (uniform)
};

// Chunk offsets of a tile's two lists in registers: lane l of w* holds the
// offset of chunk base + l, lane l of s* that of chunk base + 1 + l (window 0
// resident, window 1 loaded 64 chunks before it is needed).
struct OffWin {
  int base;
  int wa0, sa0, wb0, sb0;   // window 0
  int wa1, sa1, wb1, sb1;   // window 1 (chunks base + 64 ...)
};

static __device__ __forceinline__ int load_off(const int32_t *__restrict__ ch, int idx, int nch) {
  return ch[min(idx, nch)];
}

static __device__ __forceinline__ void load_window(int &w, int &sh, const int32_t *__restrict__ ch, int first,
                                                   int nch, int lane) {
  w = load_off(ch, first + lane, nch);
  sh = load_off(ch, first + 1 + lane, nch);
}

// Raw buffers over a tile's two lists.  Lanes past a chunk's end read with
// an offset beyond the buffer and get 0, so every load is issued
// unconditionally (exact wait counts, no branches).
struct Lists {
  __amdgpu_buffer_rsrc_t a, b;
  const uint2 *pa;
  const uint32_t *pb;
};
constexpr uint32_t OOB = 0xFFFFFFF0u;

static __device__ __forceinline__ void load_chunk(Chunk &C, const Lists &L, OffWin &W,
                                                  const int32_t *__restrict__ chA, const int32_t *__restrict__ chB,
                                                  int nch, int c, int lane) {
  if (c >= W.base + 64) {   // slide: window 1 (loaded 64 chunks ago) becomes window 0
    W.base += 64;
    W.wa0 = W.wa1;
    W.sa0 = W.sa1;
    W.wb0 = W.wb1;
    W.sb0 = W.sb1;
    load_window(W.wa1, W.sa1, chA, W.base + 64, nch, lane);
    load_window(W.wb1, W.sb1, chB, W.base + 64, nch, lane);
  }
  const int k = c - W.base;
  C.a0 = __builtin_amdgcn_readlane(W.wa0, k);
  C.na = __builtin_amdgcn_readlane(W.sa0, k) - C.a0;
  C.b0 = __builtin_amdgcn_readlane(W.wb0, k);
  C.nb = __builtin_amdgcn_readlane(W.sb0, k) - C.b0;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) {
    const int e = q * 64 + lane;
    const uint32_t off = e < C.na ? (uint32_t)(C.a0 + e) * 8u : OOB;
    const uint64_t v = (uint64_t)__builtin_amdgcn_raw_buffer_load_b64(L.a, off, 0, 0);
    C.a[q] = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
  }
#pragma unroll
  for (int q = 0; q < REG_B; ++q) {
    const int e = q * 64 + lane;
    const uint32_t off = e < C.nb ? (uint32_t)(C.b0 + e) * 4u : OOB;
    C.b[q] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(L.b, off, 0, 0);
  }
}

// Set the chunk's entries in the tiles.  Junk register entries write to a
// padding element of row 0 (column KC), which no MFMA fragment reads; entries
// beyond the register capacity (rare) come straight from the lists, after the
// register entries so that their loads do not delay those.
template <bool BF16>
static __device__ __forceinline__ void scatter_set(const Chunk &C, typename Op<BF16>::T *At,
                                                   typename Op<BF16>::T *Bt, const Lists &L, int lane) {
  typedef typename Op<BF16>::T T;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) {
    const uint32_t x = (q * 64 + lane < C.na) ? C.a[q].x : (uint32_t)KC;
    At[x] = T(__uint_as_float(C.a[q].y));
  }
#pragma unroll
  for (int q = 0; q < REG_B; ++q) {
    const uint32_t x = (q * 64 + lane < C.nb) ? C.b[q] : (uint32_t)KC;
    Bt[x] = T(1.0f);
  }
  for (int e = REG_A * 64 + lane; e < C.na; e += 64) {
    const uint2 v = L.pa[C.a0 + e];
    At[v.x] = T(__uint_as_float(v.y));
  }
  for (int e = REG_B * 64 + lane; e < C.nb; e += 64) Bt[L.pb[C.b0 + e]] = T(1.0f);
}

// Return the tiles to zero after a chunk: its register entries, or the whole
// buffer when the chunk overflowed the registers (no memory loads here).
template <bool BF16>
static __device__ __forceinline__ void scatter_clear(const Chunk &C, typename Op<BF16>::T *At,
                                                     typename Op<BF16>::T *Bt, int lane) {
  typedef typename Op<BF16>::T T;
  constexpr int TILE_ELEMS = TM * Op<BF16>::PITCH;
  if (C.na > REG_A * 64 || C.nb > REG_B * 64) {
    uint4 *p = reinterpret_cast<uint4 *>(At);
    constexpr int N16 = 2 * TILE_ELEMS * (int)sizeof(T) / 16;
    for (int e = lane; e < N16; e += 64) p[e] = make_uint4(0u, 0u, 0u, 0u);
    return;
  }
#pragma unroll
  for (int q = 0; q < REG_A; ++q) {
    const uint32_t x = (q * 64 + lane < C.na) ? C.a[q].x : (uint32_t)KC;
    At[x] = T(0.0f);
  }
#pragma unroll
  for (int q = 0; q < REG_B; ++q) {
    const uint32_t x = (q * 64 + lane < C.nb) ? C.b[q] : (uint32_t)KC;
    Bt[x] = T(0.0f);
  }
}

// MFMA operand fragments of one chunk (BF16: one K step of 32; FP32: eight
// K steps of 4) and the 16 (BF16) or 128 (FP32) MFMAs of a 64 x 64 tile.
template <bool BF16>
struct Frags;
template <>
struct Frags<true> {
  bf16x8 a[4], b[4];
};
template <>
struct Frags<false> {
  float a[KC / 4][4], b[KC / 4][4];
};

template <bool BF16>
static __device__ __forceinline__ void read_frags(Frags<BF16> &F, const typename Op<BF16>::T *At,
                                                  const typename Op<BF16>::T *Bt, int lane) {
  constexpr int P = Op<BF16>::PITCH;
  const int r16 = lane & 15, kq = lane >> 4;
  if constexpr (BF16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      F.a[q] = *reinterpret_cast<const bf16x8 *>(At + (16 * q + r16) * P + 8 * kq);
      F.b[q] = *reinterpret_cast<const bf16x8 *>(Bt + (16 * q + r16) * P + 8 * kq);
    }
  } else {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        F.a[ks][q] = At[(16 * q + r16) * P + 4 * ks + kq];
        F.b[ks][q] = Bt[(16 * q + r16) * P + 4 * ks + kq];
      }
  }
}

template <bool BF16>
static __device__ __forceinline__ void mfma_frags(const Frags<BF16> &F, f32x4 (&acc)[4][4]) {
  if constexpr (BF16) {
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a[bi], F.b[bj], acc[bi][bj], 0, 0, 0);
  } else {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(F.a[ks][bi], F.b[ks][bj], acc[bi][bj], 0, 0, 0);
  }
}

template <bool BF16>
__global__ __launch_bounds__(64) void k_score(PlanDev P, const int64_t *__restrict__ src_off,
                                              const int64_t *__restrict__ tgt_off, const uint2 *__restrict__ a_list,
                                              const int32_t *__restrict__ a_choff,
                                              const uint32_t *__restrict__ b_list,
                                              const int32_t *__restrict__ b_choff, nwm_scorer sc,
                                              float *__restrict__ S, float *__restrict__ S_raw) {
  typedef typename Op<BF16>::T T;
  constexpr int PITCH = Op<BF16>::PITCH;
  constexpr int TILE_ELEMS = TM * PITCH;  // == TN * PITCH
  extern __shared__ __align__(16) char smem[];
  T *tiles = reinterpret_cast<T *>(smem);                 // [2 buffers][A, B][TILE_ELEMS]
  float *red = reinterpret_cast<float *>(smem);           // epilogue: [TM][TN + 1]

  // XCD-aware order: consecutive tiles (same pair, shared lists) on one XCD
  const int G = P.n_gt;
  const int per = (G + 7) >> 3;
  const int gt = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (gt >= G) return;
  const int rt = P.gt_rt[gt], ct = P.gt_ct[gt];
  const int pair = P.rt_pair[rt];
  const int row0 = P.rt_row0[rt], rows = P.rt_rows[rt];
  const int col0 = P.ct_col0[ct], cols = P.ct_cols[ct];
  const int64_t s_first = P.sfirst[pair] + row0;
  const int64_t t_first = P.tfirst[pair] + col0;
  const int m = P.m[pair];
  const int nch = P.nch;
  const int lane = threadIdx.x;

  const int32_t *chA = a_choff + (int64_t)rt * (nch + 1);
  const int32_t *chB = b_choff + (int64_t)ct * (nch + 1);
  Lists L;
  L.pa = a_list + src_off[s_first] * (int64_t)P.max_deg;
  L.pb = b_list + tgt_off[t_first];
  L.a = __builtin_amdgcn_make_buffer_rsrc((void *)L.pa, (short)0, 0x7FFFFFFF, 0x00020000);
  L.b = __builtin_amdgcn_make_buffer_rsrc((void *)L.pb, (short)0, 0x7FFFFFFF, 0x00020000);
  for (int e = lane; e < 4 * TILE_ELEMS; e += 64) tiles[e] = T(0.0f);

  f32x4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};

  OffWin W;
  W.base = 0;
  load_window(W.wa0, W.sa0, chA, 0, nch, lane);
  load_window(W.wb0, W.sb0, chB, 0, nch, lane);
  load_window(W.wa1, W.sa1, chA, 64, nch, lane);
  load_window(W.wb1, W.sb1, chB, 64, nch, lane);

  // Pipeline per chunk c: operand reads of c (buffer c&1) -> clear chunk c-1
  // from the other buffer -> scatter chunk c+1 into it -> MFMAs of c -> load
  // the list entries of chunk c+3 into the registers chunk c-1 used.  Four
  // register sets rotate by unrolling (no copies of registers in flight).
  Chunk S0, S1, S2, S3;
  S3.na = S3.nb = 0;
  S3.a0 = S3.b0 = 0;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) S3.a[q] = make_uint2(0u, 0u);
#pragma unroll
  for (int q = 0; q < REG_B; ++q) S3.b[q] = 0u;
  S1 = S3;
  S2 = S3;
  load_chunk(S0, L, W, chA, chB, nch, 0, lane);
  load_chunk(S1, L, W, chA, chB, nch, 1, lane);
  load_chunk(S2, L, W, chA, chB, nch, 2, lane);
  scatter_set<BF16>(S0, tiles, tiles + TILE_ELEMS, L, lane);

  // one chunk: operand reads of c -> clear c-1 / scatter c+1 in the other
  // buffer (LDS writes overlap the reads) -> MFMAs of c -> entries of c+3
#define NWM_SCORE_CHUNK(c, prev, nxt)                                          \
  {                                                                            \
    T *At_ = tiles + ((c) & 1) * 2 * TILE_ELEMS;                               \
    T *Ao_ = tiles + (((c) + 1) & 1) * 2 * TILE_ELEMS;                         \
    wave_sync();                                                               \
    Frags<BF16> F_;                                                            \
    read_frags<BF16>(F_, At_, At_ + TILE_ELEMS, lane);                         \
    scatter_clear<BF16>(prev, Ao_, Ao_ + TILE_ELEMS, lane);                    \
    if ((c) + 1 < nch) scatter_set<BF16>(nxt, Ao_, Ao_ + TILE_ELEMS, L, lane); \
    mfma_frags<BF16>(F_, acc);                                                 \
    load_chunk(prev, L, W, chA, chB, nch, (c) + 3, lane); /* empty past nch */ \
  }
  int c = 0;
  for (; c + 4 <= nch; c += 4) {
    NWM_SCORE_CHUNK(c, S3, S1)
    NWM_SCORE_CHUNK(c + 1, S0, S2)
    NWM_SCORE_CHUNK(c + 2, S1, S3)
    NWM_SCORE_CHUNK(c + 3, S2, S0)
  }
  if (c < nch) NWM_SCORE_CHUNK(c, S3, S1)
  if (c + 1 < nch) NWM_SCORE_CHUNK(c + 1, S0, S2)
  if (c + 2 < nch) NWM_SCORE_CHUNK(c + 2, S1, S3)
#undef NWM_SCORE_CHUNK
  wave_sync();

  // ---- epilogue: accumulators -> LDS (transpose) -> coalesced rows ---------
  constexpr int RP = TN + 1;
  const int r16 = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[(16 * bi + 4 * rq + r) * RP + 16 * bj + r16] = acc[bi][bj][r];
  wave_sync();
  const int col = lane;
  const bool vcol = col < cols;
  const float lt = vcol ? (float)(tgt_off[t_first + col + 1] - tgt_off[t_first + col]) : 0.0f;
  float *Sp = S + P.s_off[pair];
  float *Rp = S_raw ? S_raw + P.s_off[pair] : nullptr;
  for (int row = 0; row < rows; ++row) {
    const float dot = red[row * RP + col];
    const float ls = (float)(src_off[s_first + row + 1] - src_off[s_first + row]);
    const float sraw = ls > 0.0f ? dot / ls : 0.0f;
    float rho;
    if (ls == 0.0f && lt == 0.0f) rho = 1.0f;
    else rho = fminf(ls, lt) / fmaxf(ls, lt);
    const float z = __builtin_fmaf(sc.w0, sraw, __builtin_fmaf(sc.w1, rho, sc.b));
    float s;
    if (z >= 0.0f) {
      s = 1.0f / (1.0f + expf(-z));
    } else {
      const float ez = expf(z);
      s = ez / (1.0f + ez);
    }
    if (vcol) {
      const int64_t o = (int64_t)(row0 + row) * m + col0 + col;
      Sp[o] = s;
      if (Rp) Rp[o] = sraw;
    }
  }
}

size_t score_lds_bytes(int, bool bf16) {
  const size_t esz = bf16 ? 2 : 4;
  const size_t pitch = bf16 ? PITCH_BF16 : PITCH_F32;
  const size_t r1 = esz * 2 * 2 * TM * pitch;
  const size_t r2 = sizeof(float) * TM * (TN + 1);
  return r1 > r2 ? r1 : r2;
}

hipError_t launch_score(const PlanDev &P, bool bf16, const int64_t *src_off, const int64_t *tgt_off,
                        const uint2 *a_list, const int32_t *a_choff, const uint32_t *b_list,
                        const int32_t *b_choff, nwm_scorer sc, float *S, float *S_raw, hipStream_t st) {
  if (P.n_gt <= 0) return hipSuccess;
  const size_t lds = score_lds_bytes(P.nch, bf16);
  const int grid = 8 * ((P.n_gt + 7) / 8);
  if (bf16)
    hipLaunchKernelGGL(k_score<true>, dim3(grid), dim3(64), lds, st, P, src_off, tgt_off, a_list, a_choff, b_list,
                       b_choff, sc, S, S_raw);
  else
    hipLaunchKernelGGL(k_score<false>, dim3(grid), dim3(64), lds, st, P, src_off, tgt_off, a_list, a_choff, b_list,
                       b_choff, sc, S, S_raw);
  return hipGetLastError();
}

hipError_t score_set_attrs(int nch) {
  hipError_t e = hipFuncSetAttribute((const void *)k_score<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)score_lds_bytes(nch, true));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void *)k_score<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)score_lds_bytes(nch, false));
}

}  // namespace nwm
