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

#include <type_traits>

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

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// List entries of one K chunk of one tile, as loaded: lane l holds entries
// l, 64 + l, ... counted from the chunk start.  Entries at or past the
// chunk's count belong to later chunks (or to the lists' slack) and are
// masked out by the count when the chunk is scattered, so the loads are
// unconditional and stay in flight until then.
struct Chunk {
  uint2 a[REG_A];     // {LDS byte offset in the A tile, FP32 value bits}
  uint32_t b[REG_B];  // LDS byte offset in the B tile
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

struct Lists {
  const uint2 *pa;      // the tile's A list (chunk-major)
  const uint32_t *pb;   // the tile's B list
};

// Window 1 (loaded 64 chunks ago) becomes window 0 when chunk c leaves
// window 0; rare, uniform, kept out of the chunk's straight-line code.
static __device__ __forceinline__ bool needs_slide(const OffWin &W, int c) { return c >= W.base + 64; }

static __device__ __forceinline__ void slide_window(OffWin &W, const int32_t *__restrict__ chA,
                                                    const int32_t *__restrict__ chB, int nch, int lane) {
  W.base += 64;
  W.wa0 = W.wa1;
  W.sa0 = W.sa1;
  W.wb0 = W.wb1;
  W.sb0 = W.sb1;
  load_window(W.wa1, W.sa1, chA, W.base + 64, nch, lane);
  load_window(W.wb1, W.sb1, chB, W.base + 64, nch, lane);
}

// The list entries of chunk c (the window must cover c) into C.
static __device__ __forceinline__ void load_chunk_regs(Chunk &C, const Lists &L, const OffWin &W, int c,
                                                       int lane) {
  const int k = c - W.base;
  C.a0 = __builtin_amdgcn_readlane(W.wa0, k);
  C.na = __builtin_amdgcn_readlane(W.sa0, k) - C.a0;
  C.b0 = __builtin_amdgcn_readlane(W.wb0, k);
  C.nb = __builtin_amdgcn_readlane(W.sb0, k) - C.b0;
  // uniform chunk base + constant lane offset: no per-entry address math;
  // reads past the last list stay inside its slack
  const uint2 *pa = L.pa + C.a0;
  const uint32_t *pb = L.pb + C.b0;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) C.a[q] = pa[q * 64 + lane];
#pragma unroll
  for (int q = 0; q < REG_B; ++q) C.b[q] = pb[q * 64 + lane];
}

static __device__ __forceinline__ void load_chunk(Chunk &C, const Lists &L, OffWin &W,
                                                  const int32_t *__restrict__ chA, const int32_t *__restrict__ chB,
                                                  int nch, int c, int lane) {
  if (needs_slide(W, c)) slide_window(W, chA, chB, nch, lane);
  load_chunk_regs(C, L, W, c, lane);
}

static __device__ __forceinline__ bool overflows(const Chunk &C) { return C.na > REG_A * 64 || C.nb > REG_B * 64; }

template <typename T>
static __device__ __forceinline__ void lds_put(char *tile, uint32_t byte_off, T v) {
  *reinterpret_cast<T *>(tile + byte_off) = v;
}

// Set the chunk's register entries in the tiles: every group of 64, with
// lanes past the count writing to a padding element no fragment reads; the
// address each lane used is kept in the chunk for the clear.  Straight-line
// code (no branches), so it can be interleaved with the MFMAs.
template <bool BF16>
static __device__ __forceinline__ void scatter_set_regs(Chunk &C, char *At, char *Bt, int lane, uint32_t junk) {
  typedef typename Op<BF16>::T T;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) {
    const uint32_t x = lane + 64 * q < C.na ? C.a[q].x : junk;
    C.a[q].x = x;
    lds_put<T>(At, x, T(__uint_as_float(C.a[q].y)));
  }
#pragma unroll
  for (int q = 0; q < REG_B; ++q) {
    const uint32_t x = lane + 64 * q < C.nb ? C.b[q] : junk;
    C.b[q] = x;
    lds_put<T>(Bt, x, T(1.0f));
  }
}

// Entries beyond the register capacity (rare) come straight from the lists.
template <bool BF16>
static __device__ __forceinline__ void scatter_set_rest(const Chunk &C, char *At, char *Bt, const Lists &L,
                                                        int lane) {
  typedef typename Op<BF16>::T T;
  for (int e = REG_A * 64 + lane; e < C.na; e += 64) {
    const uint2 v = L.pa[C.a0 + e];
    lds_put<T>(At, v.x, T(__uint_as_float(v.y)));
  }
  for (int e = REG_B * 64 + lane; e < C.nb; e += 64) lds_put<T>(Bt, L.pb[C.b0 + e], T(1.0f));
}

// Return the tiles to zero after a chunk, at the addresses its scatter used.
template <bool BF16>
static __device__ __forceinline__ void scatter_clear_regs(const Chunk &C, char *At, char *Bt) {
  typedef typename Op<BF16>::T T;
#pragma unroll
  for (int q = 0; q < REG_A; ++q) lds_put<T>(At, C.a[q].x, T(0.0f));
#pragma unroll
  for (int q = 0; q < REG_B; ++q) lds_put<T>(Bt, C.b[q], T(0.0f));
}

// Both whole tiles of a buffer, after a chunk that overflowed the registers.
template <bool BF16>
static __device__ __forceinline__ void clear_tiles(char *At, int lane) {
  constexpr int TILE_BYTES = TM * Op<BF16>::PITCH * (int)sizeof(typename Op<BF16>::T);
  uint4 *p = reinterpret_cast<uint4 *>(At);
  constexpr int N16 = 2 * TILE_BYTES / 16;
  for (int e = lane; e < N16; e += 64) p[e] = make_uint4(0u, 0u, 0u, 0u);
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
static __device__ __forceinline__ void read_frags(Frags<BF16> &F, const char *Atc, const char *Btc, int lane) {
  typedef typename Op<BF16>::T T;
  const T *At = reinterpret_cast<const T *>(Atc);
  const T *Bt = reinterpret_cast<const T *>(Btc);
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

// Instruction groups for the scheduler over one chunk's straight-line code:
// each MFMA followed by a slice of the other work -- first the LDS writes
// (clear, then scatter) with their VALU, then the fragment reads of the next
// chunk, then the list loads.  Dependencies are kept; groups that cannot be
// filled stay empty.
template <bool BF16>
static __device__ __forceinline__ void interleave() {
  constexpr int NMFMA = BF16 ? 16 : 128;
  constexpr int NW = 2 * (REG_A + REG_B);   // LDS writes: clear + set
  constexpr int NR = BF16 ? 8 : 64;         // fragment reads
  constexpr int P1 = 6, P2 = 8;             // MFMAs carrying writes, reads
  constexpr int PER_R = NR / P2;
#pragma unroll
  for (int i = 0; i < P1; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x200, (NW + P1 - 1) / P1, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
  }
#pragma unroll
  for (int i = 0; i < P2; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, PER_R, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
  __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
  __builtin_amdgcn_sched_group_barrier(0x020, REG_A + REG_B, 0);
  __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - P1 - P2 - 1, 0);
}

template <bool BF16>
struct ScoreLds {
  static constexpr int TILE = TM * Op<BF16>::PITCH * (int)sizeof(typename Op<BF16>::T);   // one operand tile
  static constexpr int OPS = 4 * TILE;                                                   // [2 buffers][A, B]
  static constexpr int RED = (int)sizeof(float) * TM * (TN + 1);                         // epilogue
  static constexpr int BYTES = OPS > RED ? OPS : RED;
};

// Features and logistic score of one cell (Sec. 4): S_raw = dot / l (0 for an
// empty source sentence), rho = min(l, l') / max(l, l') (1 when both
// sentences are empty), z = w0 S_raw + w1 rho + b, S = 1 / (1 + exp(-z)).
// rl, rlt are the reciprocals of l, l' (inf for 0), so rho = min(l / l',
// l' / l) = min(l rlt, l' rl); positive floats order as their bit patterns,
// so that minimum is an integer one.  An exponent past the FP32 range gives
// exp = inf and S = 0 (1 / inf), exp = 0 gives S = 1.  CHECKED = false drops
// the tests for empty sentences (every length of the tile is positive).
template <bool CHECKED>
static __device__ __forceinline__ float logistic_cell(float dot, float l, float rl, float lt, float rlt,
                                                      const nwm_scorer &sc, float &sraw) {
  const float LOG2E = 1.4426950408889634f;
  float sr = dot * rl;
  float rho = __uint_as_float(min(__float_as_uint(l * rlt), __float_as_uint(lt * rl)));
  if (CHECKED) {
    sr = l > 0.0f ? sr : 0.0f;
    rho = (l > 0.0f || lt > 0.0f) ? rho : 1.0f;
  }
  sraw = sr;
  const float z = __builtin_fmaf(sc.w0, sr, __builtin_fmaf(sc.w1, rho, sc.b));
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-z * LOG2E));
}

// Epilogue of a tile: accumulators -> LDS (transpose) -> per row the
// logistic scorer and coalesced stores of S (and S_raw).
static __device__ __forceinline__ void score_epilogue(const f32x4 (&acc)[4][4], float *red, const PlanDev &P,
                                                      const int64_t *__restrict__ src_off,
                                                      const int64_t *__restrict__ tgt_off, const nwm_scorer &sc,
                                                      float *__restrict__ S, float *__restrict__ S_raw, int pair,
                                                      int row0, int rows, int col0, int cols, int64_t s_first,
                                                      int64_t t_first, int m, int lane) {
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
  const float rlt = __builtin_amdgcn_rcpf(lt);
  float *Sp = S + P.s_off[pair];
  float *Rp = S_raw ? S_raw + P.s_off[pair] : nullptr;
  for (int row = 0; row < rows; ++row) {
    const float dot = red[row * RP + col];
    const float ls = (float)(src_off[s_first + row + 1] - src_off[s_first + row]);
    float sraw;
    const float sv = logistic_cell<true>(dot, ls, __builtin_amdgcn_rcpf(ls), lt, rlt, sc, sraw);
    if (vcol) {
      const int64_t o = (int64_t)(row0 + row) * m + col0 + col;
      Sp[o] = sv;
      if (Rp) Rp[o] = sraw;
    }
  }
}

// Epilogue straight from the accumulators (no LDS): lane l holds rows
// 16 bi + 4 (l >> 4) + r, column 16 bj + (l & 15) of the tile.  Sentence
// lengths come from the lane that owns that row / column index.  A full tile
// whose sentences are all non-empty (the common case) takes a path without
// per-cell tests whose stores address rows by a scalar offset and columns by
// the instruction's immediate offset: no address arithmetic per cell.
static __device__ __forceinline__ void score_epilogue_regs(const f32x4 (&acc)[4][4],
                                                           const int64_t *__restrict__ src_off,
                                                           const int64_t *__restrict__ tgt_off, const nwm_scorer &sc,
                                                           float *__restrict__ Sb, float *__restrict__ Rb, int row0,
                                                           int rows, int col0, int cols, int64_t s_first,
                                                           int64_t t_first, int m, int lane) {
  // Sb, Rb: the pair's S and S_raw blocks (Rb may be null)
  const float my_ls = lane < rows ? (float)(src_off[s_first + lane + 1] - src_off[s_first + lane]) : 0.0f;
  const float my_lt = lane < cols ? (float)(tgt_off[t_first + lane + 1] - tgt_off[t_first + lane]) : 0.0f;
  float *Sp = Sb + (int64_t)row0 * m + col0;
  float *Rp = Rb ? Rb + (int64_t)row0 * m + col0 : nullptr;
  const int r16 = lane & 15, rq = lane >> 4;
  // the lengths of this lane's 16 rows and 4 columns and their reciprocals
  float ls[4][4], rls[4][4], lt[4], rlt[4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ls[bi][r] = __shfl(my_ls, 16 * bi + 4 * rq + r, 64);
      rls[bi][r] = __builtin_amdgcn_rcpf(ls[bi][r]);
    }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    lt[bj] = __shfl(my_lt, 16 * bj + r16, 64);
    rlt[bj] = __builtin_amdgcn_rcpf(lt[bj]);
  }
  const bool full = rows == TM && cols == TN && __ballot(my_ls > 0.0f && my_lt > 0.0f) == ~0ull;
  if (full) {
    const __amdgpu_buffer_rsrc_t rS = __builtin_amdgcn_make_buffer_rsrc((void *)Sp, (short)0, 0x7FFFFFFF, 0x00020000);
    const uint32_t vbase = (uint32_t)((4 * rq * m + r16) * 4);   // row 4 rq, column r16
    auto sweep = [&](auto with_raw) {
      const __amdgpu_buffer_rsrc_t rR =
          __builtin_amdgcn_make_buffer_rsrc((void *)(Rp ? Rp : Sp), (short)0, 0x7FFFFFFF, 0x00020000);
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int srow = __builtin_amdgcn_readfirstlane((16 * bi + r) * m * 4);   // row offset, bytes
#pragma unroll
          for (int bj = 0; bj < 4; ++bj) {
            float sraw;
            const float sv =
                logistic_cell<false>(acc[bi][bj][r], ls[bi][r], rls[bi][r], lt[bj], rlt[bj], sc, sraw);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(sv), rS, vbase + 64u * bj, srow, 0);
            if (decltype(with_raw)::value)
              __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(sraw), rR, vbase + 64u * bj, srow, 0);
          }
        }
    };
    if (Rp) sweep(std::true_type{});
    else sweep(std::false_type{});
    return;
  }
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    const int col = 16 * bj + r16;
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * bi + 4 * rq + r;
        float sraw;
        const float sv = logistic_cell<true>(acc[bi][bj][r], ls[bi][r], rls[bi][r], lt[bj], rlt[bj], sc, sraw);
        if (row < rows && col < cols) {
          const int64_t o = (int64_t)row * m + col;
          Sp[o] = sv;
          if (Rp) Rp[o] = sraw;
        }
      }
  }
}

template <bool BF16>
__global__ __launch_bounds__(64) void k_score(PlanDev P, const int64_t *__restrict__ src_off,
                                              const int64_t *__restrict__ tgt_off, const uint2 *__restrict__ a_list,
                                              const int32_t *__restrict__ a_choff,
                                              const uint32_t *__restrict__ b_list,
                                              const int32_t *__restrict__ b_choff, nwm_scorer sc,
                                              float *__restrict__ S, float *__restrict__ S_raw, int xcd_map, int g0,
                                              int G) {
  typedef typename Op<BF16>::T T;
  constexpr int TB = ScoreLds<BF16>::TILE;
  // static LDS: tile addresses are compile-time constants folded into the
  // DS instruction offsets
  __shared__ __align__(16) char smem[ScoreLds<BF16>::BYTES];
  float *red = reinterpret_cast<float *>(smem);           // epilogue: [TM][TN + 1]

  // XCD-aware order: workgroups are dealt to the 8 XCDs round-robin, so
  // consecutive tiles (same pair, shared lists) go to one XCD and its L2
  // tiles [g0, g0 + G) of the plan
  const int per = (G + 7) >> 3;
  const int gl = xcd_map ? (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  if (gl >= G) return;
  const int gt = g0 + gl;
  const int rt = P.gt_rt[gt], ct = P.gt_ct[gt];
  const int pair = P.rt_pair[rt];
  const int row0 = P.rt_row0[rt], rows = P.rt_rows[rt];
  const int col0 = P.ct_col0[ct], cols = P.ct_cols[ct];
  const int64_t s_first = P.sfirst[pair] + row0;
  const int64_t t_first = P.tfirst[pair] + col0;
  const int m = P.m[pair];
  const int nch = P.nch;
  const int lane = threadIdx.x;
  // where idle lanes write: one padding element (row 0, column KC) shared
  // by all of them -- accesses to one address merge, so idle lanes add no
  // bank conflicts to the valid lanes' scattered writes
  const uint32_t junk = (uint32_t)(KC * (int)sizeof(T));

  const int32_t *chA = a_choff + (int64_t)rt * (nch + 1);
  const int32_t *chB = b_choff + (int64_t)ct * (nch + 1);
  Lists L;
  L.pa = a_list + src_off[s_first] * (int64_t)P.max_deg;
  L.pb = b_list + tgt_off[t_first];
  for (int e = lane; e < ScoreLds<BF16>::OPS / 16; e += 64)
    reinterpret_cast<uint4 *>(smem)[e] = make_uint4(0u, 0u, 0u, 0u);

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

  // Software pipeline, per chunk c: MFMAs of c (fragments read during chunk
  // c-1) -> clear chunk c-1 from the other LDS buffer -> scatter chunk c+1
  // into it -> read the fragments of c+1 -> load the list entries of chunk
  // c+3 into the registers chunk c-1 used.  Four entry register sets and two
  // fragment register sets rotate by unrolling (no register copies).
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
  Frags<BF16> F0, F1;
  wave_sync();
  scatter_set_regs<BF16>(S0, smem, smem + TB, lane, junk);
  scatter_set_rest<BF16>(S0, smem, smem + TB, L, lane);
  wave_sync();
  read_frags<BF16>(F0, smem, smem + TB, lane);

  // One chunk.  The core is straight-line code whose LDS and memory work the
  // scheduler interleaves between the MFMAs (MFMA issue blocks a wave, so
  // without interleaving a wave would start its LDS work only after its last
  // MFMA).  Rare cases sit outside it: a full clear after an overflowing
  // chunk and the offset-window slide before, the overflow entries of the
  // next chunk (then its fragments are read again) after.  Past the last
  // chunk the "next" chunk has no entries, so the core needs no test.
#define NWM_SCORE_CHUNK(c, prev, nxt, Fc, Fn)                                  \
  {                                                                            \
    char *Ao_ = smem + (((c) + 1) & 1) * 2 * TB;                               \
    if (overflows(prev)) clear_tiles<BF16>(Ao_, lane);                         \
    if (needs_slide(W, (c) + 3)) slide_window(W, chA, chB, nch, lane);         \
    mfma_frags<BF16>(Fc, acc);                                                 \
    scatter_clear_regs<BF16>(prev, Ao_, Ao_ + TB);                             \
    scatter_set_regs<BF16>(nxt, Ao_, Ao_ + TB, lane, junk);                    \
    read_frags<BF16>(Fn, Ao_, Ao_ + TB, lane);                                 \
    load_chunk_regs(prev, L, W, (c) + 3, lane);                                \
    interleave<BF16>();                                                        \
    if (overflows(nxt)) {                                                      \
      scatter_set_rest<BF16>(nxt, Ao_, Ao_ + TB, L, lane);                     \
      wave_sync();                                                             \
      read_frags<BF16>(Fn, Ao_, Ao_ + TB, lane);                               \
    }                                                                          \
  }
  int c = 0;
  for (; c + 4 <= nch; c += 4) {
    NWM_SCORE_CHUNK(c, S3, S1, F0, F1)
    NWM_SCORE_CHUNK(c + 1, S0, S2, F1, F0)
    NWM_SCORE_CHUNK(c + 2, S1, S3, F0, F1)
    NWM_SCORE_CHUNK(c + 3, S2, S0, F1, F0)
  }
  if (c < nch) NWM_SCORE_CHUNK(c, S3, S1, F0, F1)
  if (c + 1 < nch) NWM_SCORE_CHUNK(c + 1, S0, S2, F1, F0)
  if (c + 2 < nch) NWM_SCORE_CHUNK(c + 2, S1, S3, F0, F1)
#undef NWM_SCORE_CHUNK
  wave_sync();

  score_epilogue(acc, red, P, src_off, tgt_off, sc, S, S_raw, pair, row0, rows, col0, cols, s_first, t_first, m,
                 lane);
}

// ---- compacted contraction -------------------------------------------------------
// The same tile contraction with K restricted to the column tile's vocabulary
// W (built by k_build_b in compact mode): a word outside W has a zero Y
// factor in every column of the tile, so the sum over W equals the sum over
// the whole vocabulary.  Compacted chunk kc holds W's words KC kc ..
// KC kc + KC - 1; the A entries that can land in it are those of the global
// chunks c_lo(kc) .. c_hi(kc) those words span, one contiguous range of the
// row tile's chunk-major A list.  Each entry (word u, row r, value) is looked
// up in the column tile's chunk table staged in LDS and, when u is in W at a
// position of chunk kc, written to the dense A tile; entries of a global
// chunk that straddles two compacted chunks are read for both.  B entries
// come pre-encoded at their compacted positions.  The entries of chunk kc + 1
// are loaded while chunk kc is scattered and multiplied; the tiles are
// cleared whole after their fragments are read.
struct CChunk {
  uint2 a[CREG_A];     // {word << 6 | row, FP32 value bits}
  uint32_t b[CREG_B];  // LDS byte offset in the B tile
  int a0, na, b0, nb;
};

// Lane l: A range [a0, a1) and B range [b0, b1) of compacted chunk base + l.
struct CWin {
  int base;
  int a0, a1, b0, b1;
};

// LDS of the compacted contraction: KG tile pairs [A, B] (KG compacted
// chunks scattered per round).
template <bool BF16, int KG>
struct ScoreLdsC {
  static constexpr int OPS = 2 * ScoreLds<BF16>::TILE;   // one [A, B] pair
  static constexpr int BYTES = KG * OPS;
};

static __device__ __forceinline__ void cwin_load(CWin &W, int base, int Kc, const int2 *rng,
                                                 const int32_t *__restrict__ chA, const int32_t *__restrict__ chB,
                                                 int lane) {
  W.base = base;
  const int kc = base + lane;
  W.a0 = W.a1 = W.b0 = W.b1 = 0;
  if (kc < Kc) {
    const int2 r = rng[kc];
    W.a0 = chA[r.x];
    W.a1 = chA[r.y + 1];
    W.b0 = chB[kc];
    W.b1 = chB[kc + 1];
  }
}

static __device__ __forceinline__ void cload(CChunk &C, const uint2 *pa, const uint32_t *pb, const CWin &W, int kc,
                                             int lane) {
  // the chunk after a full window's last one loads an empty range
  const int k = kc - W.base;
  const bool in = k < 64;
  const int kk = in ? k : 63;
  C.a0 = __builtin_amdgcn_readlane(W.a0, kk);
  C.na = in ? __builtin_amdgcn_readlane(W.a1, kk) - C.a0 : 0;
  C.b0 = __builtin_amdgcn_readlane(W.b0, kk);
  C.nb = in ? __builtin_amdgcn_readlane(W.b1, kk) - C.b0 : 0;
  // unconditional: reads past the last list stay inside its slack
  const uint2 *a = pa + C.a0;
  const uint32_t *b = pb + C.b0;
#pragma unroll
  for (int q = 0; q < CREG_A; ++q) C.a[q] = a[q * 64 + lane];
#pragma unroll
  for (int q = 0; q < CREG_B; ++q) C.b[q] = b[q * 64 + lane];
}

// The A entries of compacted chunk kc into the dense A tile.  Register
// entries first, branch-free: every lane looks its CREG_A words up in the
// chunk table at once (lanes past the count look up word 0) and writes each
// entry either at its compacted position or, when its word is not in the
// chunk, to the shared padding element `junk`.  Entries past the registers
// (rare) follow from the list.
template <bool BF16>
static __device__ __forceinline__ void cscatter(const CChunk &C, char *At, char *Bt, const uint2 *mtl,
                                                const uint2 *pa, const uint32_t *pb, int kc, int lane,
                                                uint32_t junk) {
  typedef typename Op<BF16>::T T;
  constexpr uint32_t P = (uint32_t)Op<BF16>::PITCH;
  uint2 mm[CREG_A];
#pragma unroll
  for (int q = 0; q < CREG_A; ++q) {
    const uint32_t u = lane + 64 * q < C.na ? C.a[q].x >> 6 : 0u;
    mm[q] = mtl[u >> 5];
  }
  // BF16 entries carry the row's byte offset and the operand (see a_val in
  // the list builders); FP32 entries the row and the FP32 term
  auto put = [&](uint32_t x, uint32_t y, uint32_t pos) {
    if constexpr (BF16)
      lds_put<uint16_t>(At, (y >> 16) + (pos & 31u) * 2u, (uint16_t)y);
    else
      lds_put<T>(At, ((x & 63u) * P + (pos & 31u)) * (uint32_t)sizeof(T), T(__uint_as_float(y)));
  };
#pragma unroll
  for (int q = 0; q < CREG_A; ++q) {
    const uint32_t x = C.a[q].x, u = x >> 6, bit = u & 31u;
    const uint32_t pos = mm[q].y + (uint32_t)__popc(mm[q].x & ((1u << bit) - 1u));
    const bool hit =
        lane + 64 * q < C.na && __builtin_amdgcn_ubfe(mm[q].x, bit, 1u) != 0u && (pos >> 5) == (uint32_t)kc;
    if (hit) put(x, C.a[q].y, pos);
  }
  for (int e = CREG_A * 64 + lane; e < C.na; e += 64) {
    const uint2 v = pa[C.a0 + e];
    const uint32_t u = v.x >> 6, bit = u & 31u;
    const uint2 w = mtl[u >> 5];
    const uint32_t pos = w.y + (uint32_t)__popc(w.x & ((1u << bit) - 1u));
    if (__builtin_amdgcn_ubfe(w.x, bit, 1u) != 0u && (pos >> 5) == (uint32_t)kc) put(v.x, v.y, pos);
  }
#pragma unroll
  for (int q = 0; q < CREG_B; ++q) lds_put<T>(Bt, lane + 64 * q < C.nb ? C.b[q] : junk, T(1.0f));
  for (int e = CREG_B * 64 + lane; e < C.nb; e += 64) lds_put<T>(Bt, pb[C.b0 + e], T(1.0f));
}

// KG: compacted chunks per round (the K width of a round is 32 KG words).
// With KG = 2 both chunks of a round are scattered into their own tile pair
// before one wave barrier, then the MFMAs of the first and of the second run:
// every accumulator sums the chunks in the same order as with KG = 1, so the
// results are identical; the round's fixed costs (barrier, waits, loop) are
// shared by two chunks at the price of a fourth register set.
template <bool BF16, int KG>
__global__ __launch_bounds__(64) void k_score_c(PlanDev P, const int64_t *__restrict__ src_off,
                                                const int64_t *__restrict__ tgt_off,
                                                const uint2 *__restrict__ a_list, const int32_t *__restrict__ a_choff,
                                                const uint32_t *__restrict__ b_list,
                                                const int32_t *__restrict__ b_choff, const uint2 *__restrict__ mt,
                                                const int32_t *__restrict__ kcn, const int2 *__restrict__ krng,
                                                const int64_t *__restrict__ a_base,
                                                const int64_t *__restrict__ b_base, nwm_scorer sc,
                                                float *__restrict__ S, float *__restrict__ S_raw, int xcd_map,
                                                int g0, int G) {
  constexpr int TB = ScoreLds<BF16>::TILE;
  __shared__ __align__(16) char smem[ScoreLdsC<BF16, KG>::BYTES];   // KG x [A tile, B tile]
  extern __shared__ __align__(16) uint2 dyn[];                      // chunk table [nch]
  char *At = smem, *Bt = smem + TB;

  // tiles [g0, g0 + G) of the plan
  const int per = (G + 7) >> 3;
  const int gl = xcd_map ? (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
  if (gl >= G) return;
  const int gt = g0 + gl;
  // the tile's metadata in one record; everything else it needs is at most
  // two dependent loads away
  const GtMeta g = P.gt_meta[gt];
  const int rt = g.rt, ct = g.ct;
  const int nch = P.nch;
  const int lane = threadIdx.x;
  const int Kc = kcn[ct];
  uint2 *mtl = dyn;

  const uint2 *mtg = mt + (int64_t)ct * nch;
  const int2 *rng = krng + (int64_t)ct * nch;
  const int32_t *chA = a_choff + (int64_t)rt * (nch + 1);
  const int32_t *chB = b_choff + (int64_t)ct * (nch + 1);
  const uint2 *pa = a_list + a_base[rt];
  const uint32_t *pb = b_list + b_base[ct];
  CChunk X, Y, Z;
  // the first window of chunk ranges and the entries of the first two
  // chunks go out first (the longest chain of dependent loads); the chunk
  // table is staged in LDS meanwhile
  CWin W;
  cwin_load(W, 0, Kc, rng, chA, chB, lane);
  cload(X, pa, pb, W, 0, lane);
  cload(Y, pa, pb, W, 1, lane);
  for (int e = lane; e < ScoreLdsC<BF16, KG>::BYTES / 16; e += 64)
    reinterpret_cast<uint4 *>(smem)[e] = make_uint4(0u, 0u, 0u, 0u);
  for (int c = lane; c < nch; c += 64) mtl[c] = mtg[c];
  wave_sync();

  f32x4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};

  // padding element (row 0, column KC) no fragment reads: where lanes with
  // nothing to write go, all to one address
  const uint32_t junk = (uint32_t)(KC * (int)sizeof(typename Op<BF16>::T));
  // the clear after a chunk: only the KC columns of each of the pair's 2 TM
  // rows (the padding columns hold nothing a fragment reads), U 16-byte
  // units per row, lane l taking units l, l + 64, ...
  constexpr int RB = Op<BF16>::PITCH * (int)sizeof(typename Op<BF16>::T);   // bytes per tile row
  constexpr int U = KC * (int)sizeof(typename Op<BF16>::T) / 16;
  constexpr int NCLR = 2 * TM * U / 64;   // per lane, per tile pair
  static_assert(64 % U == 0 && (2 * TM * U) % 64 == 0 && 2 * TB == 2 * TM * RB, "tile clear");
  const int clr0 = (lane / U) * RB + (lane % U) * 16;
  Frags<BF16> F;

  // chunk kc from register set Cur while the chunk after next (of the same
  // window of 64) loads into Nxt; the tiles are cleared whole after their
  // fragments are read (LDS operations of a wave complete in order)
#define NWM_SCORE_CCHUNK(kc, Cur, Nxt)                                         \
  {                                                                            \
    cload(Nxt, pa, pb, W, (kc) + 2, lane);                                     \
    cscatter<BF16>(Cur, At, Bt, mtl, pa, pb, (kc), lane, junk);                \
    wave_sync();                                                               \
    read_frags<BF16>(F, At, Bt, lane);                                         \
    _Pragma("unroll") for (int e_ = 0; e_ < NCLR; ++e_)                        \
      *reinterpret_cast<uint4 *>(smem + clr0 + e_ * (64 / U) * RB) = make_uint4(0u, 0u, 0u, 0u); \
    mfma_frags<BF16>(F, acc);                                                  \
  }
  // windows of 64 compacted chunks (one almost always covers the tile); the
  // loads past the window's last chunk read an empty range
  if constexpr (KG == 1) {
    for (int wb = 0; wb < Kc; wb += 64) {
      if (wb > 0) {
        cwin_load(W, wb, Kc, rng, chA, chB, lane);
        cload(X, pa, pb, W, wb, lane);
        cload(Y, pa, pb, W, wb + 1, lane);
      }
      const int we = min(Kc, wb + 64) - wb;   // chunks in this window
      int k = 0;
      for (; k + 3 <= we; k += 3) {
        NWM_SCORE_CCHUNK(wb + k, X, Z)
        NWM_SCORE_CCHUNK(wb + k + 1, Y, X)
        NWM_SCORE_CCHUNK(wb + k + 2, Z, Y)
      }
      if (k < we) NWM_SCORE_CCHUNK(wb + k, X, Z)
      if (k + 1 < we) NWM_SCORE_CCHUNK(wb + k + 1, Y, X)
    }
  } else {
    // rounds of chunks (kc, kc + 1) from sets (C0, C1) while (kc + 2, kc + 3)
    // load into (N0, N1); the second tile pair follows the first in LDS.  A
    // round whose second chunk is past the window's end skips its MFMAs (its
    // tiles stay zero).
    char *At1 = smem + 2 * TB, *Bt1 = smem + 3 * TB;
    CChunk X1 = Y, Y0, Y1;
#define NWM_SCORE_CROUND(kc, C0, C1, N0, N1, has2)                                     \
  {                                                                                    \
    cload(N0, pa, pb, W, (kc) + 2, lane);                                              \
    cload(N1, pa, pb, W, (kc) + 3, lane);                                              \
    cscatter<BF16>(C0, At, Bt, mtl, pa, pb, (kc), lane, junk);                         \
    cscatter<BF16>(C1, At1, Bt1, mtl, pa, pb, (kc) + 1, lane, junk);                   \
    wave_sync();                                                                       \
    read_frags<BF16>(F, At, Bt, lane);                                                 \
    _Pragma("unroll") for (int e_ = 0; e_ < NCLR; ++e_)                                \
      *reinterpret_cast<uint4 *>(smem + clr0 + e_ * (64 / U) * RB) = make_uint4(0u, 0u, 0u, 0u); \
    mfma_frags<BF16>(F, acc);                                                          \
    if (has2) {                                                                        \
      read_frags<BF16>(F, At1, Bt1, lane);                                             \
      _Pragma("unroll") for (int e_ = 0; e_ < NCLR; ++e_)                              \
        *reinterpret_cast<uint4 *>(smem + 2 * TB + clr0 + e_ * (64 / U) * RB) = make_uint4(0u, 0u, 0u, 0u); \
      mfma_frags<BF16>(F, acc);                                                        \
    }                                                                                  \
  }
    for (int wb = 0; wb < Kc; wb += 64) {
      if (wb > 0) {
        cwin_load(W, wb, Kc, rng, chA, chB, lane);
        cload(X, pa, pb, W, wb, lane);
        cload(X1, pa, pb, W, wb + 1, lane);
      }
      const int we = min(Kc, wb + 64) - wb;   // chunks in this window
      int k = 0;
      for (; k + 4 <= we; k += 4) {
        NWM_SCORE_CROUND(wb + k, X, X1, Y0, Y1, true)
        NWM_SCORE_CROUND(wb + k + 2, Y0, Y1, X, X1, true)
      }
      if (k < we) NWM_SCORE_CROUND(wb + k, X, X1, Y0, Y1, k + 1 < we)
      if (k + 2 < we) NWM_SCORE_CROUND(wb + k + 2, Y0, Y1, X, X1, k + 3 < we)
    }
#undef NWM_SCORE_CROUND
  }
#undef NWM_SCORE_CCHUNK
  score_epilogue_regs(acc, src_off, tgt_off, sc, S + g.s_off, S_raw ? S_raw + g.s_off : nullptr, g.row0, g.rows,
                      g.col0, g.cols, g.s_first, g.t_first, g.m, lane);
}

size_t score_lds_bytes(int, bool bf16) {
  return bf16 ? (size_t)ScoreLds<true>::BYTES : (size_t)ScoreLds<false>::BYTES;
}

hipError_t launch_score(const PlanDev &P, bool bf16, const int64_t *src_off, const int64_t *tgt_off,
                        const uint2 *a_list, const int32_t *a_choff, const uint32_t *b_list,
                        const int32_t *b_choff, nwm_scorer sc, float *S, float *S_raw, int xcd_map, int compact,
                        int kgroup, const uint2 *mt, const int32_t *kcn, const int2 *krng, const int64_t *a_base,
                        const int64_t *b_base, int g0, int G, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  const int grid = xcd_map ? 8 * ((G + 7) / 8) : G;
  if (compact) {
    const size_t dyn = sizeof(uint2) * (size_t)P.nch;
#define NWM_LAUNCH_C(B_, K_)                                                                              \
  hipLaunchKernelGGL((k_score_c<B_, K_>), dim3(grid), dim3(64), dyn, st, P, src_off, tgt_off, a_list, a_choff, \
                     b_list, b_choff, mt, kcn, krng, a_base, b_base, sc, S, S_raw, xcd_map, g0, G)
    if (bf16) {
      if (kgroup == 2) NWM_LAUNCH_C(true, 2);
      else NWM_LAUNCH_C(true, 1);
    } else {
      if (kgroup == 2) NWM_LAUNCH_C(false, 2);
      else NWM_LAUNCH_C(false, 1);
    }
#undef NWM_LAUNCH_C
    return hipGetLastError();
  }
  if (bf16)
    hipLaunchKernelGGL(k_score<true>, dim3(grid), dim3(64), 0, st, P, src_off, tgt_off, a_list, a_choff, b_list,
                       b_choff, sc, S, S_raw, xcd_map, g0, G);
  else
    hipLaunchKernelGGL(k_score<false>, dim3(grid), dim3(64), 0, st, P, src_off, tgt_off, a_list, a_choff, b_list,
                       b_choff, sc, S, S_raw, xcd_map, g0, G);
  return hipGetLastError();
}

hipError_t score_set_attrs(int) { return hipSuccess; }   // static LDS only

}  // namespace nwm
