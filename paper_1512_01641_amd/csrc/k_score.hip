// Similarity of every sentence pair (Sec. 4): the dictionary-coverage
// contraction S_raw = (1/l_i) (T'.Y^T) on MFMA, with the logistic scorer
// fused into the epilogue:
//   z = w0 * S_raw + w1 * rho + b,  rho = min(l_i, l'_j) / max(l_i, l'_j),
//   S = 1 / (1 + exp(-z)).
//
// One workgroup = one TM x TN tile of one document pair.  K (the vocabulary)
// is walked in chunks of KC words; wave w owns chunks c = w (mod 4) and keeps
// private dense operand tiles in LDS, built from the chunk-major tile lists
// (k_build_a / k_build_b) by a scatter and cleared again by the same scatter
// after the MFMAs, so the K loop has no workgroup barrier.  The lists of a run
// of chunks are staged into LDS in one coalesced copy per K segment.  At the
// end the four partial tiles are summed in a fixed order (deterministic) and
// each wave finishes 16 rows: scale, features, sigmoid, coalesced stores.
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

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <bool BF16>
static __device__ __forceinline__ void mfma_chunk(const typename Op<BF16>::T *At, const typename Op<BF16>::T *Bt,
                                                  f32x4 (&acc)[4][4], int lane) {
  constexpr int P = Op<BF16>::PITCH;
  const int r16 = lane & 15, kq = lane >> 4;
  if constexpr (BF16) {
    bf16x8 a[4], b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a[q] = *reinterpret_cast<const bf16x8 *>(At + (16 * q + r16) * P + 8 * kq);
      b[q] = *reinterpret_cast<const bf16x8 *>(Bt + (16 * q + r16) * P + 8 * kq);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
  } else {
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      float a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = At[(16 * q + r16) * P + 4 * ks + kq];
        b[q] = Bt[(16 * q + r16) * P + 4 * ks + kq];
      }
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bi], b[bj], acc[bi][bj], 0, 0, 0);
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(GEMM_THREADS) void k_score(PlanDev P, const int64_t *__restrict__ src_off,
                                                        const int64_t *__restrict__ tgt_off,
                                                        const uint2 *__restrict__ a_list,
                                                        const int32_t *__restrict__ a_choff,
                                                        const uint32_t *__restrict__ b_list,
                                                        const int32_t *__restrict__ b_choff, nwm_scorer sc,
                                                        float *__restrict__ S, float *__restrict__ S_raw) {
  typedef typename Op<BF16>::T T;
  constexpr int PITCH = Op<BF16>::PITCH;
  constexpr int TILE_ELEMS = TM * PITCH;  // == TN * PITCH
  extern __shared__ __align__(16) char smem[];
  // region 1 (K loop): staged lists, chunk offsets, per-wave operand tiles
  uint2 *stA = reinterpret_cast<uint2 *>(smem);                      // [CAP_A]
  uint32_t *stB = reinterpret_cast<uint32_t *>(stA + CAP_A);         // [CAP_B]
  T *tiles = reinterpret_cast<T *>(stB + CAP_B);                     // [4][2][TILE_ELEMS]
  int *chA = reinterpret_cast<int *>(tiles + GEMM_WAVES * 2 * TILE_ELEMS);  // [nch+1]
  int *chB = chA + P.nch + 1;                                        // [nch+1]
  // region 2 (epilogue) aliases region 1: 4 partial tiles
  float *red = reinterpret_cast<float *>(smem);                      // [4][TM][TN+1]

  const int gt = blockIdx.x;
  const int rt = P.gt_rt[gt], ct = P.gt_ct[gt];
  const int pair = P.rt_pair[rt];
  const int row0 = P.rt_row0[rt], rows = P.rt_rows[rt];
  const int col0 = P.ct_col0[ct], cols = P.ct_cols[ct];
  const int64_t s_first = P.sfirst[pair] + row0;
  const int64_t t_first = P.tfirst[pair] + col0;
  const int m = P.m[pair];
  const int nch = P.nch;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  const int32_t *gA = a_choff + (int64_t)rt * (nch + 1);
  const int32_t *gB = b_choff + (int64_t)ct * (nch + 1);
  for (int c = tid; c <= nch; c += GEMM_THREADS) {
    chA[c] = gA[c];
    chB[c] = gB[c];
  }
  T *At = tiles + (2 * wave) * TILE_ELEMS;
  T *Bt = At + TILE_ELEMS;
  for (int e = lane; e < 2 * TILE_ELEMS; e += 64) At[e] = T(0.0f);
  const uint2 *listA = a_list + src_off[s_first] * (int64_t)P.max_deg;
  const uint32_t *listB = b_list + tgt_off[t_first];

  f32x4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();

  int c_lo = 0;
  while (c_lo < nch) {
    // largest c_hi such that the lists of chunks [c_lo, c_hi) fit the staging
    // buffers (a single chunk always fits: <= TM*KC and <= TN*KC entries)
    const int a0 = chA[c_lo], b0 = chB[c_lo];
    int lo = c_lo + 1, hi = nch;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (chA[mid] - a0 <= CAP_A && chB[mid] - b0 <= CAP_B) lo = mid;
      else hi = mid - 1;
    }
    const int c_hi = lo;
    const int na = min(chA[c_hi] - a0, CAP_A), nb = min(chB[c_hi] - b0, CAP_B);
    for (int e = tid; e < na; e += GEMM_THREADS) stA[e] = listA[a0 + e];
    for (int e = tid; e < nb; e += GEMM_THREADS) stB[e] = listB[b0 + e];
    __syncthreads();
    for (int c = c_lo + ((wave - c_lo) & 3); c < c_hi; c += GEMM_WAVES) {
      const int ea0 = chA[c] - a0, ea1 = min(chA[c + 1] - a0, na);
      const int eb0 = chB[c] - b0, eb1 = min(chB[c + 1] - b0, nb);
      for (int e = ea0 + lane; e < ea1; e += 64) {
        const uint2 v = stA[e];
        At[v.x] = T(__uint_as_float(v.y));
      }
      for (int e = eb0 + lane; e < eb1; e += 64) Bt[stB[e]] = T(1.0f);
      wave_sync();
      mfma_chunk<BF16>(At, Bt, acc, lane);
      wave_sync();
      for (int e = ea0 + lane; e < ea1; e += 64) At[stA[e].x] = T(0.0f);
      for (int e = eb0 + lane; e < eb1; e += 64) Bt[stB[e]] = T(0.0f);
      wave_sync();
    }
    __syncthreads();
    c_lo = c_hi;
  }

  // ---- fixed-order reduction of the four partial tiles -------------------
  constexpr int RP = TN + 1;
  float *myred = red + wave * TM * RP;
  const int r16 = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) myred[(16 * bi + 4 * rq + r) * RP + 16 * bj + r16] = acc[bi][bj][r];
  __syncthreads();

  // ---- epilogue: wave w finishes rows [16w, 16w+16) ------------------------
  const int col = lane;
  const bool vcol = col < cols;
  const float lt = vcol ? (float)(tgt_off[t_first + col + 1] - tgt_off[t_first + col]) : 0.0f;
  float *Sp = S + P.s_off[pair];
  float *Rp = S_raw ? S_raw + P.s_off[pair] : nullptr;
  for (int rr = 0; rr < 16; ++rr) {
    const int row = 16 * wave + rr;
    if (row >= rows) break;
    const int idx = row * RP + col;
    const float dot = ((red[idx] + red[TM * RP + idx]) + red[2 * TM * RP + idx]) + red[3 * TM * RP + idx];
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

size_t score_lds_bytes(int nch, bool bf16) {
  const size_t esz = bf16 ? 2 : 4;
  const size_t pitch = bf16 ? PITCH_BF16 : PITCH_F32;
  const size_t r1 = sizeof(uint2) * CAP_A + sizeof(uint32_t) * CAP_B + esz * GEMM_WAVES * 2 * TM * pitch +
                    sizeof(int) * 2 * (size_t)(nch + 1);
  const size_t r2 = sizeof(float) * GEMM_WAVES * TM * (TN + 1);
  return r1 > r2 ? r1 : r2;
}

hipError_t launch_score(const PlanDev &P, bool bf16, const int64_t *src_off, const int64_t *tgt_off,
                        const uint2 *a_list, const int32_t *a_choff, const uint32_t *b_list,
                        const int32_t *b_choff, nwm_scorer sc, float *S, float *S_raw, hipStream_t st) {
  if (P.n_gt <= 0) return hipSuccess;
  const size_t lds = score_lds_bytes(P.nch, bf16);
  if (bf16)
    hipLaunchKernelGGL(k_score<true>, dim3(P.n_gt), dim3(GEMM_THREADS), lds, st, P, src_off, tgt_off, a_list,
                       a_choff, b_list, b_choff, sc, S, S_raw);
  else
    hipLaunchKernelGGL(k_score<false>, dim3(P.n_gt), dim3(GEMM_THREADS), lds, st, P, src_off, tgt_off, a_list,
                       a_choff, b_list, b_choff, sc, S, S_raw);
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
