// Needleman-Wunsch global alignment of the sentence sequences of every
// document pair (Sec. 5.1, Figs. 1-2, eq. (1)) and the threshold filter
// (Sec. 4).
//
// k_nw_fill  anti-diagonal wavefront, one wave per pair (longest pairs
//            first).  The DP lattice is cut into strips of 64 rows; lane r
//            owns row r of the strip and at step t computes column
//            j = t - r + 1, so each step is one anti-diagonal of the strip
//            (the paper's "diagonal in parallel threads").  The value from the
//            row above arrives from lane r-1 by a DPP wave shift; lane 0
//            reads the previous strip's last row from LDS, which the strip's
//            last row overwrites in place behind it.  S is staged into an LDS
//            ring of 32-column blocks with a one-block register prefetch.
//            Per cell, in FP32 without contraction:
//               up = H[i-1][j] + g, left = H[i][j-1] + g, diag = H[i-1][j-1] + S
//               first maximum of (up, left, diag) with '>' (ties UP > LEFT > DIAG)
//            The directions of a step are packed with two ballots into one
//            16-byte word (UP bits, LEFT bits); 64 words are written per
//            64 steps by one coalesced store.  H itself never reaches HBM.
// k_nw_walk  traceback from (n, m): one wave per pair walks the direction
//            words, holding a 64-step window in registers (one word per lane)
//            and reading it with uniform-index readlane.  Aligned pairs are
//            written right-aligned (ascending) into the path area.
// k_keep     keeps the aligned pairs with S >= threshold, ascending.
#include "nwm_internal.h"

namespace nwm {

static __device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

static __device__ __forceinline__ float shr1(float x) {
  // lane l receives lane l-1's value (lane 0 receives 0 and is overwritten)
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xF, 0xF, false));
}

static __device__ __forceinline__ int steps_padded(int m) { return ((m + 63 + 63) / 64) * 64; }

// Load block q (64 rows x DP_BW columns of S, rows >= nrows / cols >= m read as 0).
static __device__ __forceinline__ void dp_load_block(float (&R)[DP_BW], const float *__restrict__ Sb, int i0,
                                                     int nrows, int m, int q, int lane) {
  const int col = DP_BW * q + (lane & (DP_BW - 1));
  const bool vc = col < m;
#pragma unroll
  for (int k = 0; k < DP_BW; ++k) {
    const int row = 2 * k + (lane >> 5);
    R[k] = (vc && row < nrows) ? Sb[(int64_t)(i0 + row) * m + col] : 0.0f;
  }
}

static __device__ __forceinline__ void dp_store_block(const float (&R)[DP_BW], float *ring, int q, int lane) {
  const int rc = (DP_BW * q + (lane & (DP_BW - 1))) & (DP_RING_COLS - 1);
#pragma unroll
  for (int k = 0; k < DP_BW; ++k) {
    const int row = 2 * k + (lane >> 5);
    ring[row * DP_PITCH + rc] = R[k];
  }
}

__global__ __launch_bounds__(64) void k_nw_fill(PlanDev P, const float *__restrict__ S, float g,
                                                float *__restrict__ score, char *__restrict__ tb) {
  extern __shared__ __align__(16) float lds[];
  float *ring = lds;                       // [64][DP_PITCH]
  float *prev = lds + 64 * DP_PITCH;       // [m+1]
  const int b = P.dp_order[blockIdx.x];
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  if (n == 0 || m == 0) {
    // H[n][0] = fl32(n*g), H[0][m] = fl32(m*g), H[0][0] = +0
    if (lane == 0) score[b] = (n + m == 0) ? 0.0f : (float)(n + m) * g;
    return;
  }
  const float *Sb = S + P.s_off[b];
  TbWord *tbb = reinterpret_cast<TbWord *>(tb + P.tb_off[b]);
  const int spad = steps_padded(m);
  for (int j = lane; j <= m; j += 64) prev[j] = (float)j * g;   // first row H[0][j]
  wave_sync();
  const int nstrips = (n + 63) / 64;
  for (int s = 0; s < nstrips; ++s) {
    const int i0 = 64 * s;
    const int rows = min(64, n - i0);
    const int i = i0 + 1 + lane;
    const bool vrow = lane < rows;
    float H = (float)i * g;                 // first column H[i][0]
    float diag = (float)i0 * g;             // lane 0: H[i0][0]
    if (lane == 0) prev[0] = diag;
    TbWord *tbs = tbb + (int64_t)s * spad;
    const int T_end = m + rows - 1;
    // stage block 0, prefetch block 1
    float R[DP_BW];
    dp_load_block(R, Sb, i0, rows, m, 0, lane);
    dp_store_block(R, ring, 0, lane);
    dp_load_block(R, Sb, i0, rows, m, 1, lane);
    wave_sync();
    uint32_t w_up_lo = 0, w_up_hi = 0, w_lf_lo = 0, w_lf_hi = 0;
    for (int t0 = 0; t0 < T_end; t0 += DP_BW) {
      const int tq = t0 / DP_BW;
      const int t1 = min(t0 + DP_BW, T_end);
      for (int t = t0; t < t1; ++t) {
        const int j = t - lane + 1;
        const bool act = vrow && j >= 1 && j <= m;
        const float from_above = shr1(H);
        const float pv = prev[min(t + 1, m)];
        const float up_in = (lane == 0) ? pv : from_above;
        const float sv = ring[lane * DP_PITCH + ((t - lane) & (DP_RING_COLS - 1))];
        const float up = up_in + g;
        const float left = H + g;
        const float dg = diag + sv;
        float best = up;
        int dir = DIR_UP;
        if (left > best) {
          best = left;
          dir = DIR_LEFT;
        }
        if (dg > best) {
          best = dg;
          dir = DIR_DIAG;
        }
        if (act) H = best;
        diag = up_in;
        if (act && lane == rows - 1) prev[j] = H;
        if (act && i == n && j == m) score[b] = H;
        const uint64_t um = __ballot(act && dir == DIR_UP);
        const uint64_t lm = __ballot(act && dir == DIR_LEFT);
        const int tl = t & 63;
        const bool mine = lane == tl;   // lane tl keeps step t's word
        w_up_lo = mine ? (uint32_t)um : w_up_lo;
        w_up_hi = mine ? (uint32_t)(um >> 32) : w_up_hi;
        w_lf_lo = mine ? (uint32_t)lm : w_lf_lo;
        w_lf_hi = mine ? (uint32_t)(lm >> 32) : w_lf_hi;
        if (tl == 63 || t == T_end - 1) {
          if (lane <= tl) {
            TbWord w;
            w.up_lo = w_up_lo;
            w.up_hi = w_up_hi;
            w.left_lo = w_lf_lo;
            w.left_hi = w_lf_hi;
            tbs[t - tl + lane] = w;
          }
        }
      }
      // block tq+1 (prefetched) enters the ring; prefetch block tq+2
      dp_store_block(R, ring, tq + 1, lane);
      dp_load_block(R, Sb, i0, rows, m, tq + 2, lane);
      wave_sync();
    }
    wave_sync();
  }
}

__global__ __launch_bounds__(64) void k_nw_walk(PlanDev P, const char *__restrict__ tb_bits,
                                                int2 *__restrict__ path, int32_t *__restrict__ n_diag) {
  const int b = P.dp_order[blockIdx.x];
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  const int cap = min(n, m);
  int2 *pa = path + P.p_off[b];
  const TbWord *tbb = reinterpret_cast<const TbWord *>(tb_bits + P.tb_off[b]);
  const int spad = steps_padded(m);
  int i = n, j = m, k = 0;
  int ws = -1, wt0 = 0;
  TbWord w = {0u, 0u, 0u, 0u};
  while (i > 0 && j > 0) {
    const int s = (i - 1) >> 6;
    const int r = (i - 1) & 63;
    const int t = j - 1 + r;
    if (s != ws || t < wt0) {
      ws = s;
      wt0 = t & ~63;
      w = tbb[(int64_t)s * spad + wt0 + lane];
    }
    const int idx = t - wt0;
    const uint32_t uw = (uint32_t)__builtin_amdgcn_readlane((int)(r < 32 ? w.up_lo : w.up_hi), idx);
    const uint32_t lw = (uint32_t)__builtin_amdgcn_readlane((int)(r < 32 ? w.left_lo : w.left_hi), idx);
    const uint32_t bit = 1u << (r & 31);
    if (uw & bit) {
      --i;
    } else if (lw & bit) {
      --j;
    } else {
      ++k;
      if (lane == 0 && k <= cap) pa[cap - k] = make_int2(i - 1, j - 1);
      --i;
      --j;
    }
  }
  if (lane == 0) n_diag[b] = k;
}

__global__ __launch_bounds__(64) void k_keep(PlanDev P, const float *__restrict__ S, float thr,
                                             const int2 *__restrict__ path, const int32_t *__restrict__ n_diag,
                                             int2 *__restrict__ kept, int32_t *__restrict__ n_kept) {
  const int b = blockIdx.x;
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  const int cap = min(n, m);
  const int k = min(n_diag[b], cap);
  const int2 *pa = path + P.p_off[b] + (cap - k);
  int2 *kp = kept + P.p_off[b];
  const float *Sb = S + P.s_off[b];
  int nk = 0;
  for (int q0 = 0; q0 < k; q0 += 64) {
    const int q = q0 + lane;
    int2 c = make_int2(0, 0);
    bool keep = false;
    if (q < k) {
      c = pa[q];
      keep = Sb[(int64_t)c.x * m + c.y] >= thr;
    }
    const uint64_t km = __ballot(keep);
    if (keep) kp[nk + __popcll(km & ((1ull << lane) - 1ull))] = c;
    nk += __popcll(km);
  }
  if (lane == 0) n_kept[b] = nk;
}

size_t fill_lds_bytes(int max_m) { return sizeof(float) * (64 * DP_PITCH + (size_t)max_m + 1); }

hipError_t launch_nw_fill(const PlanDev &P, int max_m, const float *S, float g, float *score, char *tb,
                          hipStream_t st) {
  if (P.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nw_fill, dim3(P.B), dim3(64), fill_lds_bytes(max_m), st, P, S, g, score, tb);
  return hipGetLastError();
}

hipError_t launch_nw_walk(const PlanDev &P, const char *tb, int2 *path, int32_t *n_diag, hipStream_t st) {
  if (P.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nw_walk, dim3(P.B), dim3(64), 0, st, P, tb, path, n_diag);
  return hipGetLastError();
}

hipError_t launch_keep(const PlanDev &P, const float *S, float thr, const int2 *path, const int32_t *n_diag,
                       int2 *kept, int32_t *n_kept, hipStream_t st) {
  if (P.B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_keep, dim3(P.B), dim3(64), 0, st, P, S, thr, path, n_diag, kept, n_kept);
  return hipGetLastError();
}

hipError_t fill_set_attrs(int max_m) {
  return hipFuncSetAttribute((const void *)k_nw_fill, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)fill_lds_bytes(max_m));
}

}  // namespace nwm
