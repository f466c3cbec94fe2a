// Backward of the mined alignment score through the NW DP and the logistic
// scorer (drives the tuning of threshold and penalty, Sec. 5.2).
//
// The NW score of a pair is a maximum of affine path sums
//   sum_{aligned (i,j)} S[i][j] + gap * (number of gap steps),
// so where the optimal path is unique its gradient is the path's DIAG
// indicator P for S and the gap count G = n + m - 2k for gap.  Chained through
// S = sigmoid(z), z = w0 S_raw + w1 rho + b:
//   dL/dz = dL/dS * S (1 - S);  dL/d(w0, w1, b) = sum dL/dz * (S_raw, rho, 1).
//
// k_bwd_dense   (optional) grad_S := grad_S_extra (or 0) for every cell, and
//               the dense chain of grad_S_extra, per row tile in FP32.
// k_bwd_path    one wave per pair: the path-sparse chain in FP32, grad_S += a_b
//               on the path, per-pair partials (dw0, dw1, db, a_b * G).  Not
//               launched without a score gradient (no path term).  Path cells
//               outside the pair's n x m block are skipped.
// k_bwd_reduce  one block: FP64 sum of all partials in a fixed order.
#include "nwm_internal.h"
#include "libnwmine.h"

namespace nwm {

static __device__ __forceinline__ float wave_sum(float v) {
  // fixed butterfly order: deterministic
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

static __device__ __forceinline__ float rho_of(float ls, float lt) {
  if (ls == 0.0f && lt == 0.0f) return 1.0f;
  return fminf(ls, lt) / fmaxf(ls, lt);
}

__global__ __launch_bounds__(256) void k_bwd_dense(PlanDev P, const int64_t *__restrict__ src_off,
                                                   const int64_t *__restrict__ tgt_off,
                                                   const float *__restrict__ E, const float *__restrict__ S,
                                                   const float *__restrict__ S_raw, float *__restrict__ grad_S,
                                                   float *__restrict__ part, int want_wb) {
  __shared__ float red[3][256];
  const int rt = blockIdx.x;
  const int pair = P.rt_pair[rt];
  const int row0 = P.rt_row0[rt], rows = P.rt_rows[rt];
  const int m = P.m[pair];
  const int64_t s_first = P.sfirst[pair] + row0;
  const int64_t t_first = P.tfirst[pair];
  const int64_t base = P.s_off[pair] + (int64_t)row0 * m;
  const int64_t cells = (int64_t)rows * m;
  float g0 = 0.f, g1 = 0.f, gb = 0.f;
  for (int64_t c = threadIdx.x; c < cells; c += 256) {
    const float e = E ? E[base + c] : 0.0f;
    if (grad_S) grad_S[base + c] = e;
    if (E && want_wb) {
      const int r = (int)(c / m), j = (int)(c - (int64_t)r * m);
      const float s = S[base + c];
      const float dz = e * s * (1.0f - s);
      const float ls = (float)(src_off[s_first + r + 1] - src_off[s_first + r]);
      const float lt = (float)(tgt_off[t_first + j + 1] - tgt_off[t_first + j]);
      g0 += dz * S_raw[base + c];
      g1 += dz * rho_of(ls, lt);
      gb += dz;
    }
  }
  if (!part) return;
  red[0][threadIdx.x] = g0;
  red[1][threadIdx.x] = g1;
  red[2][threadIdx.x] = gb;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (threadIdx.x < d)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[4 * rt + q] = red[q][0];
}

__global__ __launch_bounds__(64) void k_bwd_path(PlanDev P, const int64_t *__restrict__ src_off,
                                                 const int64_t *__restrict__ tgt_off,
                                                 const int2 *__restrict__ path, const int32_t *__restrict__ n_diag,
                                                 const float *__restrict__ grad_score, const float *__restrict__ S,
                                                 const float *__restrict__ S_raw, float *__restrict__ grad_S,
                                                 float *__restrict__ part, int want_wb) {
  const int b = blockIdx.x;
  const int n = P.n[b], m = P.m[b];
  const int lane = threadIdx.x;
  const int cap = min(n, m);
  const int k = min(n_diag[b], cap);
  const float a = grad_score[b];
  const int2 *pa = path + P.p_off[b] + (cap - k);
  const int64_t base = P.s_off[b];
  float g0 = 0.f, g1 = 0.f, gb = 0.f;
  for (int q = lane; q < k; q += 64) {
    const int2 c = pa[q];
    if ((unsigned)c.x >= (unsigned)n || (unsigned)c.y >= (unsigned)m) continue;
    const int64_t o = base + (int64_t)c.x * m + c.y;
    if (grad_S) grad_S[o] += a;
    if (want_wb) {
      const float s = S[o];
      const float dz = a * s * (1.0f - s);
      const float ls = (float)(src_off[P.sfirst[b] + c.x + 1] - src_off[P.sfirst[b] + c.x]);
      const float lt = (float)(tgt_off[P.tfirst[b] + c.y + 1] - tgt_off[P.tfirst[b] + c.y]);
      g0 += dz * S_raw[o];
      g1 += dz * rho_of(ls, lt);
      gb += dz;
    }
  }
  g0 = wave_sum(g0);
  g1 = wave_sum(g1);
  gb = wave_sum(gb);
  if (lane == 0) {
    part[4 * b + 0] = g0;
    part[4 * b + 1] = g1;
    part[4 * b + 2] = gb;
    part[4 * b + 3] = a * (float)(n + m - 2 * k);
  }
}

__global__ __launch_bounds__(256) void k_bwd_reduce(int n_path, const float *__restrict__ part_path, int n_dense,
                                                    const float *__restrict__ part_dense,
                                                    double *__restrict__ grad_gap, double *__restrict__ grad_wb) {
  __shared__ double red[4][256];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < n_path; b += 256)
    for (int q = 0; q < 4; ++q) v[q] += (double)part_path[4 * b + q];
  for (int r = threadIdx.x; r < n_dense; r += 256)
    for (int q = 0; q < 3; ++q) v[q] += (double)part_dense[4 * r + q];
  for (int q = 0; q < 4; ++q) red[q][threadIdx.x] = v[q];
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (threadIdx.x < d)
      for (int q = 0; q < 4; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (grad_wb) {
      grad_wb[0] = red[0][0];
      grad_wb[1] = red[1][0];
      grad_wb[2] = red[2][0];
    }
    if (grad_gap) grad_gap[0] = red[3][0];
  }
}

hipError_t launch_backward(const PlanDev &P, const int64_t *src_off, const int64_t *tgt_off, const int2 *path,
                           const int32_t *n_diag, const float *grad_score, const float *E, float *grad_S,
                           double *grad_gap, const float *S, const float *S_raw, double *grad_wb,
                           float *part_path, float *part_dense, hipStream_t st) {
  if (P.B <= 0) return hipSuccess;
  const int want_wb = grad_wb != nullptr;
  const bool dense = (grad_S != nullptr) || (E != nullptr && want_wb);
  if (dense && P.n_rt > 0) {
    hipLaunchKernelGGL(k_bwd_dense, dim3(P.n_rt), dim3(256), 0, st, P, src_off, tgt_off, E, S, S_raw, grad_S,
                       (E && want_wb) ? part_dense : nullptr, want_wb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // without a score gradient there is no path term (tb and n_diag unused)
  const int n_path = grad_score ? P.B : 0;
  if (n_path > 0) {
    hipLaunchKernelGGL(k_bwd_path, dim3(P.B), dim3(64), 0, st, P, src_off, tgt_off, path, n_diag, grad_score, S,
                       S_raw, grad_S, part_path, want_wb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int nd = (E && want_wb) ? P.n_rt : 0;
  hipLaunchKernelGGL(k_bwd_reduce, dim3(1), dim3(256), 0, st, n_path, part_path, nd, part_dense, grad_gap, grad_wb);
  return hipGetLastError();
}

}  // namespace nwm
