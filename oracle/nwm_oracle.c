/*
 * nwm_oracle.c -- plain, slow CPU oracle for the comparable-corpus mining hot
 * path (score every sentence pair, Needleman-Wunsch align, keep pairs at or
 * above the threshold, and the path-sparse backward).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no code, header, table or helper with
 * the HIP path.
 *
 * Precision: scores in FP64; the DP in FP32 with one fixed per-cell operation
 * order (build with -O2 -ffp-contract=off, no fast-math; x86-64 SSE FP32).
 *
 * Paper: Wolk & Marasek, "Unsupervised comparable corpora preparation and
 * exploration for bi-lingual translation equivalents" (arXiv 1512.01641).
 *   Sec. 4   -- classifier likelihood in [0,1], SVM distance through a sigmoid,
 *               dictionary with translation probabilities; threshold filter.
 *   Sec. 5.1 -- NW: similarity matrix, gap penalty, DP matrix with (0,0)=0,
 *               first row/column initialised, each cell from its top, left and
 *               top-left neighbours; eq. (1).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - the classifier features are phi = (S_raw, rho) with S_raw the
 *     dictionary-coverage contraction (X.D).Y^T and rho the length ratio;
 *   - the boundary is H[i][0] = fl32(i*g), H[0][j] = fl32(j*g) (global
 *     alignment, end gaps pay the linear gap score g < 0);
 *   - eq. (1)'s match/mismatch term becomes +S[i][j], its -2 becomes g;
 *   - exact ties resolve UP > LEFT > DIAG (compare with IEEE '>' only);
 *   - a pair is kept iff S >= threshold (FP32 compare).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { DIR_DIAG = 0, DIR_UP = 1, DIR_LEFT = 2 };

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int nwo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sec. 4: the classifier's likelihood normalised into [0,1].  Steps:
 *  O1  S_raw[i][j] = (1/l_i) * sum over tokens t of source sentence i (with
 *      multiplicity) of sum over dictionary entries (u, d) of row t of
 *      d * [u occurs in target sentence j]  (= ((X.D).Y^T)[i][j] with X the
 *      term frequency over l_i and Y binary presence); 0 when l_i = 0.
 *  O2  rho[i][j] = min(l_i, l'_j) / max(l_i, l'_j), 1 when both are 0.
 *  O3  z = w0*S_raw + w1*rho + b;  S = sigmoid(z) (distance through a
 *      sigmoid), evaluated in the overflow-free form; S32 = fl32(S).
 * Output arrays are indexed s_off[b] + i*m_b + j.  Any output may be NULL. */
int nwo_score(int B, int V, const int32_t *n, const int32_t *m,
              const int64_t *src_off, const int32_t *src_tok,
              const int64_t *tgt_off, const int32_t *tgt_tok,
              const int32_t *d_row_off, const int32_t *d_col, const float *d_val,
              double w0, double w1, double bias, const int64_t *s_off,
              double *S_raw_out, double *rho_out, double *S64_out, float *S32_out,
              int nthreads) {
  if (B < 0 || V <= 0) return 1;
  int64_t *sfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B + 1));
  int64_t *tfirst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(B + 1));
  sfirst[0] = tfirst[0] = 0;
  for (int b = 0; b < B; ++b) {
    sfirst[b + 1] = sfirst[b] + n[b];
    tfirst[b + 1] = tfirst[b] + m[b];
  }
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    unsigned char *present = (unsigned char *)calloc((size_t)V, 1);
#pragma omp for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
      for (int j = 0; j < m[b]; ++j) {
        int64_t tj = tfirst[b] + j;
        int64_t t0 = tgt_off[tj], t1 = tgt_off[tj + 1];
        for (int64_t q = t0; q < t1; ++q) present[tgt_tok[q]] = 1;
        double lt = (double)(t1 - t0);
        for (int i = 0; i < n[b]; ++i) {
          int64_t si = sfirst[b] + i;
          int64_t s0 = src_off[si], s1 = src_off[si + 1];
          double ls = (double)(s1 - s0);
          double acc = 0.0;
          for (int64_t p = s0; p < s1; ++p) {
            int t = src_tok[p];
            for (int32_t e = d_row_off[t]; e < d_row_off[t + 1]; ++e)
              if (present[d_col[e]]) acc += (double)d_val[e];
          }
          double sraw = (ls > 0.0) ? acc / ls : 0.0;
          double rho;
          if (ls == 0.0 && lt == 0.0) rho = 1.0;
          else rho = (ls < lt ? ls : lt) / (ls > lt ? ls : lt);
          double z = w0 * sraw + w1 * rho + bias;
          double S;
          if (z >= 0.0) S = 1.0 / (1.0 + exp(-z));
          else { double ez = exp(z); S = ez / (1.0 + ez); }
          int64_t o = s_off[b] + (int64_t)i * m[b] + j;
          if (S_raw_out) S_raw_out[o] = sraw;
          if (rho_out) rho_out[o] = rho;
          if (S64_out) S64_out[o] = S;
          if (S32_out) S32_out[o] = (float)S;
        }
        for (int64_t q = t0; q < t1; ++q) present[tgt_tok[q]] = 0;
      }
    }
    free(present);
  }
  free(sfirst);
  free(tfirst);
  return err;
}

/* Sec. 5.1, Figs. 1-2 and eq. (1): fill the (n+1) x (m+1) DP matrix H for one
 * pair and record the chosen predecessor of every inner cell in T.
 * H and T are caller-provided, (n+1)*(m+1) each, row-major. */
static void nw_fill(int n, int m, const float *S, float g, float *H, unsigned char *T) {
  const int64_t W = (int64_t)m + 1;
  H[0] = 0.0f;                                        /* S(0,0) = 0 by definition */
  for (int i = 1; i <= n; ++i) H[(int64_t)i * W] = (float)i * g;   /* first column */
  for (int j = 1; j <= m; ++j) H[j] = (float)j * g;                /* first row    */
  for (int i = 1; i <= n; ++i) {
    for (int j = 1; j <= m; ++j) {
      float up = H[(int64_t)(i - 1) * W + j] + g;
      float left = H[(int64_t)i * W + (j - 1)] + g;
      float diag = H[(int64_t)(i - 1) * W + (j - 1)] + S[(int64_t)(i - 1) * m + (j - 1)];
      float best = up;
      unsigned char dir = DIR_UP;
      if (left > best) { best = left; dir = DIR_LEFT; }
      if (diag > best) { best = diag; dir = DIR_DIAG; }
      H[(int64_t)i * W + j] = best;
      T[(int64_t)i * W + j] = dir;
    }
  }
}

/* Walk back from (n, m) to (0, 0).  On the first row only LEFT moves remain,
 * on the first column only UP moves.  DIAG steps are the aligned sentence
 * pairs; they are written to path[] in ascending order.  Returns k. */
static int nw_traceback(int n, int m, const unsigned char *T, int32_t *path) {
  const int64_t W = (int64_t)m + 1;
  int i = n, j = m, k = 0;
  int cap = n < m ? n : m;
  int32_t *rev = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(cap > 0 ? cap : 1));
  while (i > 0 || j > 0) {
    int dir;
    if (i == 0) dir = DIR_LEFT;
    else if (j == 0) dir = DIR_UP;
    else dir = T[(int64_t)i * W + j];
    if (dir == DIR_DIAG) {
      rev[2 * k] = i - 1;
      rev[2 * k + 1] = j - 1;
      ++k;
      --i;
      --j;
    } else if (dir == DIR_UP) {
      --i;
    } else {
      --j;
    }
  }
  for (int q = 0; q < k; ++q) {
    path[2 * q] = rev[2 * (k - 1 - q)];
    path[2 * q + 1] = rev[2 * (k - 1 - q) + 1];
  }
  free(rev);
  return k;
}

/* Align every pair: NW fill + traceback + threshold filter (Sec. 4: a pair
 * whose similarity is below the threshold is excluded).
 *   path/kept: pair b's pairs start at element 2*path_off[b] (capacity
 *   min(n_b, m_b) pairs each).  score, n_diag, n_kept: [B].
 *   H_out / T_out: optional, full matrices of pair 0 only (for tests). */
int nwo_align(int B, const int32_t *n, const int32_t *m, const int64_t *s_off,
              const float *S32, float gap, float thr, const int64_t *path_off,
              float *score, int32_t *n_diag, int32_t *path, int32_t *kept,
              int32_t *n_kept, float *H_out, unsigned char *T_out, int nthreads) {
  if (B < 0) return 1;
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < B; ++b) {
    int nb = n[b], mb = m[b];
    size_t cells = (size_t)(nb + 1) * (size_t)(mb + 1);
    float *H = (float *)malloc(sizeof(float) * cells);
    unsigned char *T = (unsigned char *)malloc(cells);
    if (!H || !T) {
      free(H); free(T);
#pragma omp atomic write
      err = 2;
      continue;
    }
    const float *S = S32 + s_off[b];
    nw_fill(nb, mb, S, gap, H, T);
    int32_t *pb = path + 2 * path_off[b];
    int k = nw_traceback(nb, mb, T, pb);
    score[b] = H[(size_t)nb * (size_t)(mb + 1) + (size_t)mb];
    n_diag[b] = k;
    int32_t *kb = kept + 2 * path_off[b];
    int nk = 0;
    for (int q = 0; q < k; ++q) {
      int i = pb[2 * q], j = pb[2 * q + 1];
      if (S[(int64_t)i * mb + j] >= thr) {
        kb[2 * nk] = i;
        kb[2 * nk + 1] = j;
        ++nk;
      }
    }
    n_kept[b] = nk;
    if (b == 0 && H_out) memcpy(H_out, H, sizeof(float) * cells);
    if (b == 0 && T_out) memcpy(T_out, T, cells);
    free(H);
    free(T);
  }
  return err;
}

/* Backward of L(Score(S, g)) through the logistic scorer, in FP64.
 * The NW score is a maximum of path sums, each path contributing
 * sum_{diag cells} S + g * (#gaps); its (sub)gradient is the optimal path's
 * DIAG indicator P for S and the gap count G = n + m - 2k for g.
 *   dL/dS[i][j] = a_b * P[i][j] + E[i][j]        (E = grad_S_extra, nullable)
 *   dL/dg       = sum_b a_b * G_b
 *   dL/dz       = dL/dS * S (1 - S)              (sigmoid derivative)
 *   dL/d(w0, w1, b) = sum dL/dz * (S_raw, rho, 1)
 * grad_S (nullable) receives dL/dS densely in the S layout. */
int nwo_backward(int B, const int32_t *n, const int32_t *m, const int64_t *s_off,
                 const int64_t *path_off, const int32_t *path, const int32_t *n_diag,
                 const double *grad_score, const double *grad_S_extra,
                 const double *S64, const double *S_raw, const double *rho,
                 double *grad_S, double *grad_gap, double *grad_wb) {
  double gg = 0.0, g0 = 0.0, g1 = 0.0, gb = 0.0;
  for (int b = 0; b < B; ++b) {
    int64_t base = s_off[b];
    int64_t cells = (int64_t)n[b] * m[b];
    double a = grad_score[b];
    int k = n_diag[b];
    gg += a * (double)(n[b] + m[b] - 2 * k);
    if (grad_S) {
      for (int64_t c = 0; c < cells; ++c) grad_S[base + c] = grad_S_extra ? grad_S_extra[base + c] : 0.0;
      for (int q = 0; q < k; ++q) {
        int i = path[2 * (path_off[b] + q)], j = path[2 * (path_off[b] + q) + 1];
        grad_S[base + (int64_t)i * m[b] + j] += a;
      }
    }
    if (grad_S_extra) {
      for (int64_t c = 0; c < cells; ++c) {
        double s = S64[base + c];
        double dz = grad_S_extra[base + c] * s * (1.0 - s);
        g0 += dz * S_raw[base + c];
        g1 += dz * rho[base + c];
        gb += dz;
      }
    }
    for (int q = 0; q < k; ++q) {
      int i = path[2 * (path_off[b] + q)], j = path[2 * (path_off[b] + q) + 1];
      int64_t c = base + (int64_t)i * m[b] + j;
      double s = S64[c];
      double dz = a * s * (1.0 - s);
      g0 += dz * S_raw[c];
      g1 += dz * rho[c];
      gb += dz;
    }
  }
  if (grad_gap) *grad_gap = gg;
  if (grad_wb) {
    grad_wb[0] = g0;
    grad_wb[1] = g1;
    grad_wb[2] = gb;
  }
  return 0;
}
