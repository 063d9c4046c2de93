// Small dense kernels around the ACE build and the localization:
//   * symmetrization, trace and sign flip of M (Appendix A: -M = L L^T);
//   * FP64 Cholesky and triangular inverse of the N_orb x N_orb factor;
//   * the column-pivoted QR pivot search of the SCDM localization;
//   * Newton-Schulz polar iteration for the Loewdin rotation;
//   * screening-pair compaction; pair-energy reduction; conversions.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "ace_internal.h"

namespace ace {

// ---------------------------------------------------------------- M handling
// Msym = (M + M^T)/2 -> out (nullable); negM = -Msym; ex = trace(M).
__global__ void k_symmetrize(const double* __restrict__ M, int n, double* __restrict__ out,
                             double* __restrict__ negM, double* __restrict__ ex, double* __restrict__ asym) {
  __shared__ double red[2][256];
  double tr = 0.0, am = 0.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const double a = M[e], b = M[j * n + i];
    const double v = 0.5 * (a + b);
    if (out) out[e] = v;
    negM[e] = -v;
    if (i == j) tr += a;
    const double d = fabs(a - b);
    am = d > am ? d : am;
  }
  red[0][threadIdx.x] = tr;
  red[1][threadIdx.x] = am;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (ex) ex[0] = red[0][0];
    if (asym) asym[0] = red[1][0];
  }
}

// In-place right-looking Cholesky of the lower triangle of A (n x n, one
// workgroup).  info: 0 ok, k+1 if the pivot of column k is not positive,
// -(k+1) if it is not finite.  The strict upper triangle is zeroed.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int n, int* __restrict__ info) {
  __shared__ double piv;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double d = A[k * n + k];
      if (!isfinite(d)) bad = -(k + 1);
      else if (!(d > 0.0)) bad = k + 1;
      else { piv = sqrt(d); A[k * n + k] = piv; }
    }
    __syncthreads();
    if (bad) break;
    const double inv = 1.0 / piv;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * n + k] *= inv;
    __syncthreads();
    const int m = n - k - 1;  // trailing size
    const int64_t tot = int64_t(m) * (m + 1) / 2;
    for (int64_t t = threadIdx.x; t < tot; t += blockDim.x) {
      // t -> (i, j) with 0 <= j <= i < m  (row-major lower triangle)
      int i = int((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
      while (int64_t(i) * (i + 1) / 2 > t) --i;
      while (int64_t(i + 1) * (i + 2) / 2 <= t) ++i;
      const int j = int(t - int64_t(i) * (i + 1) / 2);
      const int gi = k + 1 + i, gj = k + 1 + j;
      A[gi * n + gj] -= A[gi * n + k] * A[gj * n + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) info[0] = bad;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    if (j > i) A[e] = 0.0;
  }
}

// Inverse of a lower-triangular L (n x n): one thread per column c solves
// L x = e_c by forward substitution; X is lower triangular.
__global__ void k_trinv_lower(const double* __restrict__ L, int n, double* __restrict__ X) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = 0; i < c; ++i) X[i * n + c] = 0.0;
  for (int i = c; i < n; ++i) {
    double s = (i == c) ? 1.0 : 0.0;
    for (int k = c; k < i; ++k) s -= L[i * n + k] * X[k * n + c];
    X[i * n + c] = s / L[i * n + i];
  }
}

// ---------------------------------------------------------------- SCDM pivot search
// Residual column norms res[r] = sum_i A[i][r]^2, A = psi [n][ng].
__global__ void k_colnorm(const double* __restrict__ A, int n, int64_t ng, double* __restrict__ res) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < ng; r += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const double a = A[int64_t(i) * ng + r];
      s += a * a;
    }
    res[r] = s;
  }
}

constexpr int TOPK = 8;

// Is (v, i) ranked before (w, j)?  Larger value first; ties to smaller index.
__device__ __forceinline__ bool ranks_before(double v, int64_t i, double w, int64_t j) {
  return v > w || (v == w && i < j);
}

template <int NT>
__device__ void block_topk(double (&tv)[TOPK], int64_t (&ti)[TOPK], double* outv, int64_t* outi) {
  // repeated block-wide extraction of the best remaining head
  __shared__ double sv[NT / 64];
  __shared__ int64_t si[NT / 64];
  __shared__ int st[NT / 64];
  int head = 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int round = 0; round < TOPK; ++round) {
    double v = head < TOPK ? tv[0] : -INFINITY;
    int64_t idx = head < TOPK ? ti[0] : INT64_MAX;
    // (tv[0], ti[0]) always holds the current head: the list is shifted on pop
    int who = threadIdx.x;
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(v, off, 64);
      const int64_t oi = __shfl_down(idx, off, 64);
      const int ow = __shfl_down(who, off, 64);
      if (ranks_before(ov, oi, v, idx)) { v = ov; idx = oi; who = ow; }
    }
    if (lane == 0) { sv[wv] = v; si[wv] = idx; st[wv] = who; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double bv = sv[0]; int64_t bi = si[0]; int bw = st[0];
      for (int w = 1; w < NT / 64; ++w)
        if (ranks_before(sv[w], si[w], bv, bi)) { bv = sv[w]; bi = si[w]; bw = st[w]; }
      outv[round] = bv; outi[round] = bi;
      st[0] = bw;
    }
    __syncthreads();
    const int winner = st[0];
    __syncthreads();
    if (threadIdx.x == winner) {
#pragma unroll
      for (int q = 0; q < TOPK - 1; ++q) { tv[q] = tv[q + 1]; ti[q] = ti[q + 1]; }
      tv[TOPK - 1] = -INFINITY; ti[TOPK - 1] = INT64_MAX;
      ++head;
    }
  }
}

__device__ __forceinline__ void topk_insert(double (&tv)[TOPK], int64_t (&ti)[TOPK], double v, int64_t i) {
  if (!ranks_before(v, i, tv[TOPK - 1], ti[TOPK - 1])) return;
  tv[TOPK - 1] = v; ti[TOPK - 1] = i;
#pragma unroll
  for (int q = TOPK - 1; q > 0; --q) {
    if (ranks_before(tv[q], ti[q], tv[q - 1], ti[q - 1])) {
      const double a = tv[q]; tv[q] = tv[q - 1]; tv[q - 1] = a;
      const int64_t b = ti[q]; ti[q] = ti[q - 1]; ti[q - 1] = b;
    }
  }
}

// One pivot step, bulk part: ell[r] = q . A[:, r]; res[r] -= ell^2 (if q given);
// then per-block top-8 of res into pv/pi [block][8].
template <int NT>
__global__ __launch_bounds__(NT) void k_qrcp_update(const double* __restrict__ A, int n, int64_t ng,
                                                    const double* __restrict__ q, double* __restrict__ res,
                                                    double* __restrict__ pv, int64_t* __restrict__ pi) {
  __shared__ double qs[1024];
  const bool upd = q != nullptr;
  if (upd)
    for (int i = threadIdx.x; i < n; i += NT) qs[i] = q[i];
  __syncthreads();
  double tv[TOPK];
  int64_t ti[TOPK];
#pragma unroll
  for (int t = 0; t < TOPK; ++t) { tv[t] = -INFINITY; ti[t] = INT64_MAX; }
  for (int64_t r = blockIdx.x * int64_t(NT) + threadIdx.x; r < ng; r += int64_t(gridDim.x) * NT) {
    double v = res[r];
    if (upd) {
      double l = 0.0;
      for (int i = 0; i < n; ++i) l += qs[i] * A[int64_t(i) * ng + r];
      v -= l * l;
      res[r] = v;
    }
    topk_insert(tv, ti, v, r);
  }
  block_topk<NT>(tv, ti, pv + blockIdx.x * TOPK, pi + blockIdx.x * TOPK);
}

// One pivot step, selection part (single workgroup of NT threads):
// merge block candidates -> global top-8; recompute their residuals by
// explicit double projection against Q[0..k); pick the best (ties: smaller
// grid index); append q_k = residual / |residual| to Q; record the pivot and
// retire the column (res = -1).
template <int NT>
__global__ __launch_bounds__(NT) void k_qrcp_select(const double* __restrict__ A, int n, int64_t ng, int k,
                                                    const double* __restrict__ pv, const int64_t* __restrict__ pi,
                                                    int nblk, double* __restrict__ Q, double* __restrict__ res,
                                                    int32_t* __restrict__ piv, double* __restrict__ qout) {
  __shared__ double cv[TOPK];
  __shared__ int64_t ci[TOPK];
  __shared__ double vec[TOPK][512];
  __shared__ double dots[TOPK][512];
  __shared__ double r2[TOPK];
  __shared__ int best;
  {
    double tv[TOPK];
    int64_t ti[TOPK];
#pragma unroll
    for (int t = 0; t < TOPK; ++t) { tv[t] = -INFINITY; ti[t] = INT64_MAX; }
    for (int e = threadIdx.x; e < nblk * TOPK; e += NT) topk_insert(tv, ti, pv[e], pi[e]);
    block_topk<NT>(tv, ti, cv, ci);
  }
  __syncthreads();
  int nc = 0;
  for (int t = 0; t < TOPK; ++t)
    if (ci[t] != INT64_MAX && ci[t] < ng) nc = t + 1;
  // gather candidate columns
  for (int e = threadIdx.x; e < nc * n; e += NT) {
    const int c = e / n, i = e % n;
    vec[c][i] = A[int64_t(i) * ng + ci[c]];
  }
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    // dots[c][m] = Q[m] . vec[c]
    for (int e = threadIdx.x; e < nc * k; e += NT) {
      const int c = e / k, m = e % k;
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += Q[int64_t(m) * n + i] * vec[c][i];
      dots[c][m] = s;
    }
    __syncthreads();
    // vec[c][i] -= sum_m dots[c][m] Q[m][i]
    for (int e = threadIdx.x; e < nc * n; e += NT) {
      const int c = e / n, i = e % n;
      double s = 0.0;
      for (int m = 0; m < k; ++m) s += dots[c][m] * Q[int64_t(m) * n + i];
      vec[c][i] -= s;
    }
    __syncthreads();
  }
  if (threadIdx.x < nc) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += vec[threadIdx.x][i] * vec[threadIdx.x][i];
    r2[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int b = 0;
    for (int c = 1; c < nc; ++c)
      if (ranks_before(r2[c], ci[c], r2[b], ci[b])) b = c;
    best = b;
    piv[k] = int32_t(ci[b]);
    res[ci[b]] = -1.0;
  }
  __syncthreads();
  const double inv = 1.0 / sqrt(r2[best]);
  for (int i = threadIdx.x; i < n; i += NT) {
    const double v = vec[best][i] * inv;
    Q[int64_t(k) * n + i] = v;
    qout[i] = v;
  }
}

// AC[i][k] = A[i][piv[k]]
__global__ void k_gather_cols(const double* __restrict__ A, int n, int64_t ng, const int32_t* __restrict__ piv,
                              double* __restrict__ AC) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int i = e / n, k = e % n;
    AC[e] = A[int64_t(i) * ng + piv[k]];
  }
}

// ---------------------------------------------------------------- Newton-Schulz helpers
// X <- alpha * X (scale by 1/||X||_F computed in one workgroup)
__global__ void k_scale_frob(double* __restrict__ X, int64_t cnt) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) s += X[e] * X[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) X[e] *= inv;
}

// Y <- 1.5 X - 0.5 Z ; also dev = max |G - I| where G = X^T X (given)
__global__ void k_ns_combine(const double* __restrict__ X, const double* __restrict__ Z, double* __restrict__ Y,
                             int64_t cnt) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < cnt; e += int64_t(gridDim.x) * blockDim.x)
    Y[e] = 1.5 * X[e] - 0.5 * Z[e];
}

__global__ void k_dev_identity(const double* __restrict__ G, int n, double* __restrict__ out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    const double d = fabs(G[e] - (i == j ? 1.0 : 0.0));
    m = d > m ? d : m;
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// ---------------------------------------------------------------- screening
// Upper-triangle entries (i <= j) with O_ij >= rho_cut, or i == j, in
// row-major order; writes at most cap pairs and the full count to *count.
__global__ __launch_bounds__(1024) void k_compact_pairs(const double* __restrict__ O, int n, double rho_cut,
                                                        int64_t cap, int32_t* __restrict__ pairs,
                                                        double* __restrict__ ov, int64_t* __restrict__ count) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int64_t tot = int64_t(n) * (n + 1) / 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t c0 = 0; c0 < tot; c0 += blockDim.x) {
    const int64_t t = c0 + threadIdx.x;
    int i = 0, j = 0;
    bool keep = false;
    if (t < tot) {
      // t -> (i, j), i <= j, row-major over the upper triangle
      // row i starts at i*n - i*(i-1)/2
      double a = 2.0 * n + 1.0;
      i = int((a - sqrt(a * a - 8.0 * double(t))) * 0.5);
      while (i > 0 && int64_t(i) * n - int64_t(i) * (i - 1) / 2 > t) --i;
      while (int64_t(i + 1) * n - int64_t(i + 1) * i / 2 <= t) ++i;
      j = i + int(t - (int64_t(i) * n - int64_t(i) * (i - 1) / 2));
      keep = (i == j) || (O[int64_t(i) * n + j] >= rho_cut);
    }
    const unsigned long long m = __ballot(keep);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(m);
    __syncthreads();
    int64_t off = base;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    if (keep) {
      const int64_t p = off + before;
      if (p < cap) {
        pairs[2 * p] = i;
        pairs[2 * p + 1] = j;
        if (ov) ov[p] = O[int64_t(i) * n + j];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t s = 0;
      for (int w = 0; w < int(blockDim.x / 64); ++w) s += wsum[w];
      base += s;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) count[0] = base;
}

// ---------------------------------------------------------------- pair energies
// e[pair] = -(2 - delta_ij) dV sum_blocks epart; pack p carries pairs pa[p], pb[p].
__global__ void k_pair_energy(const double* __restrict__ epart, int npacks, int nblk, const Pack* __restrict__ packs,
                              const int64_t* __restrict__ pidx, double dV, double* __restrict__ e) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npacks) return;
  double sa = 0.0, sb = 0.0;
  for (int b = 0; b < nblk; ++b) {
    sa += epart[2 * (int64_t(p) * nblk + b)];
    sb += epart[2 * (int64_t(p) * nblk + b) + 1];
  }
  const Pack pk = packs[p];
  e[pidx[2 * p]] = -(pk.ia == pk.ja ? 1.0 : 2.0) * dV * sa;
  if (pk.jb >= 0) e[pidx[2 * p + 1]] = -(pk.ib == pk.jb ? 1.0 : 2.0) * dV * sb;
}

// ---------------------------------------------------------------- conversions
__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    b[e] = float(a[e]);
}
__global__ void k_f2d(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    b[e] = double(a[e]);
}
__global__ void k_nonfinite(const double* __restrict__ a, int64_t n, int* __restrict__ flag) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    if (!isfinite(a[e])) flag[0] = 1;
}

// ---------------------------------------------------------------- host launchers
static int grid_for(int64_t n, int nt, int cap = 4096) {
  int64_t g = (n + nt - 1) / nt;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return int(g);
}

void launch_symmetrize(const double* M, int n, double* out, double* negM, double* ex, double* asym, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrize, dim3(1), dim3(256), 0, s, M, n, out, negM, ex, asym);
}
void launch_cholesky(double* A, int n, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, s, A, n, info);
}
void launch_trinv(const double* L, int n, double* X, hipStream_t s) {
  hipLaunchKernelGGL(k_trinv_lower, dim3((n + 63) / 64), dim3(64), 0, s, L, n, X);
}
void launch_colnorm(const double* A, int n, int64_t ng, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_colnorm, dim3(grid_for(ng, 256)), dim3(256), 0, s, A, n, ng, res);
}
int qrcp_blocks(int64_t ng) { return grid_for(ng, 256, 2048); }
void launch_qrcp_update(const double* A, int n, int64_t ng, const double* q, double* res, double* pv, int64_t* pi,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_qrcp_update<256>, dim3(qrcp_blocks(ng)), dim3(256), 0, s, A, n, ng, q, res, pv, pi);
}
void launch_qrcp_select(const double* A, int n, int64_t ng, int k, const double* pv, const int64_t* pi, int nblk,
                        double* Q, double* res, int32_t* piv, double* qout, hipStream_t s) {
  hipLaunchKernelGGL(k_qrcp_select<512>, dim3(1), dim3(512), 0, s, A, n, ng, k, pv, pi, nblk, Q, res, piv, qout);
}
void launch_gather_cols(const double* A, int n, int64_t ng, const int32_t* piv, double* AC, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, s, A, n, ng, piv, AC);
}
void launch_scale_frob(double* X, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_frob, dim3(1), dim3(1024), 0, s, X, cnt);
}
void launch_ns_combine(const double* X, const double* Z, double* Y, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_ns_combine, dim3(grid_for(cnt, 256)), dim3(256), 0, s, X, Z, Y, cnt);
}
void launch_dev_identity(const double* G, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dev_identity, dim3(1), dim3(1024), 0, s, G, n, out);
}
void launch_compact_pairs(const double* O, int n, double rho_cut, int64_t cap, int32_t* pairs, double* ov,
                          int64_t* count, hipStream_t s) {
  hipLaunchKernelGGL(k_compact_pairs, dim3(1), dim3(1024), 0, s, O, n, rho_cut, cap, pairs, ov, count);
}
void launch_pair_energy(const double* epart, int npacks, int nblk, const Pack* packs, const int64_t* pidx, double dV,
                        double* e, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_energy, dim3((npacks + 127) / 128), dim3(128), 0, s, epart, npacks, nblk, packs, pidx,
                     dV, e);
}
void launch_d2f(const double* a, float* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_d2f, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}
void launch_f2d(const float* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_f2d, dim3(grid_for(n, 256)), dim3(256), 0, s, a, b, n);
}
void launch_nonfinite(const double* a, int64_t n, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_nonfinite, dim3(grid_for(n, 256)), dim3(256), 0, s, a, n, flag);
}

}  // namespace ace
