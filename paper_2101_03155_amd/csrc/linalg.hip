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


// ---------------------------------------------------------------- blocked Cholesky
// -M = L L^T for n <= 512, right-looking over panels of CB = 64 columns:
//   diagonal block: factor in LDS and form its inverse (one workgroup);
//   panel:          L21 = A21 L11^-T (rows below the block);
//   update:         A22 -= L21 L21^T (lower 64 x 64 tiles of the trailing matrix).
// Only the lower triangle is read; the strict upper triangle is zeroed.  info
// = k + 1 when the pivot of column k is not positive, -(k + 1) when it is not
// finite; every kernel returns at once when info is already set.
constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ A, int n, int k0,
                                                   double* __restrict__ Tinv, int* __restrict__ info) {
  __shared__ double D[CB][CB + 1];
  __shared__ double X[CB][CB + 1];
  __shared__ double col[2][CB];
  if (*info) return;
  const int b = (n - k0 < CB) ? n - k0 : CB;
  const int tid = threadIdx.x;
  // thread (tr, tc) owns rows 4 tr .. 4 tr + 3 and columns 4 tc .. 4 tc + 3,
  // kept in registers during the elimination
  const int r0 = (tid >> 4) * 4, c0 = (tid & 15) * 4;
  double v[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + a, j = c0 + q;
      v[a][q] = (i < b && j <= i) ? A[int64_t(k0 + i) * n + k0 + j] : 0.0;
    }
  // a_ij -= a_ik a_jk / a_kk on unscaled columns.  Column k is published by
  // the threads that own it to an LDS vector (two alternating buffers, so one
  // barrier per column suffices); every element sees the same updates in the
  // same order as an in-place elimination.
  int bad = 0;
  for (int k = 0; k < b; ++k) {
    double* ck = col[k & 1];
    if ((tid & 15) == (k >> 2)) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (q == (k & 3)) ck[r0 + a] = v[a][q];
    }
    __syncthreads();
    const double d = ck[k];
    if (!isfinite(d)) { bad = -(k0 + k + 1); break; }
    if (!(d > 0.0)) { bad = k0 + k + 1; break; }
    const double inv = 1.0 / d;
    double li[4], lj[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) { li[a] = ck[r0 + a] * inv; lj[a] = ck[c0 + a]; }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = r0 + a, j = c0 + q;
        if (j > k && j <= i) v[a][q] -= li[a] * lj[q];
      }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) D[r0 + a][c0 + q] = v[a][q];
  __syncthreads();
  if (bad) {
    if (tid == 0) *info = bad;
    return;
  }
  // scale: L[i][k] = a_ik / sqrt(a_kk) (zero above the diagonal and beyond b)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + a, k = c0 + q;
      X[i][k] = (i < b && k <= i) ? D[i][k] / sqrt(D[k][k]) : 0.0;
    }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) D[r0 + a][c0 + q] = X[r0 + a][c0 + q];
  __syncthreads();
  // inverse by rows: X[i][c] = (delta_ic - sum_{c <= k < i} L[i][k] X[k][c]) / L[i][i],
  // four lanes per column c, combined with shuffles.  Only the panel below
  // the block reads it, so the last block skips it (uniform over the block).
  const bool last = k0 + b >= n;
  const int c = tid >> 2, part = tid & 3;
  for (int i = 0; i < (last ? 0 : b); ++i) {
    double acc = 0.0;
    if (c < i)
      for (int k = c + part; k < i; k += 4) acc += D[i][k] * X[k][c];
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (part == 0 && c < b) X[i][c] = (c > i) ? 0.0 : (((i == c) ? 1.0 : 0.0) - acc) / D[i][i];
    __syncthreads();
  }
  for (int e = tid; e < b * b; e += 256) {
    const int i = e / b, j = e % b;
    A[int64_t(k0 + i) * n + k0 + j] = D[i][j];
    if (!last) Tinv[i * CB + j] = X[i][j];
  }
  // the strict upper triangle right of the block
  for (int e = tid; e < b * (n - k0 - b); e += 256) {
    const int i = e / (n - k0 - b), j = k0 + b + e % (n - k0 - b);
    A[int64_t(k0 + i) * n + j] = 0.0;
  }
}

// Rows r0 .. r0 + 63 (below the block): L21[i][c] = sum_{d <= c} A21[i][d] Tinv[c][d].
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ A, int n, int k0,
                                                    const double* __restrict__ Tinv, const int* __restrict__ info) {
  __shared__ double T[CB][CB + 1];
  __shared__ double R[CB][CB + 1];
  if (*info) return;
  const int b = (n - k0 < CB) ? n - k0 : CB;
  const int r0 = k0 + b + blockIdx.x * CB;
  const int rows = (n - r0 < CB) ? n - r0 : CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += 256) {
    const int i = e / CB, j = e % CB;
    T[i][j] = (i < b && j < b) ? Tinv[i * CB + j] : 0.0;
    R[i][j] = (i < rows && j < b) ? A[int64_t(r0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < rows * b; e += 256) {
    const int i = e / b, c = e % b;
    double acc = 0.0;
    for (int d = 0; d <= c; ++d) acc += R[i][d] * T[c][d];
    A[int64_t(r0 + i) * n + k0 + c] = acc;
  }
}

// Trailing update of the lower 64 x 64 tile (ti, tj), tj <= ti, of rows and
// columns from k0 + b: A[i][j] -= sum_c L21[i][c] L21[j][c] for j <= i.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ A, int n, int k0,
                                                     const int* __restrict__ info) {
  __shared__ double Li[CB][CB + 1];
  __shared__ double Lj[CB][CB + 1];
  if (*info) return;
  const int b = (n - k0 < CB) ? n - k0 : CB;
  const int base = k0 + b;
  int t = blockIdx.x, ti = 0;
  while (t > ti) { t -= ti + 1; ++ti; }
  const int tj = t;
  const int i0 = base + ti * CB, j0 = base + tj * CB;
  const int ri = (n - i0 < CB) ? n - i0 : CB, rj = (n - j0 < CB) ? n - j0 : CB;
  const int tid = threadIdx.x;
  for (int e = tid; e < CB * CB; e += 256) {
    const int r = e / CB, c = e % CB;
    Li[r][c] = (r < ri && c < b) ? A[int64_t(i0 + r) * n + k0 + c] : 0.0;
    Lj[r][c] = (r < rj && c < b) ? A[int64_t(j0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < ri * rj; e += 256) {
    const int r = e / rj, q = e % rj;
    if (j0 + q > i0 + r) continue;
    double acc = 0.0;
    for (int c = 0; c < b; ++c) acc += Li[r][c] * Lj[q][c];
    A[int64_t(i0 + r) * n + j0 + q] -= acc;
  }
}

// For n <= 128 the factorization and the inverse in one workgroup with the
// matrix resident in LDS.  A (n x n, lower triangle read) = L L^T, X = L^-1
// (lower triangular, zeros above the diagonal).  Right-looking over panels
// of 16 columns: wave 0 factors a panel in registers (lane l holds panel
// rows k0 + l and k0 + l + 64, the pivot column passed through LDS), then
// all threads apply the panel to the trailing lower triangle in 4 x 4
// blocks.  The inverse runs by 16-row block rows: the diagonal blocks'
// inverses by substitution, one thread per column, then each block row from
// the ones above it (all its blocks at once).  Both triangles sit packed in
// LDS (row i at i (i + 1) / 2).  info as the blocked factorization: k + 1 for a
// non-positive pivot in column k, -(k + 1) for a non-finite one.
constexpr int SMALL_N = 128;
__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }

__global__ __launch_bounds__(1024) void k_chol_inv_small(const double* __restrict__ A, int n, int* __restrict__ info,
                                                         double* __restrict__ X) {
  constexpr int PB = 16, NP = SMALL_N * (SMALL_N + 1) / 2;
  __shared__ double S[NP];
  __shared__ double XP[NP];
  __shared__ double T[(SMALL_N / 16 - 1) * 256];
  __shared__ double pc[17];
  __shared__ int sbad;
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) sbad = 0;
  for (int e = tid; e < n * (n + 1) / 2; e += 1024) {
    // row i of the packed triangle holds elements i (i + 1) / 2 .. + i
    int i = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > e) --i;
    while ((i + 1) * (i + 2) / 2 <= e) ++i;
    const int j = e - i * (i + 1) / 2;
    S[e] = A[int64_t(i) * n + j];
  }
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += PB) {
    const int kb = n - k0 < PB ? n - k0 : PB;
    if (tid < 64) {
      const int r0 = k0 + lane, r1 = k0 + lane + 64;
      double v0[PB], v1[PB];
#pragma unroll
      for (int jj = 0; jj < PB; ++jj) {
        v0[jj] = (jj < kb && r0 < n && k0 + jj <= r0) ? S[pk(r0, k0 + jj)] : 0.0;
        v1[jj] = (jj < kb && r1 < n && k0 + jj <= r1) ? S[pk(r1, k0 + jj)] : 0.0;
      }
      // the pivot and the scaled pivot column inside the panel reach the
      // other lanes through pc[] (one wave: its LDS accesses run in order)
      int bad = 0;
#pragma unroll
      for (int kk = 0; kk < PB; ++kk) {
        if (kk < kb && !bad) {
          const int k = k0 + kk;
          if (lane == kk) pc[0] = v0[kk];
          __builtin_amdgcn_wave_barrier();
          const double d = pc[0];
          if (!isfinite(d)) bad = -(k + 1);
          else if (!(d > 0.0)) bad = k + 1;
          if (!bad) {
            const double r = sqrt(d), inv = 1.0 / r;
            if (r0 > k) v0[kk] *= inv;
            else if (r0 == k) v0[kk] = r;
            if (r1 < n) v1[kk] *= inv;  // r1 >= k0 + 64 > k
            if (lane > kk && lane < PB) pc[1 + lane] = v0[kk];  // L[k0 + lane][k]
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int jj = kk + 1; jj < PB; ++jj) {
              if (jj < kb) {
                const double lj = pc[1 + jj];
                if (r0 >= k0 + jj) v0[jj] -= v0[kk] * lj;
                if (r1 < n) v1[jj] -= v1[kk] * lj;
              }
            }
          }
          __builtin_amdgcn_wave_barrier();
        }
      }
#pragma unroll
      for (int jj = 0; jj < PB; ++jj) {
        if (jj < kb && r0 < n && k0 + jj <= r0) S[pk(r0, k0 + jj)] = v0[jj];
        if (jj < kb && r1 < n) S[pk(r1, k0 + jj)] = v1[jj];
      }
      if (lane == 0 && bad) sbad = bad;
    }
    __syncthreads();
    if (sbad) break;
    // trailing update S[i][j] -= sum_kk L[i][k0 + kk] L[j][k0 + kk], k0 + kb <= j <= i < n
    const int t0 = k0 + kb, nt = (n - t0 + 3) / 4;
    for (int b = tid; b < nt * (nt + 1) / 2; b += 1024) {
      int bi = int((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
      while (bi * (bi + 1) / 2 > b) --bi;
      while ((bi + 1) * (bi + 2) / 2 <= b) ++bi;
      const int bj = b - bi * (bi + 1) / 2;
      const int i0 = t0 + 4 * bi, j0 = t0 + 4 * bj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[a][q] = 0.0;
      for (int kk = 0; kk < kb; ++kk) {
        double li[4], lj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          li[a] = i0 + a < n ? S[pk(i0 + a, k0 + kk)] : 0.0;
          lj[a] = j0 + a < n ? S[pk(j0 + a, k0 + kk)] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[a][q] += li[a] * lj[q];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + a, j = j0 + q;
          if (i < n && j <= i) S[pk(i, j)] -= acc[a][q];
        }
    }
    __syncthreads();
  }
  if (sbad) {
    if (tid == 0) *info = sbad;
    return;
  }
  // X = L^-1 by 16-row block rows.  First the inverses of the diagonal
  // blocks, one thread per column (forward substitution within the block),
  // into X's diagonal blocks; then for each block row I: T_IJ = sum over
  // K = J .. I-1 of L_IK X_KJ for every J < I, and X_IJ = -X_II T_IJ.
  {
    const int b = tid >> 4, lc = tid & 15, r0 = b * 16;
    if (tid < n) {
      const int m = n - r0 < 16 ? n - r0 : 16;  // rows of this diagonal block
      double x[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double v = 0.0;
        if (r >= lc && r < m) {
          double acc = r == lc ? 1.0 : 0.0;
#pragma unroll
          for (int t = 0; t < 16; ++t)
            if (t >= lc && t < r) acc -= S[pk(r0 + r, r0 + t)] * x[t];
          v = acc / S[pk(r0 + r, r0 + r)];
          XP[pk(r0 + r, r0 + lc)] = v;
        }
        x[r] = v;
      }
    }
  }
  __syncthreads();
  for (int I = 1; I * 16 < n; ++I) {
    const int i0 = I * 16, m = n - i0 < 16 ? n - i0 : 16;
    for (int f = tid; f < I * 256; f += 1024) {
      const int J = f >> 8, r = (f >> 4) & 15, q = f & 15, col = J * 16 + q;
      double acc = 0.0;
      if (r < m)
        for (int k = col; k < i0; ++k) acc += S[pk(i0 + r, k)] * XP[pk(k, col)];
      T[f] = acc;
    }
    __syncthreads();
    for (int f = tid; f < I * 256; f += 1024) {
      const int J = f >> 8, r = (f >> 4) & 15, q = f & 15;
      if (r < m) {
        double acc = 0.0;
        for (int t = 0; t <= r; ++t) acc += XP[pk(i0 + r, i0 + t)] * T[(J << 8) + (t << 4) + q];
        XP[pk(i0 + r, J * 16 + q)] = -acc;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < n * n; e += 1024) {
    const int i = e / n, j = e % n;
    X[e] = j <= i ? XP[pk(i, j)] : 0.0;
  }
}

// Inverse of a lower-triangular L (n x n, n <= 512): one 64-lane wave per
// column c solves L x = e_c by forward substitution, each step a wave-wide
// dot product; x lives in LDS.  X is lower triangular.
__global__ __launch_bounds__(64) void k_trinv_lower(const double* __restrict__ L, int n, double* __restrict__ X) {
  __shared__ double x[512];
  const int c = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) x[i] = 0.0;
  __syncthreads();
  for (int i = c; i < n; ++i) {
    double s = 0.0;
    for (int k = c + lane; k < i; k += 64) s += L[int64_t(i) * n + k] * x[k];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[i] = ((i == c ? 1.0 : 0.0) - s) / L[int64_t(i) * n + i];
    __syncthreads();
  }
  for (int i = lane; i < n; i += 64) X[int64_t(i) * n + c] = x[i];
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
// then per-block top-8 of res into pv/pi [block][8].  A is [n][ng]: either
// the orbitals themselves or a compact pool of candidate columns.  A set stop
// flag turns the launch into a no-op.
template <int NT>
__global__ __launch_bounds__(NT) void k_qrcp_update(const double* __restrict__ A, int n, int64_t ng,
                                                    const double* __restrict__ q, double* __restrict__ res,
                                                    double* __restrict__ pv, int64_t* __restrict__ pi,
                                                    const int* __restrict__ stop) {
  if (stop && *stop) return;
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
// column index); append q_k = residual / |residual| to Q; record the pivot and
// retire the column (res = -1).
//
// k is read from and advanced in device memory.  With a candidate pool
// (pool != nullptr, columns sorted by grid index), the pick is accepted only
// if its exact residual is at least t_out, an upper bound of every residual
// outside the pool; otherwise the stop flag is raised and the host refreshes
// the pool.  A raised stop flag turns the launch into a no-op.
template <int NT>
__global__ __launch_bounds__(NT) void k_qrcp_select(const double* __restrict__ A, int n, int64_t ng,
                                                    int* __restrict__ kdev, const double* __restrict__ pv,
                                                    const int64_t* __restrict__ pi, int nblk, double* __restrict__ Q,
                                                    double* __restrict__ res, int32_t* __restrict__ piv,
                                                    double* __restrict__ qout, const int32_t* __restrict__ pool,
                                                    const double* __restrict__ t_out, int* __restrict__ stop) {
  if (*stop) return;
  __shared__ double cv[TOPK];
  __shared__ int64_t ci[TOPK];
  __shared__ double vec[TOPK][512];
  __shared__ double dots[TOPK][512];
  __shared__ double part[TOPK * NT];
  constexpr int QCH = 4096;
  __shared__ double Qs[QCH];
  __shared__ double r2[TOPK];
  __shared__ int best, accept;
  const int k = *kdev;
  {
    double tv[TOPK];
    int64_t ti[TOPK];
#pragma unroll
    for (int t = 0; t < TOPK; ++t) { tv[t] = -INFINITY; ti[t] = INT64_MAX; }
    for (int e = threadIdx.x; e < nblk * TOPK; e += NT) topk_insert(tv, ti, pv[e], pi[e]);
    block_topk<NT>(tv, ti, cv, ci);
  }
  __syncthreads();
  // valid candidates: real columns that are not retired (res = -1)
  int nc = 0;
  for (int t = 0; t < TOPK; ++t)
    if (ci[t] != INT64_MAX && ci[t] < ng && cv[t] > -0.5) nc = t + 1;
  if (nc == 0) {
    if (threadIdx.x == 0) *stop = 1;
    return;
  }
  for (int e = threadIdx.x; e < TOPK * n; e += NT) {
    const int c = e / n, i = e % n;
    vec[c][i] = c < nc ? A[int64_t(i) * ng + ci[c]] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int NW = NT / 64;
  // Q is read in chunks of mc rows staged through LDS (coalesced bulk loads)
  const int mc = QCH / n;
  const int G = NT / n;
  const int g = threadIdx.x / n, gi = threadIdx.x % n;
  for (int pass = 0; pass < 2; ++pass) {
    // dots[c][m] = Q[m] . vec[c]: one wave per row, lanes across i
    for (int m0 = 0; m0 < k; m0 += mc) {
      const int rows = (k - m0 < mc) ? k - m0 : mc;
      for (int e = threadIdx.x; e < rows * n; e += NT) Qs[e] = Q[int64_t(m0) * n + e];
      __syncthreads();
      for (int r = wv; r < rows; r += NW) {
        double acc[TOPK];
#pragma unroll
        for (int c = 0; c < TOPK; ++c) acc[c] = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double qv = Qs[r * n + i];
#pragma unroll
          for (int c = 0; c < TOPK; ++c) acc[c] += qv * vec[c][i];
        }
#pragma unroll
        for (int c = 0; c < TOPK; ++c) {
          double v = acc[c];
          for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
          if (lane == 0) dots[c][m0 + r] = v;
        }
      }
      __syncthreads();
    }
    // vec[c][i] -= sum_m dots[c][m] Q[m][i]: G thread groups split the rows,
    // their partial sums meet in LDS
    double acc[TOPK];
#pragma unroll
    for (int c = 0; c < TOPK; ++c) acc[c] = 0.0;
    for (int m0 = 0; m0 < k; m0 += mc) {
      const int rows = (k - m0 < mc) ? k - m0 : mc;
      for (int e = threadIdx.x; e < rows * n; e += NT) Qs[e] = Q[int64_t(m0) * n + e];
      __syncthreads();
      if (g < G)
        for (int r = g; r < rows; r += G) {
          const double qv = Qs[r * n + gi];
#pragma unroll
          for (int c = 0; c < TOPK; ++c) acc[c] += dots[c][m0 + r] * qv;
        }
      __syncthreads();
    }
    if (g < G) {
#pragma unroll
      for (int c = 0; c < TOPK; ++c) part[(g * TOPK + c) * n + gi] = acc[c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < TOPK * n; e += NT) {
      const int c = e / n, ii = e % n;
      double sum = 0.0;
      for (int gg = 0; gg < G; ++gg) sum += part[(gg * TOPK + c) * n + ii];
      vec[c][ii] -= sum;
    }
    __syncthreads();
  }
  // squared residual norms: one wave per candidate
  for (int c = wv; c < TOPK; c += NW) {
    double v = 0.0;
    for (int i = lane; i < n; i += 64) v += vec[c][i] * vec[c][i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) r2[c] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int b = 0;
    for (int c = 1; c < nc; ++c)
      if (ranks_before(r2[c], ci[c], r2[b], ci[b])) b = c;
    best = b;
    const bool ok = (t_out == nullptr) || (r2[b] >= *t_out);
    accept = ok ? 1 : 0;
    if (ok) {
      piv[k] = pool ? pool[ci[b]] : int32_t(ci[b]);
      res[ci[b]] = -1.0;
    } else {
      *stop = 1;
    }
  }
  __syncthreads();
  if (!accept) return;
  const double inv = 1.0 / sqrt(r2[best]);
  for (int i = threadIdx.x; i < n; i += NT) {
    const double v = vec[best][i] * inv;
    Q[int64_t(k) * n + i] = v;
    qout[i] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) *kdev = k + 1;
}

// ---------------------------------------------------------------- pool steps on explicit residuals
// On a candidate pool the residual columns are kept explicitly,
// R = (I - Q^T Q) A_pool ([n][P], row-major), so every step's norms are exact
// and no re-ranking against Q is needed: with the new direction q,
// l_c = q . R[:,c], R[:,c] -= q l_c, res_c = |R[:,c]|^2.

// Best (value, index) of the block, ties to the smaller index; result in
// out[0], idx_out[0] (shared) for every thread after the call.
template <int NT>
__device__ void block_top1(double v, int64_t idx, double* outv, int64_t* outi) {
  __shared__ double sv[NT / 64];
  __shared__ int64_t si[NT / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_down(v, off, 64);
    const int64_t oi = __shfl_down(idx, off, 64);
    if (ranks_before(ov, oi, v, idx)) { v = ov; idx = oi; }
  }
  if (lane == 0) { sv[wv] = v; si[wv] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double bv = sv[0];
    int64_t bi = si[0];
    for (int w = 1; w < NT / 64; ++w)
      if (ranks_before(sv[w], si[w], bv, bi)) { bv = sv[w]; bi = si[w]; }
    *outv = bv;
    *outi = bi;
  }
  __syncthreads();
}

// One update of the pool residuals (q == nullptr: only the norms).  A block
// covers CW columns with NT/CW row groups (a wave reads CW-column row
// segments); partial sums meet in LDS in a fixed order.  Retired columns
// (res = -1) are skipped.  Writes the block's best live column to
// pv[blockIdx.x], pi[blockIdx.x].
template <int NT, int CW>
__global__ __launch_bounds__(NT) void k_qrcp_update_r(double* __restrict__ R, int n, int P,
                                                      const double* __restrict__ q, double* __restrict__ res,
                                                      double* __restrict__ pv, int64_t* __restrict__ pi,
                                                      const int* __restrict__ stop) {
  if (*stop) return;
  constexpr int RG = NT / CW;
  __shared__ double qs[1024];
  __shared__ double red[RG][CW];
  __shared__ double bv;
  __shared__ int64_t bi;
  const int lane = threadIdx.x % CW, g = threadIdx.x / CW;
  const int c = blockIdx.x * CW + lane;
  const bool upd = q != nullptr;
  if (upd)
    for (int i = threadIdx.x; i < n; i += NT) qs[i] = q[i];
  const bool live = c < P && res[c] > -0.5;
  __syncthreads();
  double* col = R + c;
  double l = 0.0;
  if (upd) {
    if (live) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = g;
      for (; i + 3 * RG < n; i += 4 * RG) {
        a0 += qs[i] * col[int64_t(i) * P];
        a1 += qs[i + RG] * col[int64_t(i + RG) * P];
        a2 += qs[i + 2 * RG] * col[int64_t(i + 2 * RG) * P];
        a3 += qs[i + 3 * RG] * col[int64_t(i + 3 * RG) * P];
      }
      for (; i < n; i += RG) a0 += qs[i] * col[int64_t(i) * P];
      l = (a0 + a1) + (a2 + a3);
    }
    red[g][lane] = l;
    __syncthreads();
    l = 0.0;
#pragma unroll
    for (int h = 0; h < RG; ++h) l += red[h][lane];
    __syncthreads();
  }
  double v = 0.0;
  if (live) {
    double v0 = 0.0, v1 = 0.0;
    int i = g;
    for (; i + RG < n; i += 2 * RG) {
      double x0 = col[int64_t(i) * P], x1 = col[int64_t(i + RG) * P];
      if (upd) {
        x0 -= qs[i] * l;
        x1 -= qs[i + RG] * l;
        col[int64_t(i) * P] = x0;
        col[int64_t(i + RG) * P] = x1;
      }
      v0 += x0 * x0;
      v1 += x1 * x1;
    }
    for (; i < n; i += RG) {
      double x = col[int64_t(i) * P];
      if (upd) {
        x -= qs[i] * l;
        col[int64_t(i) * P] = x;
      }
      v0 += x * x;
    }
    v = v0 + v1;
  }
  red[g][lane] = v;
  __syncthreads();
  double cand = -INFINITY;
  int64_t cidx = INT64_MAX;
  if (g == 0) {
    v = 0.0;
#pragma unroll
    for (int h = 0; h < RG; ++h) v += red[h][lane];
    if (live) {
      res[c] = v;
      cand = v;
      cidx = c;
    }
  }
  block_top1<NT>(cand, cidx, &bv, &bi);
  if (threadIdx.x == 0) {
    pv[blockIdx.x] = bv;
    pi[blockIdx.x] = bi;
  }
}

// Selection on the pool (single workgroup): the best block candidate is the
// best live column; its norm is recomputed, certified against t_out (an upper
// bound of every residual outside the pool), and q_k = R[:,b] / |R[:,b]| is
// appended to Q.  A failed certification or an exhausted pool raises the
// stop flag, after which the queued steps are no-ops.
template <int NT>
__global__ __launch_bounds__(NT) void k_qrcp_select_r(const double* __restrict__ R, int n, int P,
                                                      int* __restrict__ kdev, const double* __restrict__ pv,
                                                      const int64_t* __restrict__ pi, int nblk,
                                                      double* __restrict__ Q, double* __restrict__ res,
                                                      int32_t* __restrict__ piv, double* __restrict__ qout,
                                                      const int32_t* __restrict__ pool,
                                                      const double* __restrict__ t_out, int* __restrict__ stop) {
  if (*stop) return;
  __shared__ double bv;
  __shared__ int64_t bi;
  __shared__ double r2s[NT / 64];
  __shared__ int accept;
  const int k = *kdev;
  {
    double v = -INFINITY;
    int64_t idx = INT64_MAX;
    for (int e = threadIdx.x; e < nblk; e += NT)
      if (ranks_before(pv[e], pi[e], v, idx)) { v = pv[e]; idx = pi[e]; }
    block_top1<NT>(v, idx, &bv, &bi);
  }
  const int64_t b = bi;
  if (b < 0 || b >= P) {
    if (threadIdx.x == 0) *stop = 1;
    return;
  }
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) {
    const double x = R[int64_t(i) * P + b];
    v += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) r2s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r2 = 0.0;
    for (int w = 0; w < NT / 64; ++w) r2 += r2s[w];
    r2s[0] = r2;
    const bool ok = r2 > 0.0 && (t_out == nullptr || r2 >= *t_out);
    accept = ok ? 1 : 0;
    if (ok) {
      piv[k] = pool[b];
      res[b] = -1.0;
    } else {
      *stop = 1;
    }
  }
  __syncthreads();
  if (!accept) return;
  const double inv = 1.0 / sqrt(r2s[0]);
  for (int i = threadIdx.x; i < n; i += NT) {
    const double x = R[int64_t(i) * P + b] * inv;
    Q[int64_t(k) * n + i] = x;
    qout[i] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) *kdev = k + 1;
}

// One pool step in one launch: every block repeats the selection (the best
// of the previous step's block candidates pv_in/pi_in, its norm recomputed
// and certified against t_out, q = R[:,b] / |R[:,b]| in LDS) with the same
// reductions as k_qrcp_select_r, so all blocks hold the same q; block 0
// alone appends q to Q, records the pivot, retires the column and advances
// the step counter.  Then each block updates its columns as
// k_qrcp_update_r does and writes its best live column to pv_out/pi_out
// (candidates double buffered: blocks of this launch still read pv_in).  The
// pivot column itself is left untouched, so the blocks that read it are not
// racing with its owner.  A failed certification or an exhausted pool
// raises the stop flag (block 0), and every block returns.
template <int NT, int CW, int MP>
__global__ __launch_bounds__(NT) void k_qrcp_step_r(double* __restrict__ R, int n, int P, int* __restrict__ kdev,
                                                    const double* __restrict__ pv_in,
                                                    const int64_t* __restrict__ pi_in, int nblk,
                                                    double* __restrict__ Q, double* __restrict__ res,
                                                    int32_t* __restrict__ piv, const int32_t* __restrict__ pool,
                                                    const double* __restrict__ t_out, int* __restrict__ stop,
                                                    double* __restrict__ pv_out, int64_t* __restrict__ pi_out) {
  constexpr int RG = NT / CW;
  __shared__ double qs[1024];
  __shared__ double red[RG][CW];
  __shared__ double r2s[NT / 64];
  __shared__ double bv;
  __shared__ int64_t bi;
  // The block's residual tile (its CW columns, rows g + m RG) and their
  // bounds are loaded first: no block writes them before this block does,
  // so the loads stay in flight through the selection.
  const int lane = threadIdx.x % CW, g = threadIdx.x / CW;
  const int c = blockIdx.x * CW + lane;
  const bool inb = c < P;
  const int nm = g < n ? (n - g + RG - 1) / RG : 0;  // rows of this thread
  double xr[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m)
    if (inb && m < nm) xr[m] = R[int64_t(g + m * RG) * P + c];
  const double rc = inb ? res[c] : -1.0;
  if (*stop) return;
  // selection, as k_qrcp_select_r
  {
    double v = -INFINITY;
    int64_t idx = INT64_MAX;
    for (int e = threadIdx.x; e < nblk; e += NT)
      if (ranks_before(pv_in[e], pi_in[e], v, idx)) { v = pv_in[e]; idx = pi_in[e]; }
    block_top1<NT>(v, idx, &bv, &bi);
  }
  const int64_t b = bi;
  if (b < 0 || b >= P) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *stop = 1;
    return;
  }
  {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) {
      const double x = R[int64_t(i) * P + b];
      v += x * x;
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) r2s[threadIdx.x >> 6] = v;
  }
  __syncthreads();
  double r2 = 0.0;
  for (int w = 0; w < NT / 64; ++w) r2 += r2s[w];
  const bool ok = r2 > 0.0 && (t_out == nullptr || r2 >= *t_out);
  if (!ok) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *stop = 1;
    return;
  }
  const double inv = 1.0 / sqrt(r2);
  for (int i = threadIdx.x; i < n; i += NT) qs[i] = R[int64_t(i) * P + b] * inv;
  __syncthreads();
  if (blockIdx.x == 0) {
    const int k = *kdev;
    for (int i = threadIdx.x; i < n; i += NT) Q[int64_t(k) * n + i] = qs[i];
    if (threadIdx.x == 0) {
      piv[k] = pool[b];
      res[b] = -1.0;
      *kdev = k + 1;
    }
  }
  // update, as k_qrcp_update_r with q (the same sums in the same order)
  const bool live = inb && c != b && rc > -0.5;
  double* col = R + c;
  double l = 0.0;
  if (live) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int m0 = 0;
#pragma unroll
    for (int m = 0; m + 3 < MP; m += 4)
      if (m + 3 < nm) {
        a0 += qs[g + m * RG] * xr[m];
        a1 += qs[g + (m + 1) * RG] * xr[m + 1];
        a2 += qs[g + (m + 2) * RG] * xr[m + 2];
        a3 += qs[g + (m + 3) * RG] * xr[m + 3];
        m0 = m + 4;
      }
#pragma unroll
    for (int m = 0; m < MP; ++m)
      if (m >= m0 && m < nm) a0 += qs[g + m * RG] * xr[m];
    l = (a0 + a1) + (a2 + a3);
  }
  red[g][lane] = l;
  __syncthreads();
  l = 0.0;
#pragma unroll
  for (int h = 0; h < RG; ++h) l += red[h][lane];
  __syncthreads();
  double v = 0.0;
  if (live) {
    double v0 = 0.0, v1 = 0.0;
    int m0 = 0;
#pragma unroll
    for (int m = 0; m + 1 < MP; m += 2)
      if (m + 1 < nm) {
        double x0 = xr[m], x1 = xr[m + 1];
        x0 -= qs[g + m * RG] * l;
        x1 -= qs[g + (m + 1) * RG] * l;
        col[int64_t(g + m * RG) * P] = x0;
        col[int64_t(g + (m + 1) * RG) * P] = x1;
        v0 += x0 * x0;
        v1 += x1 * x1;
        m0 = m + 2;
      }
#pragma unroll
    for (int m = 0; m < MP; ++m)
      if (m >= m0 && m < nm) {
        double x = xr[m];
        x -= qs[g + m * RG] * l;
        col[int64_t(g + m * RG) * P] = x;
        v0 += x * x;
      }
    v = v0 + v1;
  }
  red[g][lane] = v;
  __syncthreads();
  double cand = -INFINITY;
  int64_t cidx = INT64_MAX;
  if (g == 0) {
    v = 0.0;
#pragma unroll
    for (int h = 0; h < RG; ++h) v += red[h][lane];
    if (live) {
      res[c] = v;
      cand = v;
      cidx = c;
    }
  }
  block_top1<NT>(cand, cidx, &bv, &bi);
  if (threadIdx.x == 0) {
    pv_out[blockIdx.x] = bv;
    pi_out[blockIdx.x] = bi;
  }
}

// a += b (elementwise)
__global__ void k_add_inplace(double* __restrict__ a, const double* __restrict__ b, int64_t cnt) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < cnt; e += int64_t(gridDim.x) * blockDim.x)
    a[e] += b[e];
}

// ---------------------------------------------------------------- candidate pool
// The pool holds every column whose residual bound is at least a threshold t
// picked from a histogram of the top 14 bits of the (positive) residuals, so
// that the pool has at most pmax columns.  t_out = the largest residual
// below t bounds every column left out.
constexpr int HBIN = 1 << 14;

__device__ __forceinline__ int res_bin(double v) { return int(__double_as_longlong(v) >> 49); }

__global__ __launch_bounds__(256) void k_res_hist(const double* __restrict__ res, int64_t ng,
                                                  unsigned* __restrict__ hist) {
  __shared__ unsigned h[HBIN];
  for (int i = threadIdx.x; i < HBIN; i += 256) h[i] = 0u;
  __syncthreads();
  for (int64_t r = blockIdx.x * int64_t(256) + threadIdx.x; r < ng; r += int64_t(gridDim.x) * 256) {
    const double v = res[r];
    if (v > 0.0) atomicAdd(&h[res_bin(v)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < HBIN; i += 256)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Lowest bin b such that the columns in bins >= b number at most pmax;
// t = lower edge of bin b (as a double).
__global__ __launch_bounds__(1024) void k_pool_threshold(const unsigned* __restrict__ hist, int pmax,
                                                         double* __restrict__ t) {
  constexpr int SEG = HBIN / 1024;
  __shared__ unsigned long long above[1024];
  __shared__ int tb;
  unsigned long long seg = 0;
  for (int b = 0; b < SEG; ++b) seg += hist[threadIdx.x * SEG + b];
  above[threadIdx.x] = seg;
  if (threadIdx.x == 0) tb = 0;
  __syncthreads();
  // inclusive suffix sum over segments
  for (int off = 1; off < 1024; off <<= 1) {
    unsigned long long v = (threadIdx.x + off < 1024) ? above[threadIdx.x + off] : 0ull;
    __syncthreads();
    above[threadIdx.x] += v;
    __syncthreads();
  }
  const unsigned long long incl = above[threadIdx.x];
  const unsigned long long excl = incl - seg;  // columns in higher segments
  if (excl <= (unsigned long long)pmax && incl > (unsigned long long)pmax) {
    unsigned long long c = excl;
    int pick = threadIdx.x * SEG + SEG;
    for (int b = threadIdx.x * SEG + SEG - 1; b >= threadIdx.x * SEG; --b) {
      if (c + hist[b] > (unsigned long long)pmax) break;
      c += hist[b];
      pick = b;
    }
    tb = pick;
  }
  __syncthreads();
  // tb == HBIN: not even the top bin fits; an infinite threshold empties the pool
  if (threadIdx.x == 0) t[0] = tb >= HBIN ? INFINITY : __longlong_as_double((long long)tb << 49);
}

// Per block (contiguous chunk of columns): count of res >= t, max of 0 < res < t.
__global__ __launch_bounds__(256) void k_pool_count(const double* __restrict__ res, int64_t ng, int64_t chunk,
                                                    const double* __restrict__ t, int64_t* __restrict__ cnt,
                                                    double* __restrict__ tmax) {
  __shared__ int64_t sc[256];
  __shared__ double sm[256];
  const double th = t[0];
  const int64_t r0 = int64_t(blockIdx.x) * chunk;
  const int64_t r1 = (r0 + chunk < ng) ? r0 + chunk : ng;
  int64_t c = 0;
  double m = 0.0;
  for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
    const double v = res[r];
    if (v >= th && v > 0.0) ++c;
    else if (v > 0.0 && v > m) m = v;
  }
  sc[threadIdx.x] = c;
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      sc[threadIdx.x] += sc[threadIdx.x + h];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { cnt[blockIdx.x] = sc[0]; tmax[blockIdx.x] = sm[0]; }
}

// Exclusive scan of the block counts (in place), total count and t_out.
__global__ __launch_bounds__(1024) void k_pool_scan(int64_t* __restrict__ cnt, const double* __restrict__ tmax,
                                                    int nblk, int* __restrict__ total, double* __restrict__ t_out) {
  __shared__ int64_t s[1024];
  __shared__ double m[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  double mx = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 1024) mx = fmax(mx, tmax[b]);
  m[threadIdx.x] = mx;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (threadIdx.x < h) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + h]);
    __syncthreads();
  }
  for (int base = 0; base < nblk; base += 1024) {
    const int b = base + threadIdx.x;
    const int64_t v = b < nblk ? cnt[b] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int64_t u = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += u;
      __syncthreads();
    }
    if (b < nblk) cnt[b] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) { total[0] = int(carry); t_out[0] = m[0]; }
}

// Ordered compaction: pool[off..] = columns with res >= t, by increasing index.
__global__ __launch_bounds__(256) void k_pool_write(const double* __restrict__ res, int64_t ng, int64_t chunk,
                                                    const double* __restrict__ t, const int64_t* __restrict__ off,
                                                    int32_t* __restrict__ pool, double* __restrict__ pres) {
  __shared__ int wsum[4];
  __shared__ int64_t base;
  const double th = t[0];
  const int64_t r0 = int64_t(blockIdx.x) * chunk;
  const int64_t r1 = (r0 + chunk < ng) ? r0 + chunk : ng;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) base = off[blockIdx.x];
  __syncthreads();
  for (int64_t c0 = r0; c0 < r1; c0 += 256) {
    const int64_t r = c0 + threadIdx.x;
    double v = 0.0;
    bool keep = false;
    if (r < r1) {
      v = res[r];
      keep = v >= th && v > 0.0;
    }
    const unsigned long long bal = __ballot(keep);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int64_t o = base;
    for (int w = 0; w < wv; ++w) o += wsum[w];
    if (keep) {
      pool[o + before] = int32_t(r);
      pres[o + before] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) base += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
  }
}

// Apool[i][p] = A[i][pool[p]]
__global__ void k_pool_gather(const double* __restrict__ A, int n, int64_t ng, const int32_t* __restrict__ pool,
                              int np, double* __restrict__ Apool) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < int64_t(n) * np;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int i = int(e / np), p = int(e % np);
    Apool[e] = A[int64_t(i) * ng + pool[p]];
  }
}

// Residual bounds: res[r] = base[r] - sum_m L[m][r]^2 over the projections
// L = Q A of a chunk of columns onto k directions (L is [k][rc]).  base may
// be res itself (each element is read before it is written).
__global__ void k_refresh_res(const double* __restrict__ L, int k, int64_t rc, const double* norm0, double* res) {
  for (int64_t r = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; r < rc; r += int64_t(gridDim.x) * blockDim.x) {
    double s = norm0[r];
    for (int m = 0; m < k; ++m) {
      const double l = L[int64_t(m) * rc + r];
      s -= l * l;
    }
    res[r] = s;
  }
}

__global__ void k_retire(const int32_t* __restrict__ piv, int k, double* __restrict__ res) {
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < k; m += gridDim.x * blockDim.x) res[piv[m]] = -1.0;
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
// X <- X / sqrt(max_i sum_j |G_ij|) with G = X^T X (n x n): the largest
// absolute row sum of G bounds its largest eigenvalue, so every singular
// value of the scaled X is at most 1 (the Newton-Schulz polar iteration then
// converges from any nonsingular start).  One block.
__global__ void k_scale_inf(double* __restrict__ X, const double* __restrict__ G, int n) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) r += fabs(G[int64_t(i) * n + j]);
    m = fmax(m, r);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  for (int64_t e = threadIdx.x; e < int64_t(n) * n; e += blockDim.x) X[e] *= inv;
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
// out[0] = -sum c^2 over n values: the summed exchange energy of a set of
// functions from their projector coefficients c_ka = <xi_k | x_a>.  One block,
// fixed summation order (deterministic).
__global__ void k_neg_sumsq(const double* __restrict__ c, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) a = fma(c[e], c[e], a);
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = -red[0];
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

void launch_neg_sumsq(const double* c, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_neg_sumsq, dim3(1), dim3(256), 0, s, c, n, out);
}
void launch_symmetrize(const double* M, int n, double* out, double* negM, double* ex, double* asym, hipStream_t s) {
  hipLaunchKernelGGL(k_symmetrize, dim3(1), dim3(256), 0, s, M, n, out, negM, ex, asym);
}
// info must be zero on entry (the blocked kernels skip work once it is set).
void launch_cholesky(double* A, int n, int* info, double* tinv, hipStream_t s) {
  for (int k0 = 0; k0 < n; k0 += CB) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, A, n, k0, tinv, info);
    const int rest = n - k0 - CB;
    if (rest <= 0) break;
    const int tiles = (rest + CB - 1) / CB;
    hipLaunchKernelGGL(k_chol_panel, dim3(tiles), dim3(256), 0, s, A, n, k0, tinv, info);
    hipLaunchKernelGGL(k_chol_update, dim3(tiles * (tiles + 1) / 2), dim3(256), 0, s, A, n, k0, info);
  }
}
void launch_trinv(const double* L, int n, double* X, hipStream_t s) {
  hipLaunchKernelGGL(k_trinv_lower, dim3(n), dim3(64), 0, s, L, n, X);
}
void launch_chol_inv(double* A, int n, int* info, double* X, double* tinv, hipStream_t s) {
  if (n <= SMALL_N) {
    hipLaunchKernelGGL(k_chol_inv_small, dim3(1), dim3(1024), 0, s, A, n, info, X);
  } else {
    launch_cholesky(A, n, info, tinv, s);
    launch_trinv(A, n, X, s);
  }
}
void launch_colnorm(const double* A, int n, int64_t ng, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_colnorm, dim3(grid_for(ng, 256)), dim3(256), 0, s, A, n, ng, res);
}
int qrcp_blocks(int64_t ng) { return grid_for(ng, 256, 2048); }
void launch_qrcp_update(const double* A, int n, int64_t ng, const double* q, double* res, double* pv, int64_t* pi,
                        const int* stop, hipStream_t s) {
  hipLaunchKernelGGL(k_qrcp_update<256>, dim3(qrcp_blocks(ng)), dim3(256), 0, s, A, n, ng, q, res, pv, pi, stop);
}
void launch_qrcp_select(const double* A, int n, int64_t ng, int* kdev, const double* pv, const int64_t* pi,
                        int nblk, double* Q, double* res, int32_t* piv, double* qout, const int32_t* pool,
                        const double* t_out, int* stop, hipStream_t s) {
  hipLaunchKernelGGL(k_qrcp_select<512>, dim3(1), dim3(512), 0, s, A, n, ng, kdev, pv, pi, nblk, Q, res, piv, qout,
                     pool, t_out, stop);
}
constexpr int QCW = 16;  // pool columns per update block
int qrcp_pool_blocks(int P) { return (P + QCW - 1) / QCW; }
void launch_qrcp_update_r(double* R, int n, int P, const double* q, double* res, double* pv, int64_t* pi,
                          const int* stop, hipStream_t s) {
  hipLaunchKernelGGL((k_qrcp_update_r<256, QCW>), dim3(qrcp_pool_blocks(P)), dim3(256), 0, s, R, n, P, q, res, pv, pi, stop);
}
void launch_qrcp_select_r(const double* R, int n, int P, int* kdev, const double* pv, const int64_t* pi,
                          double* Q, double* res, int32_t* piv, double* qout, const int32_t* pool,
                          const double* t_out, int* stop, hipStream_t s) {
  hipLaunchKernelGGL(k_qrcp_select_r<256>, dim3(1), dim3(256), 0, s, R, n, P, kdev, pv, pi, qrcp_pool_blocks(P), Q,
                     res, piv, qout, pool, t_out, stop);
}
void launch_qrcp_step_r(double* R, int n, int P, int* kdev, const double* pv_in, const int64_t* pi_in, double* Q,
                        double* res, int32_t* piv, const int32_t* pool, const double* t_out, int* stop,
                        double* pv_out, int64_t* pi_out, hipStream_t s) {
  // rows per thread of the block's tile: n / (256 / QCW), held in registers
#define QSTEP(MPV)                                                                                                 \
  hipLaunchKernelGGL((k_qrcp_step_r<256, QCW, MPV>), dim3(qrcp_pool_blocks(P)), dim3(256), 0, s, R, n, P, kdev,   \
                     pv_in, pi_in, qrcp_pool_blocks(P), Q, res, piv, pool, t_out, stop, pv_out, pi_out)
  constexpr int RG = 256 / QCW;
  if (n <= 8 * RG) QSTEP(8);
  else if (n <= 16 * RG) QSTEP(16);
  else if (n <= 32 * RG) QSTEP(32);
  else QSTEP(64);
#undef QSTEP
}
void launch_add_inplace(double* a, const double* b, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_add_inplace, dim3(grid_for(cnt, 256)), dim3(256), 0, s, a, b, cnt);
}
int pool_blocks(int64_t ng) { return grid_for(ng, 4096, 2048); }
void launch_pool_build(const double* res, int64_t ng, int pmax, unsigned* hist, double* t, int64_t* cnt,
                       double* tmax, int* total, double* t_out, hipStream_t s) {
  hipLaunchKernelGGL(k_res_hist, dim3(grid_for(ng, 256, 1024)), dim3(256), 0, s, res, ng, hist);
  hipLaunchKernelGGL(k_pool_threshold, dim3(1), dim3(1024), 0, s, hist, pmax, t);
  const int nb = pool_blocks(ng);
  const int64_t chunk = (ng + nb - 1) / nb;
  hipLaunchKernelGGL(k_pool_count, dim3(nb), dim3(256), 0, s, res, ng, chunk, t, cnt, tmax);
  hipLaunchKernelGGL(k_pool_scan, dim3(1), dim3(1024), 0, s, cnt, tmax, nb, total, t_out);
}
void launch_pool_write(const double* res, int64_t ng, const double* t, const int64_t* off, int32_t* pool,
                       double* pres, hipStream_t s) {
  const int nb = pool_blocks(ng);
  const int64_t chunk = (ng + nb - 1) / nb;
  hipLaunchKernelGGL(k_pool_write, dim3(nb), dim3(256), 0, s, res, ng, chunk, t, off, pool, pres);
}
void launch_pool_gather(const double* A, int n, int64_t ng, const int32_t* pool, int np, double* Apool,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_pool_gather, dim3(grid_for(int64_t(n) * np, 256)), dim3(256), 0, s, A, n, ng, pool, np,
                     Apool);
}
void launch_refresh_res(const double* L, int k, int64_t rc, const double* norm0, double* res, hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_res, dim3(grid_for(rc, 256)), dim3(256), 0, s, L, k, rc, norm0, res);
}
void launch_retire(const int32_t* piv, int k, double* res, hipStream_t s) {
  if (k > 0) hipLaunchKernelGGL(k_retire, dim3((k + 255) / 256), dim3(256), 0, s, piv, k, res);
}
void launch_gather_cols(const double* A, int n, int64_t ng, const int32_t* piv, double* AC, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_cols, dim3(grid_for(int64_t(n) * n, 256)), dim3(256), 0, s, A, n, ng, piv, AC);
}
void launch_scale_inf(double* X, const double* G, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_inf, dim3(1), dim3(1024), 0, s, X, G, n);
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
