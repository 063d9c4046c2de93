// Dense contractions on the matrix cores (MFMA), used for
//   M = dV * Phi W^T                   (Appendix A: M_kl = <phi_k|V_X|phi_l>)
//   O = dV * |Phi| |Phi|^T              (screening integrals)
//   P = W L^-T, i.e. xi = L^-1 W        (Appendix A projectors)
//   Phi = U^T Psi                       (Eq. unit)
//   V_ACE x = -xi^T (xi x^T dV)         (ACE application)
//
// Two shapes occur.  "NT split-K": both operands are [rows][K] with K the grid
// size (10^4 .. 4*10^6) and at most a few hundred rows; K is split over
// workgroups, each writes a partial tile, and a second kernel reduces the
// partials.  "Left-small": C[m][r] = sum_k S(m,k) B[k][r] with a small square
// S (K = number of orbitals) and r running over the grid.
//
// MFMA operand layout (v_mfma_f64_16x16x4f64 and v_mfma_f32_16x16x4f32, one
// block): lane l supplies A[l%16][l/16] and B[l/16][l%16].  Accumulator
// element r of lane l is D[l/16 + 4r][l%16] for the FP64 instruction and
// D[4(l/16) + r][l%16] for the FP32 one (checked on gfx950 by a lane probe).
#include <hip/hip_runtime.h>
#include <cstdint>
#include "ace_internal.h"

namespace ace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int GB = 64;   // output tile edge
constexpr int GK = 32;   // K step staged through LDS

// elementwise operand map of the split-K product: 0 identity, 1 |x|, 2 x^2
template <int OP, typename T>
__device__ __forceinline__ T opmap(T v) { return OP == 1 ? (v < T(0) ? -v : v) : OP == 2 ? v * v : v; }

// ---------------------------------------------------------------- NT split-K, FP64
// Cpart[split][m][n] = sum_{k in split} f(A[m][k]) f(B[n][k]), f = opmap<OP>.
template <int OP>
__global__ __launch_bounds__(256) void k_gemm_nt_f64(const double* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb, int M,
                                                     int Nn, int64_t K, int64_t kchunk,
                                                     double* __restrict__ Cpart) {
  __shared__ double As[GK][GB + 1];
  __shared__ double Bs[GK][GB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int n0 = blockIdx.x * GB, m0 = blockIdx.y * GB;
  const int64_t kb = int64_t(blockIdx.z) * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
  for (int64_t k0 = kb; k0 < ke; k0 += GK) {
    // 64 rows x 32 k per operand: 8 elements per thread, k fastest
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int e = tid + s * 256;
      const int r = e / GK, c = e % GK;
      const int64_t k = k0 + c;
      double va = 0.0, vb = 0.0;
      if (k < ke) {
        if (m0 + r < M) va = opmap<OP>(A[int64_t(m0 + r) * lda + k]);
        if (n0 + r < Nn) vb = opmap<OP>(B[int64_t(n0 + r) * ldb + k]);
      }
      As[c][r] = va;
      Bs[c][r] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + lane / 16, li = lane % 16;
      double a0 = As[kr][wm * 32 + li], a1 = As[kr][wm * 32 + 16 + li];
      double b0 = Bs[kr][wn * 32 + li], b1 = Bs[kr][wn * 32 + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = Cpart + int64_t(blockIdx.z) * M * Nn;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * 32 + a * 16 + lane / 16 + 4 * r;
        const int j = n0 + wn * 32 + b * 16 + lane % 16;
        if (i < M && j < Nn) out[int64_t(i) * Nn + j] = acc[a][b][r];
      }
}

// ---------------------------------------------------------------- NT split-K, FP32 compensated
// FP32 MFMA over sub-chunks of SUB products, each sub-chunk result merged into
// an FP32 (hi, lo) pair with an error-free TwoSum; the block writes hi and lo.
__device__ __forceinline__ void two_sum(float& hi, float& lo, float x) {
  const float s = hi + x;
  const float bp = s - hi;
  const float err = (hi - (s - bp)) + (x - bp);
  hi = s;
  lo += err;
}

__global__ __launch_bounds__(256) void k_gemm_nt_f32c(const float* __restrict__ A, int64_t lda,
                                                      const float* __restrict__ B, int64_t ldb, int M,
                                                      int Nn, int64_t K, int64_t kchunk, int sub,
                                                      double* __restrict__ Cpart) {
  __shared__ float As[GK][GB + 1];
  __shared__ float Bs[GK][GB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int n0 = blockIdx.x * GB, m0 = blockIdx.y * GB;
  const int64_t kb = int64_t(blockIdx.z) * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  f4 acc[2][2];
  float hi[2][2][4], lo[2][2][4];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      acc[a][b] = f4{0, 0, 0, 0};
      for (int r = 0; r < 4; ++r) hi[a][b][r] = lo[a][b][r] = 0.f;
    }
  int64_t since = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += GK) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int e = tid + s * 256;
      const int r = e / GK, c = e % GK;
      const int64_t k = k0 + c;
      float va = 0.f, vb = 0.f;
      if (k < ke) {
        if (m0 + r < M) va = A[int64_t(m0 + r) * lda + k];
        if (n0 + r < Nn) vb = B[int64_t(n0 + r) * ldb + k];
      }
      As[c][r] = va;
      Bs[c][r] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + lane / 16, li = lane % 16;
      float a0 = As[kr][wm * 32 + li], a1 = As[kr][wm * 32 + 16 + li];
      float b0 = Bs[kr][wn * 32 + li], b1 = Bs[kr][wn * 32 + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
    since += GK;
    if (since >= sub || k0 + GK >= ke) {
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          for (int r = 0; r < 4; ++r) two_sum(hi[a][b][r], lo[a][b][r], acc[a][b][r]);
          acc[a][b] = f4{0, 0, 0, 0};
        }
      since = 0;
    }
  }
  double* out = Cpart + int64_t(blockIdx.z) * M * Nn;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * 32 + a * 16 + 4 * (lane / 16) + r;
        const int j = n0 + wn * 32 + b * 16 + lane % 16;
        if (i < M && j < Nn) out[int64_t(i) * Nn + j] = double(hi[a][b][r]) + double(lo[a][b][r]);
      }
}

// C[m][n] = alpha * sum_s Cpart[s][m][n]   (FP64, fixed order: deterministic)
__global__ void k_reduce_parts(const double* __restrict__ Cpart, int nsplit, int64_t mn, double alpha,
                               double* __restrict__ C) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < mn; e += int64_t(gridDim.x) * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += Cpart[int64_t(p) * mn + e];
    C[e] = alpha * s;
  }
}

// ---------------------------------------------------------------- left-small
// C[m][r] = alpha * sum_k S(m,k) B[k][r],  S(m,k) = TRANS ? S[k][m] : S[m][k].
// LOWER: S(m,k) = 0 for k > m (skip those K tiles).
template <typename TB, bool TRANS, bool LOWER, int BM>
__global__ __launch_bounds__(256) void k_gemm_ls(const double* __restrict__ S, int lds,
                                                 const TB* __restrict__ B, int64_t ldb,
                                                 double* __restrict__ C, int64_t ldc, int M, int K,
                                                 int64_t R, double alpha) {
  constexpr int TM = BM / 32;  // 16-row MFMA tiles per wave along m
  __shared__ double Ss[GK][BM + 1];
  __shared__ double Bs[GK][GB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int64_t r0 = int64_t(blockIdx.x) * GB;
  const int m0 = blockIdx.y * BM;
  d4 acc[TM][2];
  for (int a = 0; a < TM; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0, 0, 0, 0};
  const int kend = LOWER ? ((m0 + BM < K) ? m0 + BM : K) : K;
  for (int k0 = 0; k0 < kend; k0 += GK) {
    for (int e = tid; e < GK * BM; e += 256) {
      int kk, mm;
      if (TRANS) { mm = e % BM; kk = e / BM; } else { kk = e % GK; mm = e / GK; }
      const int k = k0 + kk, m = m0 + mm;
      double v = 0.0;
      if (k < K && m < M) v = TRANS ? S[int64_t(k) * lds + m] : S[int64_t(m) * lds + k];
      Ss[kk][mm] = v;
    }
#pragma unroll
    for (int s = 0; s < (GK * GB) / 256; ++s) {
      const int e = tid + s * 256;
      const int kk = e / GB, c = e % GB;
      const int k = k0 + kk;
      const int64_t r = r0 + c;
      Bs[kk][c] = (k < K && r < R) ? double(B[int64_t(k) * ldb + r]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      const int kr = kk + lane / 16, li = lane % 16;
      double b0 = Bs[kr][wn * 32 + li], b1 = Bs[kr][wn * 32 + 16 + li];
#pragma unroll
      for (int a = 0; a < TM; ++a) {
        double av = Ss[kr][wm * (BM / 2) + a * 16 + li];
        acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b0, acc[a][0], 0, 0, 0);
        acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b1, acc[a][1], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  for (int a = 0; a < TM; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        const int i = m0 + wm * (BM / 2) + a * 16 + lane / 16 + 4 * r;
        const int64_t j = r0 + wn * 32 + b * 16 + lane % 16;
        if (i < M && j < R) C[int64_t(i) * ldc + j] = alpha * acc[a][b][r];
      }
}

// ---------------------------------------------------------------- small outputs
// Same contraction as the left-small kernel for small outputs (R <= 1024):
// one wave per 16 x 16 output tile, operands read straight from global memory
// (L2-resident at these sizes), so even a 128^3 product spreads over 64 CUs.
template <typename TB, bool TRANS, bool LOWER>
__global__ __launch_bounds__(64) void k_gemm_tiny(const double* __restrict__ S, int lds, const TB* __restrict__ B,
                                                  int64_t ldb, double* __restrict__ C, int64_t ldc, int M, int K,
                                                  int64_t R, double alpha) {
  const int lane = threadIdx.x;
  const int r0 = blockIdx.x * 16, m0 = blockIdx.y * 16;
  const int li = lane % 16, lk = lane / 16;
  d4 acc = d4{0, 0, 0, 0};
  const int kend = LOWER ? ((m0 + 16 < K) ? m0 + 16 : K) : K;
  for (int k0 = 0; k0 < kend; k0 += 4) {
    const int k = k0 + lk, m = m0 + li;
    const int64_t r = r0 + li;
    double a = 0.0, b = 0.0;
    if (k < K && m < M) a = TRANS ? S[int64_t(k) * lds + m] : S[int64_t(m) * lds + k];
    if (k < K && r < R) b = double(B[int64_t(k) * ldb + r]);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  for (int q = 0; q < 4; ++q) {
    const int i = m0 + lk + 4 * q;
    const int64_t j = r0 + li;
    if (i < M && j < R) C[int64_t(i) * ldc + j] = alpha * acc[q];
  }
}

// ---------------------------------------------------------------- host wrappers

int64_t gemm_nt_nsplit(int M, int Nn, int64_t K, int64_t* kchunk_out) {
  // aim for >= ~1024 workgroups in total, chunks a multiple of GK
  const int64_t tiles = int64_t((M + GB - 1) / GB) * ((Nn + GB - 1) / GB);
  int64_t want = (2048 + tiles - 1) / tiles;
  int64_t kchunk = (K + want - 1) / want;
  kchunk = ((kchunk + 1023) / 1024) * 1024;
  if (kchunk < 1024) kchunk = 1024;
  const int64_t nsplit = (K + kchunk - 1) / kchunk;
  *kchunk_out = kchunk;
  return nsplit;
}

hipError_t gemm_nt(int prec, int op, const void* A, int64_t lda, const void* B, int64_t ldb, int M,
                   int Nn, int64_t K, double alpha, double* Cpart, double* C, hipStream_t s,
                   EventRecorder* rec) {
  int64_t kchunk;
  const int64_t nsplit = gemm_nt_nsplit(M, Nn, K, &kchunk);
  dim3 grid((Nn + GB - 1) / GB, (M + GB - 1) / GB, unsigned(nsplit));
  rec_begin(rec, KC_GEMM_NT, s);
  if (prec == 0) {
    if (op == 1)
      hipLaunchKernelGGL(k_gemm_nt_f64<1>, grid, dim3(256), 0, s, (const double*)A, lda, (const double*)B,
                         ldb, M, Nn, K, kchunk, Cpart);
    else if (op == 2)
      hipLaunchKernelGGL(k_gemm_nt_f64<2>, grid, dim3(256), 0, s, (const double*)A, lda, (const double*)B,
                         ldb, M, Nn, K, kchunk, Cpart);
    else
      hipLaunchKernelGGL(k_gemm_nt_f64<0>, grid, dim3(256), 0, s, (const double*)A, lda, (const double*)B,
                         ldb, M, Nn, K, kchunk, Cpart);
  } else {
    hipLaunchKernelGGL(k_gemm_nt_f32c, grid, dim3(256), 0, s, (const float*)A, lda, (const float*)B, ldb, M, Nn,
                       K, kchunk, 256, Cpart);
  }
  const int64_t mn = int64_t(M) * Nn;
  int nb = int((mn + 255) / 256);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(k_reduce_parts, dim3(nb), dim3(256), 0, s, Cpart, int(nsplit), mn, alpha, C);
  rec_end(rec, KC_GEMM_NT, s, 2.0 * double(M) * Nn * double(K));
  return hipGetLastError();
}

template <typename TB, bool TRANS, bool LOWER>
static void launch_ls(const double* S, int lds, const TB* B, int64_t ldb, double* C, int64_t ldc, int M, int K,
                      int64_t R, double alpha, hipStream_t s) {
  if (R <= 1024) {
    dim3 grid(unsigned((R + 15) / 16), unsigned((M + 15) / 16));
    hipLaunchKernelGGL((k_gemm_tiny<TB, TRANS, LOWER>), grid, dim3(64), 0, s, S, lds, B, ldb, C, ldc, M, K, R, alpha);
  } else if (M > 64) {
    dim3 grid(unsigned((R + GB - 1) / GB), unsigned((M + 127) / 128));
    hipLaunchKernelGGL((k_gemm_ls<TB, TRANS, LOWER, 128>), grid, dim3(256), 0, s, S, lds, B, ldb, C, ldc, M, K, R,
                       alpha);
  } else {
    dim3 grid(unsigned((R + GB - 1) / GB), unsigned((M + 63) / 64));
    hipLaunchKernelGGL((k_gemm_ls<TB, TRANS, LOWER, 64>), grid, dim3(256), 0, s, S, lds, B, ldb, C, ldc, M, K, R,
                       alpha);
  }
}

// bprec: precision of B (0 FP64, 1 FP32); C is always FP64.
hipError_t gemm_ls(int bprec, bool trans, bool lower, const double* S, int lds, const void* B, int64_t ldb,
                   double* C, int64_t ldc, int M, int K, int64_t R, double alpha, hipStream_t s,
                   EventRecorder* rec) {
  rec_begin(rec, KC_GEMM_TN, s);
  if (bprec == 0) {
    const double* b = (const double*)B;
    if (trans) {
      if (lower) launch_ls<double, true, true>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
      else launch_ls<double, true, false>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
    } else {
      if (lower) launch_ls<double, false, true>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
      else launch_ls<double, false, false>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
    }
  } else {
    const float* b = (const float*)B;
    if (trans) {
      if (lower) launch_ls<float, true, true>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
      else launch_ls<float, true, false>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
    } else {
      if (lower) launch_ls<float, false, true>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
      else launch_ls<float, false, false>(S, lds, b, ldb, C, ldc, M, K, R, alpha, s);
    }
  }
  rec_end(rec, KC_GEMM_TN, s, (lower ? 1.0 : 2.0) * double(M) * K * double(R));
  return hipGetLastError();
}

}  // namespace ace
