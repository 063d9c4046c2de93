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
#include <type_traits>
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

// ---------------------------------------------------------------- 128 x 128 MFMA tiles
// One workgroup (4 waves) computes a 128 x 128 tile of
//   C(m, n) = sum_{k in [kb, ke)} f(A(m, k)) f(B(k, n)),
// each wave a 64 x 64 quarter (4 x 4 blocks of v_mfma_f64_16x16x4f64).
// Operand sources: A(m, k) = A[m][k] (AK = false) or A[k][m] (AK = true);
// B(k, n) = B[n][k] (BK = false) or B[k][n] (BK = true).  Each K step of 16
// is staged in k-major LDS tiles, double buffered: the next step's global
// loads are issued before the current step's MFMAs.  Row pitch TP = 144
// doubles puts the four k-rows a lane group reads in alternating halves of
// the LDS banks.
constexpr int TT = 128, KS = 16, TP = TT + 16;

// element e (0..2047) of a 128 x 16 step: (row, k) in the operand's tile
template <bool KM>
__device__ __forceinline__ void tile_rk(int e, int& r, int& k) {
  if (KM) { r = e % TT; k = e / TT; } else { r = e / KS; k = e % KS; }
}

// Threads of a tile workgroup: 2 row waves x NW column waves.
template <int NW> __host__ __device__ constexpr int tile_threads() { return 128 * NW; }
// elements of one operand's 128 x 16 step per thread
template <int NW> __host__ __device__ constexpr int tile_per() { return 2048 / tile_threads<NW>(); }
// Minimum waves per SIMD for the launch bounds.  NW = 2: 64 x 64 outputs per
// wave, two waves per SIMD (up to 256 registers); NW = 4: 64 x 32 per wave,
// four per SIMD (capped at 128 registers).
template <int NW> __host__ __device__ constexpr int tile_waves() { return NW == 2 ? 2 : 4; }

// Loads stay in the operand's own type: the conversion to double and the
// element map are applied by tile_store, after the current step's MFMAs, so
// the next step's loads remain in flight meanwhile.
template <typename TX, bool KM, int NW = 2>
__device__ __forceinline__ void tile_load(const TX* __restrict__ X, int64_t ld, int r0, int rows, int64_t k0,
                                          int64_t ke, int tid, TX (&v)[tile_per<NW>()]) {
#pragma unroll
  for (int i = 0; i < tile_per<NW>(); ++i) {
    int r, k;
    tile_rk<KM>(tid + tile_threads<NW>() * i, r, k);
    const int64_t kk = k0 + k;
    TX x = TX(0);
    if (r0 + r < rows && kk < ke) x = KM ? X[kk * ld + r0 + r] : X[int64_t(r0 + r) * ld + kk];
    v[i] = x;
  }
}

// k-contiguous operands (KM false) are kept row-major in LDS, RP doubles per
// row: the stores of a wave (16 lanes along k per row) are then contiguous,
// and the MFMA operand reads (16 rows by 4 k per wave) fall in distinct
// banks within each half-wave.  (The k-major layout with the TP pitch would
// put the 16 lanes of a row on the same two banks.)
constexpr int RP = KS + 1;
static_assert(TT * RP <= KS * TP, "a row-major tile must fit a k-major tile's buffer");

template <bool KM, int OP, int NW, typename TX>
__device__ __forceinline__ void tile_store(double* S, int tid, const TX (&v)[tile_per<NW>()]) {
  if constexpr (!KM) {
#pragma unroll
    for (int i = 0; i < tile_per<NW>(); ++i) {
      int r, k;
      tile_rk<false>(tid + tile_threads<NW>() * i, r, k);
      S[r * RP + k] = opmap<OP>(double(v[i]));
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < tile_per<NW>(); ++i) {
    int r, k;
    tile_rk<KM>(tid + tile_threads<NW>() * i, r, k);
    S[k * TP + r] = opmap<OP>(double(v[i]));
  }
}

// First row, within the 128-row tile, of 16-row block i of row wave wm.
// With a lower-triangular left factor (IL) the two row waves take alternate
// blocks (0, 2, 4, 6 and 1, 3, 5, 7): block b needs k < 16 (b + 1), and
// alternating balances the two waves' MFMAs in every K step, where
// contiguous halves leave the upper wave idle for the second half of K.
template <bool IL>
__device__ __forceinline__ int rowblk(int wm, int i) {
  return IL ? (2 * i + wm) * 16 : wm * 64 + i * 16;
}

// Accumulate the tile over [kb, ke) into acc: each of the 2 x NW waves owns
// 64 rows x (128 / NW) columns, JB = 8 / NW blocks of 16 columns.  With NW = 4
// (512 threads) a wave holds half the accumulators, so four waves fit per
// SIMD instead of two.
// LOWA: A(m, k) = 0 for k > m (lower-triangular left factor, global row and
// k indices): a 16-row block skips the MFMAs of the k beyond its last row.
// MIR (NW = 4): wave column wn takes the 16-column blocks wn and 7 - wn of
// the tile (else 2 wn and 2 wn + 1); with upper (a tile on the diagonal of a
// symmetric product) the blocks below the diagonal are skipped, and the two
// waves of every SIMD then share nine of its sixteen blocks.
template <int NW, bool MIR>
__device__ __forceinline__ int colblk(int wn, int j) {
  return MIR ? (j == 0 ? wn : 2 * NW - 1 - wn) : wn * (8 / NW) + j;
}
template <typename TA, typename TB, bool AK, bool BK, int OP, bool LOWA = false, int NW = 2, bool MIR = false>
__device__ __forceinline__ void tile_mma(const TA* __restrict__ A, int64_t lda, const TB* __restrict__ B,
                                         int64_t ldb, int m0, int M, int n0, int Nn, int64_t kb, int64_t ke,
                                         double* As, double* Bs, d4 (&acc)[4][8 / NW], bool upper = false) {
  constexpr int JB = 8 / NW, PER = tile_per<NW>();
  static_assert(!MIR || NW == 4, "mirrored column blocks need four wave columns");
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / NW, wn = wv % NW;
  TA va[PER];
  TB vb[PER];
  int buf = 0;
  if (kb < ke) {
    tile_load<TA, AK, NW>(A, lda, m0, M, kb, ke, tid, va);
    tile_load<TB, BK, NW>(B, ldb, n0, Nn, kb, ke, tid, vb);
    tile_store<AK, OP, NW>(As, tid, va);
    tile_store<BK, OP, NW>(Bs, tid, vb);
  }
  __syncthreads();
  for (int64_t k0 = kb; k0 < ke; k0 += KS) {
    const bool more = k0 + KS < ke;
    if (more) {
      tile_load<TA, AK, NW>(A, lda, m0, M, k0 + KS, ke, tid, va);
      tile_load<TB, BK, NW>(B, ldb, n0, Nn, k0 + KS, ke, tid, vb);
    }
    const double* as = As + buf * KS * TP;
    const double* bs = Bs + buf * KS * TP;
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const int kq = kk + lane / 16, kr = kq * TP, li = lane % 16;
      double a[4], b[JB];
#pragma unroll
      for (int i = 0; i < 4; ++i)
        a[i] = AK ? as[kr + rowblk<LOWA>(wm, i) + li] : as[(rowblk<LOWA>(wm, i) + li) * RP + kq];
#pragma unroll
      for (int j = 0; j < JB; ++j) {
        const int cb = colblk<NW, MIR>(wn, j) * 16;
        b[j] = BK ? bs[kr + cb + li] : bs[(cb + li) * RP + kq];
      }
      // blocks with rows < M and columns < Nn (the others stay zero, so their
      // MFMAs are skipped; wave-uniform)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JB; ++j)
          if (m0 + rowblk<LOWA>(wm, i) < M && n0 + colblk<NW, MIR>(wn, j) * 16 < Nn &&
              (!upper || rowblk<LOWA>(wm, i) <= colblk<NW, MIR>(wn, j) * 16) &&
              (!LOWA || k0 + kk < int64_t(m0) + rowblk<LOWA>(wm, i) + 16))
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      buf ^= 1;
      tile_store<AK, OP, NW>(As + buf * KS * TP, tid, va);
      tile_store<BK, OP, NW>(Bs + buf * KS * TP, tid, vb);
    }
    __syncthreads();
  }
}

// acc -> out[m][n] (ld) for rows < M, columns < Nn, times alpha
template <int NW = 2, bool IL = false, bool MIR = false>
__device__ __forceinline__ void tile_write(const d4 (&acc)[4][8 / NW], int m0, int M, int64_t n0, int64_t Nn,
                                           double* __restrict__ out, int64_t ld, double alpha) {
  constexpr int JB = 8 / NW;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wm = wv / NW, wn = wv % NW;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + rowblk<IL>(wm, i) + lane / 16 + 4 * r;
        const int64_t n = n0 + colblk<NW, MIR>(wn, j) * 16 + lane % 16;
        if (m < M && n < Nn) out[int64_t(m) * ld + n] = alpha * acc[i][j][r];
      }
}

// NT split-K: blockIdx.x = tile t of the tile list (tm, tn) = (t / ntn, t % ntn),
// or with SYM the t-th tile of the upper triangle tm <= tn; blockIdx.y = split.
// Cpart[split][M][Nn] receives the tile's partial sums.
template <int OP, bool SYM, int NW = 2>
__global__ __launch_bounds__(tile_threads<NW>(), tile_waves<NW>()) void k_gemm_nt_t128(
    const double* __restrict__ A, int64_t lda, const double* __restrict__ B, int64_t ldb, int M, int Nn, int64_t K,
    int64_t kchunk, int ntn, double* __restrict__ Cpart) {
  __shared__ double As[2 * KS * TP];
  __shared__ double Bs[2 * KS * TP];
  int tm, tn;
  if (SYM) {
    // upper-triangle enumeration row by row: row tm holds ntn - tm tiles
    int t = blockIdx.x;
    tm = 0;
    while (t >= ntn - tm) { t -= ntn - tm; ++tm; }
    tn = tm + t;
  } else {
    tm = blockIdx.x / ntn;
    tn = blockIdx.x % ntn;
  }
  const int m0 = tm * TT, n0 = tn * TT;
  const int64_t kb = int64_t(blockIdx.y) * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  d4 acc[4][8 / NW];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8 / NW; ++j) acc[i][j] = d4{0, 0, 0, 0};
  // a symmetric product forms the upper triangle only (tiles tm <= tn and,
  // on the diagonal, 16 x 16 blocks on or above it); the reduction mirrors
  tile_mma<double, double, false, false, OP, false, NW, SYM>(A, lda, B, ldb, m0, M, n0, Nn, kb, ke, As, Bs, acc,
                                                             SYM && tm == tn);
  tile_write<NW, false, SYM>(acc, m0, M, n0, Nn, Cpart + int64_t(blockIdx.y) * M * Nn, Nn, 1.0);
}

// ---------------------------------------------------------------- 128 x 64 FP32 compensated tiles
// The compensated FP32 product on 128 x 64 tiles: each wave accumulates a
// 64 x 32 quarter (4 x 2 blocks of v_mfma_f32_16x16x4f32) over K steps of 16
// staged in row-major LDS tiles (pitch RPF = 20 floats: the MFMA operand reads
// of 16 rows by 4 k fall in 64 distinct banks) and double buffered through
// registers (float4 loads of four consecutive k); every `sub` products the FP32 block sums are
// merged into (hi, lo) pairs by TwoSum (the hi/lo pairs of a 64 x 64 quarter
// would not fit the register file), and the tile writes hi + lo in FP64 to
// its split's partial-sum slice.  Requires K, lda and ldb multiples of 4 and
// 16-byte aligned operands.
constexpr int RPF = KS + 4;   // row pitch of the FP32 LDS tiles (floats)
constexpr int TNF = 64;       // tile columns

// rows r0 .. r0 + 16 * Q - 1 of a 16-wide K step: Q float4 per thread
template <int Q>
__device__ __forceinline__ void f32t_load(const float* __restrict__ X, int64_t ld, int r0, int rows, int64_t k0,
                                          int64_t ke, int tid, f4 (&v)[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 2, kq = (e & 3) * 4;
    const int64_t k = k0 + kq;
    f4 x = f4{0.f, 0.f, 0.f, 0.f};
    if (r0 + r < rows && k < ke) x = *reinterpret_cast<const f4*>(X + int64_t(r0 + r) * ld + k);
    v[i] = x;
  }
}

template <int Q>
__device__ __forceinline__ void f32t_store(float* S, int tid, const f4 (&v)[Q]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int e = tid + 256 * i;
    const int r = e >> 2, kq = (e & 3) * 4;
    *reinterpret_cast<f4*>(S + r * RPF + kq) = v[i];
  }
}

__global__ __launch_bounds__(256, 2) void k_gemm_nt_f32t(const float* __restrict__ A, int64_t lda,
                                                         const float* __restrict__ B, int64_t ldb, int M, int Nn,
                                                         int64_t K, int64_t kchunk, int ntn, int sub,
                                                         double* __restrict__ Cpart) {
  __shared__ __attribute__((aligned(16))) float As[2 * TT * RPF];
  __shared__ __attribute__((aligned(16))) float Bs[2 * TNF * RPF];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int tm = blockIdx.x / ntn, tn = blockIdx.x % ntn;
  const int m0 = tm * TT, n0 = tn * TNF;
  const int64_t kb = int64_t(blockIdx.y) * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  f4 acc[4][2];
  float hi[4][2][4], lo[4][2][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) hi[i][j][r] = lo[i][j][r] = 0.f;
    }
  f4 va[2], vb[1];
  int buf = 0;
  if (kb < ke) {
    f32t_load<2>(A, lda, m0, M, kb, ke, tid, va);
    f32t_load<1>(B, ldb, n0, Nn, kb, ke, tid, vb);
    f32t_store<2>(As, tid, va);
    f32t_store<1>(Bs, tid, vb);
  }
  __syncthreads();
  int64_t since = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += KS) {
    const bool more = k0 + KS < ke;
    if (more) {
      f32t_load<2>(A, lda, m0, M, k0 + KS, ke, tid, va);
      f32t_load<1>(B, ldb, n0, Nn, k0 + KS, ke, tid, vb);
    }
    const float* as = As + buf * TT * RPF;
    const float* bs = Bs + buf * TNF * RPF;
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      const int kq = kk + lane / 16, li = lane % 16;
      float a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = as[(wm * 64 + i * 16 + li) * RPF + kq];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = bs[(wn * 32 + j * 16 + li) * RPF + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    since += KS;
    if (since >= sub || !more) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) two_sum(hi[i][j][r], lo[i][j][r], acc[i][j][r]);
          acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
        }
      since = 0;
    }
    if (more) {
      buf ^= 1;
      f32t_store<2>(As + buf * TT * RPF, tid, va);
      f32t_store<1>(Bs + buf * TNF * RPF, tid, vb);
    }
    __syncthreads();
  }
  double* out = Cpart + int64_t(blockIdx.y) * M * Nn;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 64 + i * 16 + 4 * (lane / 16) + r;
        const int n = n0 + wn * 32 + j * 16 + lane % 16;
        if (m < M && n < Nn) out[int64_t(m) * Nn + n] = double(hi[i][j][r]) + double(lo[i][j][r]);
      }
}

// C = alpha * sum_s Cpart[s]; with SYM only tiles tm <= tn were computed and
// the lower triangle of tiles is read transposed.  A block reduces RO
// consecutive outputs with RG groups of threads, group g summing the splits
// s = g mod RG (four loads in flight per thread); the groups meet in LDS in a
// fixed order, so the result is deterministic.  (One thread per output
// summing every split in turn was latency-bound: 125 us for a 128 x 128
// result of 500 splits.)
constexpr int RO = 32, RGR = 8;
template <bool SYM>
__global__ __launch_bounds__(256) void k_reduce_parts_t(const double* __restrict__ Cpart, int nsplit, int M, int Nn,
                                                        double alpha, double* __restrict__ C) {
  __shared__ double part[RGR][RO];
  const int o = threadIdx.x % RO, g = threadIdx.x / RO;
  const int64_t mn = int64_t(M) * Nn;
  const int64_t e = int64_t(blockIdx.x) * RO + o;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < mn) {
    int64_t src = e;
    if (SYM) {
      // only blocks on or above the diagonal (16 x 16) were formed
      const int i = int(e / Nn), j = int(e % Nn);
      if (i / 16 > j / 16) src = int64_t(j) * Nn + i;
    }
    int p = g;
    for (; p + 3 * RGR < nsplit; p += 4 * RGR) {
      s0 += Cpart[int64_t(p) * mn + src];
      s1 += Cpart[int64_t(p + RGR) * mn + src];
      s2 += Cpart[int64_t(p + 2 * RGR) * mn + src];
      s3 += Cpart[int64_t(p + 3 * RGR) * mn + src];
    }
    for (; p < nsplit; p += RGR) s0 += Cpart[int64_t(p) * mn + src];
  }
  part[g][o] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && e < mn) {
    double t = 0.0;
#pragma unroll
    for (int h = 0; h < RGR; ++h) t += part[h][o];
    C[e] = alpha * t;
  }
}

// Left-small: C[m][r] = alpha * sum_k S(m, k) B[k][r], S(m, k) = TRANS ? S[k][m] : S[m][k];
// LOWER: S(m, k) = 0 for k > m.  blockIdx.x = 128-column tile of r (fastest:
// neighbouring workgroups write neighbouring segments of the same rows of C,
// measured faster than the row tiles fastest), blockIdx.y = 128-row tile of m.
template <typename TB, bool TRANS, bool LOWER, int NW = 2>
__global__ __launch_bounds__(tile_threads<NW>(), tile_waves<NW>()) void k_gemm_ls_t128(
    const double* __restrict__ S, int lds, const TB* __restrict__ B, int64_t ldb, double* __restrict__ C, int64_t ldc,
    int M, int K, int64_t R, double alpha) {
  __shared__ double As[2 * KS * TP];
  __shared__ double Bs[2 * KS * TP];
  const int m0 = blockIdx.y * TT;
  const int64_t r0 = int64_t(blockIdx.x) * TT;
  const int64_t ke = LOWER ? ((m0 + TT < K) ? m0 + TT : K) : K;
  d4 acc[4][8 / NW];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8 / NW; ++j) acc[i][j] = d4{0, 0, 0, 0};
  // B columns r0 .. r0 + 127 are addressed from the tile origin
  const TB* Bt = B + r0;
  const int64_t rrem = R - r0;
  tile_mma<double, TB, TRANS, true, 0, LOWER, NW>(S, lds, Bt, ldb, m0, M, 0, int(rrem < TT ? rrem : TT), 0, ke, As,
                                                 Bs, acc);
  tile_write<NW, LOWER>(acc, m0, M, 0, rrem < TT ? rrem : TT, C + r0, ldc, alpha);
}

// Bound refresh of the pivot search in one pass: for the 128 grid columns of
// this tile, L = Q Psi[:, cols] (M <= 128 rows of Q, K = ldq columns) on the
// MFMA tile, then res[r] -= sum_m L[m][r]^2, without writing L.  Column sums
// run over each lane's rows, then across the four lane groups, then across
// the two row halves of the tile (fixed order).
template <int NW = 2>
__global__ __launch_bounds__(tile_threads<NW>(), tile_waves<NW>()) void k_refresh_t128(
    const double* __restrict__ Q, int ldq, const double* __restrict__ Psi, int64_t ldp, int M, int K, int64_t R,
    double* __restrict__ res) {
  __shared__ double As[2 * KS * TP];
  __shared__ double Bs[2 * KS * TP];
  __shared__ double colsum[2][TT];
  const int64_t r0 = int64_t(blockIdx.x) * TT;
  const int64_t rrem = R - r0;
  const int ncol = int(rrem < TT ? rrem : TT);
  constexpr int JB = 8 / NW, WC = 128 / NW;
  d4 acc[4][JB];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < JB; ++j) acc[i][j] = d4{0, 0, 0, 0};
  tile_mma<double, double, false, true, 0, false, NW>(Q, ldq, Psi + r0, ldp, 0, M, 0, ncol, 0, K, As, Bs, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wm = wv / NW, wn = wv % NW;
#pragma unroll
  for (int j = 0; j < JB; ++j) {
    double sq = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) sq += acc[i][j][r] * acc[i][j][r];
    sq += __shfl_xor(sq, 16, 64);
    sq += __shfl_xor(sq, 32, 64);
    if (lane < 16) colsum[wm][wn * WC + j * 16 + lane] = sq;
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < ncol) res[r0 + t] -= colsum[0][t] + colsum[1][t];
}

hipError_t refresh_bounds(const double* Q, int ldq, const double* Psi, int64_t ldp, int M, int K, int64_t R,
                          double* res, hipStream_t s) {
  if (M < 1 || M > TT || K < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_refresh_t128<4>, dim3(unsigned((R + TT - 1) / TT)), dim3(tile_threads<4>()), 0, s, Q, ldq, Psi,
                     ldp, M, K, R, res);
  return hipGetLastError();
}

// ---------------------------------------------------------------- host wrappers

int64_t gemm_nt_nsplit(int M, int Nn, int64_t K, int64_t* kchunk_out, bool sym, int64_t max_split) {
  // about 512 workgroups (two per CU) over the 128 x 128 tiles that are
  // computed (the upper triangle only for a symmetric product), K chunks a
  // multiple of 256 (the compensated FP32 sub-chunk).  With sym = true for a
  // square product the count is the larger of the two cases, which is what
  // partial-sum buffers are sized for.
  const int64_t tm = (M + TT - 1) / TT, tn = (Nn + TT - 1) / TT;
  const int64_t tiles = (sym && M == Nn) ? tm * (tm + 1) / 2 : tm * tn;
  const int64_t want = (512 + tiles - 1) / tiles;
  int64_t kchunk = (K + want - 1) / want;
  kchunk = ((kchunk + 255) / 256) * 256;
  if (kchunk < 256) kchunk = 256;
  // a caller with a fixed partial-sum buffer caps the split count: longer chunks
  if (max_split > 0 && (K + kchunk - 1) / kchunk > max_split) {
    kchunk = (K + max_split - 1) / max_split;
    kchunk = ((kchunk + 255) / 256) * 256;
  }
  const int64_t nsplit = (K + kchunk - 1) / kchunk;
  *kchunk_out = kchunk;
  return nsplit;
}

hipError_t gemm_nt(int prec, int op, const void* A, int64_t lda, const void* B, int64_t ldb, int M,
                   int Nn, int64_t K, double alpha, double* Cpart, double* C, hipStream_t s,
                   EventRecorder* rec, bool sym, int64_t max_split) {
  int64_t kchunk;
  sym = sym && prec == 0 && M == Nn && A == B && lda == ldb;
  const int64_t nsplit = gemm_nt_nsplit(M, Nn, K, &kchunk, sym, max_split);
  rec_begin(rec, KC_GEMM_NT, s);
  const int64_t mn = int64_t(M) * Nn;
  const unsigned nbr = unsigned((mn + RO - 1) / RO);
  if (prec == 0) {
    const int ntm = (M + TT - 1) / TT, ntn = (Nn + TT - 1) / TT;
    const unsigned ntiles = unsigned(sym ? ntn * (ntn + 1) / 2 : ntm * ntn);
    dim3 grid(ntiles, unsigned(nsplit));
    const double* a = (const double*)A;
    const double* b = (const double*)B;
#define NT_LAUNCH(OPV, SYMV)                                                                                  \
    hipLaunchKernelGGL((k_gemm_nt_t128<OPV, SYMV, 4>), grid, dim3(tile_threads<4>()), 0, s, a, lda, b, ldb, M, Nn, K, \
                       kchunk, ntn, Cpart)
    if (sym) {
      if (op == 1) NT_LAUNCH(1, true);
      else if (op == 2) NT_LAUNCH(2, true);
      else NT_LAUNCH(0, true);
      hipLaunchKernelGGL(k_reduce_parts_t<true>, dim3(nbr), dim3(256), 0, s, Cpart, int(nsplit), M, Nn, alpha, C);
    } else {
      if (op == 1) NT_LAUNCH(1, false);
      else if (op == 2) NT_LAUNCH(2, false);
      else NT_LAUNCH(0, false);
      hipLaunchKernelGGL(k_reduce_parts_t<false>, dim3(nbr), dim3(256), 0, s, Cpart, int(nsplit), M, Nn, alpha, C);
    }
#undef NT_LAUNCH
  } else {
    const bool vec = K % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 && (uintptr_t(A) & 15) == 0 &&
                     (uintptr_t(B) & 15) == 0;
    if (vec) {
      const int ntm = (M + TT - 1) / TT, ntn = (Nn + TNF - 1) / TNF;
      hipLaunchKernelGGL(k_gemm_nt_f32t, dim3(unsigned(ntm * ntn), unsigned(nsplit)), dim3(256), 0, s,
                         (const float*)A, lda, (const float*)B, ldb, M, Nn, K, kchunk, ntn, 256, Cpart);
    } else {
      dim3 grid((Nn + GB - 1) / GB, (M + GB - 1) / GB, unsigned(nsplit));
      hipLaunchKernelGGL(k_gemm_nt_f32c, grid, dim3(256), 0, s, (const float*)A, lda, (const float*)B, ldb, M, Nn,
                         K, kchunk, 256, Cpart);
    }
    hipLaunchKernelGGL(k_reduce_parts_t<false>, dim3(nbr), dim3(256), 0, s, Cpart, int(nsplit), M, Nn, alpha, C);
  }
  rec_end(rec, KC_GEMM_NT, s, (sym && prec == 0 ? 1.0 : 2.0) * double(M) * Nn * double(K));
  return hipGetLastError();
}

template <typename TB, bool TRANS, bool LOWER>
static void launch_ls(const double* S, int lds, const TB* B, int64_t ldb, double* C, int64_t ldc, int M, int K,
                      int64_t R, double alpha, hipStream_t s) {
  if (R <= 1024) {
    dim3 grid(unsigned((R + 15) / 16), unsigned((M + 15) / 16));
    hipLaunchKernelGGL((k_gemm_tiny<TB, TRANS, LOWER>), grid, dim3(64), 0, s, S, lds, B, ldb, C, ldc, M, K, R, alpha);
  } else if (M > 64) {
    dim3 grid(unsigned((R + TT - 1) / TT), unsigned((M + TT - 1) / TT));
    // FP32 right operands run 8 waves per tile; with FP64 ones the 512-thread
    // tile spills and was slower, so they keep 4.
    constexpr int NW = std::is_same<TB, float>::value ? 4 : 2;
    hipLaunchKernelGGL((k_gemm_ls_t128<TB, TRANS, LOWER, NW>), grid, dim3(tile_threads<NW>()), 0, s, S, lds, B, ldb, C,
                       ldc, M, K, R, alpha);
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
