// Device bodies of the pair-stage passes, shared by the per-pass kernels and
// the persistent batched kernel.  Every body works on one pack's complex
// field spec_p (N^3 values, [z][y][x]) and a workgroup-private LDS buffer;
// the caller has loaded the twiddles tw[m] = exp(-2 pi i m / N) into LDS.
// Each body starts by filling buf and synchronizing, so the twiddle load is
// covered by that barrier; it ends after its last global store.
#pragma once
#include "ace_internal.h"
#include "fft.h"

namespace ace {

__host__ __device__ constexpr int pick_tx(int n) { return (n % 16 == 0) ? 16 : (n % 8 == 0) ? 8 : (n % 4 == 0) ? 4 : 2; }
__host__ __device__ constexpr int pick_rows(int n) { return (n % 8 == 0) ? 8 : (n % 4 == 0) ? 4 : 2; }

// v(G)/N^3 at integer grid frequencies (kx, ky, kz) in FFT order.
template <typename T, int N>
__device__ __forceinline__ T kernel_value(const KernelParams& kp, int kx, int ky, int kz) {
  const int sx = kx < (N + 1) / 2 ? kx : kx - N;
  const int sy = ky < (N + 1) / 2 ? ky : ky - N;
  const int sz = kz < (N + 1) / 2 ? kz : kz - N;
  const double gx = kp.g[0] * sx, gy = kp.g[1] * sy, gz = kp.g[2] * sz;
  const double g2 = gx * gx + gy * gy + gz * gz;
  const double four_pi = 12.566370614359172953850573533118011537;
  double v;
  if (g2 == 0.0) {
    v = (kp.kind == 0) ? 0.0 : 3.14159265358979323846264338327950288 / (kp.omega * kp.omega);
  } else if (kp.kind == 0) {
    v = four_pi / g2;
  } else {
    v = -four_pi / g2 * expm1(-g2 / (4.0 * kp.omega * kp.omega));
  }
  return T(v * kp.inv_ng);
}

template <typename T, int NT>
__device__ __forceinline__ void block_sum2(T a, T b, double* out, double* red) {
  double x = a, y = b;
  for (int off = 32; off > 0; off >>= 1) {
    x += __shfl_down(x, off, 64);
    y += __shfl_down(y, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { red[2 * wv] = x; red[2 * wv + 1] = y; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0, sy = 0;
    for (int w = 0; w < NT / 64; ++w) { sx += red[2 * w]; sy += red[2 * w + 1]; }
    out[0] = sx; out[1] = sy;
  }
}


// W_i -= v phi_j and (i != j) W_j -= v phi_i for the E grid points starting
// at ro, with v = Re (pair a) and Im (pair b) of buf; with W == nullptr only
// the energy sums are formed.  Optional partial sums of v rho go to eslot.
template <typename T, int NT, bool EN>
__device__ __forceinline__ void accumulate_w(const T* __restrict__ phi, const Pack& pk, size_t NG, size_t ro, int E,
                                             T* W, double* eslot, const cplx<T>* buf, double* red, int tid) {
  const T* pia = phi + size_t(pk.ia) * NG + ro;
  const T* pja = phi + size_t(pk.ja) * NG + ro;
  T ea = T(0), eb = T(0);
  const bool offa = pk.ia != pk.ja;
  if (W) {
    T* wia = W + size_t(pk.ia) * NG + ro;
    T* wja = W + size_t(pk.ja) * NG + ro;
    for (int e = tid; e < E; e += NT) {
      const T v = buf[e].x, fi = pia[e], fj = pja[e];
      wia[e] -= v * fj;
      if (offa) wja[e] -= v * fi;
      if (EN) ea += v * fi * fj;
    }
  } else if (EN) {
    for (int e = tid; e < E; e += NT) ea += buf[e].x * pia[e] * pja[e];
  }
  if (pk.jb >= 0) {
    const T* pib = phi + size_t(pk.ib) * NG + ro;
    const T* pjb = phi + size_t(pk.jb) * NG + ro;
    const bool offb = pk.ib != pk.jb;
    if (W) {
      T* wib = W + size_t(pk.ib) * NG + ro;
      T* wjb = W + size_t(pk.jb) * NG + ro;
      for (int e = tid; e < E; e += NT) {
        const T v = buf[e].y, fi = pib[e], fj = pjb[e];
        wib[e] -= v * fj;
        if (offb) wjb[e] -= v * fi;
        if (EN) eb += v * fi * fj;
      }
    } else if (EN) {
      for (int e = tid; e < E; e += NT) eb += buf[e].y * pib[e] * pjb[e];
    }
  }
  if (EN) block_sum2<T, NT>(ea, eb, eslot, red);
}

// x pass, forward: product of the pack's two pairs over ROWS rows starting at
// linear offset ro, row FFTs, store.
template <typename T, int N, int ROWS, int NT, int V = 0>
__device__ __forceinline__ void body_fwd_x(const T* __restrict__ phi, cplx<T>* spec_p, const Pack& pk, size_t ro,
                                           cplx<T>* buf, const cplx<T>* tw, int tid) {
  using C = cplx<T>;
  constexpr size_t NG = size_t(N) * N * N;
  constexpr int E = ROWS * N;
  const T* pia = phi + size_t(pk.ia) * NG + ro;
  const T* pja = phi + size_t(pk.ja) * NG + ro;
  if (pk.jb >= 0) {
    const T* pib = phi + size_t(pk.ib) * NG + ro;
    const T* pjb = phi + size_t(pk.jb) * NG + ro;
    for (int e = tid; e < E; e += NT) { C v; v.x = pia[e] * pja[e]; v.y = pib[e] * pjb[e]; buf[e] = v; }
  } else {
    for (int e = tid; e < E; e += NT) { C v; v.x = pia[e] * pja[e]; v.y = T(0); buf[e] = v; }
  }
  __syncthreads();
  fft_lines<T, N, ROWS, N, 1, NT, -1, true, V>(buf, tw, tid);
  C* out = spec_p + ro;
  for (int e = tid; e < E; e += NT) out[e] = buf[e];
}

// Lines along y for the x-tile [x0, x0 + TX) of plane z, forward (S = -1) or
// inverse (S = +1); in place.
template <typename T, int N, int TX, int NT, int S, int V = 0>
__device__ __forceinline__ void body_line_y(cplx<T>* spec_p, int x0, int z, cplx<T>* buf, const cplx<T>* tw, int tid) {
  constexpr int E = N * TX;
  cplx<T>* base = spec_p + size_t(z) * N * N + x0;
  for (int e = tid; e < E; e += NT) buf[e] = base[size_t(e / TX) * N + (e % TX)];
  __syncthreads();
  fft_lines<T, N, TX, 1, TX, NT, S, false, V>(buf, tw, tid);
  for (int e = tid; e < E; e += NT) base[size_t(e / TX) * N + (e % TX)] = buf[e];
}

// Lines along z for the x-tile [x0, x0 + TX) of row y: forward FFT, multiply
// by v(G)/N^3, inverse FFT; in place.
template <typename T, int N, int TX, int NT, int V = 0>
__device__ __forceinline__ void body_conv_z(cplx<T>* spec_p, int x0, int y, const KernelParams& kp, cplx<T>* buf,
                                            const cplx<T>* tw, int tid) {
  using C = cplx<T>;
  constexpr int E = N * TX;
  C* base = spec_p + size_t(y) * N + x0;
  for (int e = tid; e < E; e += NT) buf[e] = base[size_t(e / TX) * N * N + (e % TX)];
  __syncthreads();
  fft_lines<T, N, TX, 1, TX, NT, -1, false, V>(buf, tw, tid);
  for (int e = tid; e < E; e += NT) {
    const T v = kernel_value<T, N>(kp, x0 + e % TX, y, e / TX);
    C c = buf[e];
    c.x *= v; c.y *= v;
    buf[e] = c;
  }
  __syncthreads();
  fft_lines<T, N, TX, 1, TX, NT, +1, false, V>(buf, tw, tid);
  for (int e = tid; e < E; e += NT) base[size_t(e / TX) * N * N + (e % TX)] = buf[e];
}

// x pass, inverse: row FFTs of the potentials, then W_i -= v phi_j and
// (i != j) W_j -= v phi_i for both pairs of the pack; optional partial sums
// of v rho for the pair energies into eslot[0..1].
template <typename T, int N, int ROWS, int NT, bool EN, int V = 0>
__device__ __forceinline__ void body_inv_x(const T* __restrict__ phi, const cplx<T>* spec_p, const Pack& pk, size_t ro,
                                           T* W, double* eslot, cplx<T>* buf, const cplx<T>* tw, double* red,
                                           int tid) {
  constexpr size_t NG = size_t(N) * N * N;
  constexpr int E = ROWS * N;
  const cplx<T>* in = spec_p + ro;
  for (int e = tid; e < E; e += NT) buf[e] = in[e];
  __syncthreads();
  fft_lines<T, N, ROWS, N, 1, NT, +1, true, V>(buf, tw, tid);
  accumulate_w<T, NT, EN>(phi, pk, NG, ro, E, W, eslot, buf, red, tid);
}

}  // namespace ace
