// Complex Bloch orbitals with k-points: the pair stage and the small dense
// kernels of the k-point build.
//
// The orbitals are Bloch functions psi_a(r) = exp(i k_a.r) u_a(r), held by
// their cell-periodic parts u (complex, [a][z][y][x], a = q * norb + m over
// k-point q and band m).  The screening criterion of Sec. Theory is written
// with phi_j*; for the pair (a, b) the density conj(psi_a) psi_b carries the
// Bloch phase exp(i (k_b - k_a).r), so its convolution with the lattice-summed
// kernel (Eq. e:vij) is that phase times
//     V = IFFT( v(|G + d|) FFT(conj(u_a) u_b) ),   d = k_b - k_a,
// and, with the Brillouin-zone average c = 1/N_k, Eq. (vx) on the periodic
// parts reads w_b -= c u_a V and, for a != b, w_a -= c u_b conj(V) (the kernel
// is real and depends on |G + d| only, so the pair (b, a) transforms to
// conj(V)).  Every pair is one full complex N^3 field: there is no Hermitian
// symmetry to halve it and no second pair to pack into its imaginary part.
//
// The passes are the split ones of the real build (x rows in LDS, y and z
// lines over x-tiles), with W updated by read-modify-write in conflict-free
// rounds: within one launch no orbital appears in two pairs.
#include <hip/hip_runtime.h>

#include "ace_internal.h"
#include "fft.h"
#include "pair_phases.h"

namespace ace {

// v(|G + d|) / N^3 at integer frequencies (kx, ky, kz) in FFT order.
template <int N>
__device__ __forceinline__ double kernel_value_shift(const KernelParams& kp, const double* d, int kx, int ky, int kz) {
  const int sx = kx < (N + 1) / 2 ? kx : kx - N;
  const int sy = ky < (N + 1) / 2 ? ky : ky - N;
  const int sz = kz < (N + 1) / 2 ? kz : kz - N;
  const double gx = kp.g[0] * sx + d[0], gy = kp.g[1] * sy + d[1], gz = kp.g[2] * sz + d[2];
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
  return v * kp.inv_ng;
}

// Forward x pass: f = conj(u_a) u_b over ROWS rows, row FFTs, store.
template <int N, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_kfwd_x(const double2* __restrict__ u, double2* __restrict__ spec,
                                               const KPair* __restrict__ slots, const double2* __restrict__ twg) {
  constexpr size_t NG = size_t(N) * N * N;
  constexpr int E = ROWS * N;
  __shared__ double2 buf[E];
  __shared__ double2 tw[N];
  const KPair kq = slots[blockIdx.y];
  if (kq.b < 0) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const size_t ro = size_t(blockIdx.x) * E;
  const double2* ua = u + size_t(kq.a) * NG + ro;
  const double2* ub = u + size_t(kq.b) * NG + ro;
  for (int e = tid; e < E; e += NT) {
    const double2 x = ua[e], y = ub[e];
    double2 f;
    f.x = x.x * y.x + x.y * y.y;  // conj(x) * y
    f.y = x.x * y.y - x.y * y.x;
    buf[e] = f;
  }
  __syncthreads();
  fft_lines<double, N, ROWS, N, 1, NT, -1, true>(buf, tw, tid);
  double2* out = spec + size_t(blockIdx.y) * NG + ro;
  for (int e = tid; e < E; e += NT) out[e] = buf[e];
}

// y lines of the x-tile [x0, x0 + TX) of plane z, forward (S = -1) or inverse.
template <int N, int TX, int NT, int S>
__global__ __launch_bounds__(NT) void k_kline_y(double2* __restrict__ spec, const KPair* __restrict__ slots,
                                                const double2* __restrict__ twg) {
  __shared__ double2 buf[N * TX];
  __shared__ double2 tw[N];
  if (slots[blockIdx.z].b < 0) return;
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  body_line_y<double, N, TX, NT, S>(spec + size_t(blockIdx.z) * N * N * N, blockIdx.x * TX, blockIdx.y, buf, tw,
                                    threadIdx.x);
}

// z lines of the x-tile [x0, x0 + TX) of row y: forward FFT, times
// v(|G + d|) / N^3 with the slot's shift d, inverse FFT; in place.
template <int N, int TX, int NT>
__global__ __launch_bounds__(NT) void k_kconv_z(double2* __restrict__ spec, const KPair* __restrict__ slots,
                                                const double2* __restrict__ twg, KernelParams kp) {
  constexpr int E = N * TX;
  __shared__ double2 buf[E];
  __shared__ double2 tw[N];
  const KPair kq = slots[blockIdx.z];
  if (kq.b < 0) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const int x0 = blockIdx.x * TX, y = blockIdx.y;
  double2* base = spec + size_t(blockIdx.z) * N * N * N + size_t(y) * N + x0;
  for (int e = tid; e < E; e += NT) buf[e] = base[size_t(e / TX) * N * N + (e % TX)];
  __syncthreads();
  fft_lines<double, N, TX, 1, TX, NT, -1, false>(buf, tw, tid);
  for (int e = tid; e < E; e += NT) {
    const double v = kernel_value_shift<N>(kp, kq.d, x0 + e % TX, y, e / TX);
    double2 c = buf[e];
    c.x *= v;
    c.y *= v;
    buf[e] = c;
  }
  __syncthreads();
  fft_lines<double, N, TX, 1, TX, NT, +1, false>(buf, tw, tid);
  for (int e = tid; e < E; e += NT) base[size_t(e / TX) * N * N + (e % TX)] = buf[e];
}

// Inverse x pass: row FFTs give V; then w_b -= c u_a V and, for a != b,
// w_a -= c u_b conj(V).
template <int N, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_kinv_x(const double2* __restrict__ u, const double2* __restrict__ spec,
                                               const KPair* __restrict__ slots, double2* __restrict__ W,
                                               const double2* __restrict__ twg, double c) {
  constexpr size_t NG = size_t(N) * N * N;
  constexpr int E = ROWS * N;
  __shared__ double2 buf[E];
  __shared__ double2 tw[N];
  const KPair kq = slots[blockIdx.y];
  if (kq.b < 0) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const size_t ro = size_t(blockIdx.x) * E;
  const double2* in = spec + size_t(blockIdx.y) * NG + ro;
  for (int e = tid; e < E; e += NT) buf[e] = in[e];
  __syncthreads();
  fft_lines<double, N, ROWS, N, 1, NT, +1, true>(buf, tw, tid);
  const double2* ua = u + size_t(kq.a) * NG + ro;
  const double2* ub = u + size_t(kq.b) * NG + ro;
  double2* wa = W + size_t(kq.a) * NG + ro;
  double2* wb = W + size_t(kq.b) * NG + ro;
  const bool off = kq.a != kq.b;
  for (int e = tid; e < E; e += NT) {
    const double2 V = buf[e], xa = ua[e];
    double2 t = wb[e];
    t.x -= c * (xa.x * V.x - xa.y * V.y);
    t.y -= c * (xa.x * V.y + xa.y * V.x);
    wb[e] = t;
    if (off) {
      const double2 xb = ub[e];
      double2 s = wa[e];
      s.x -= c * (xb.x * V.x + xb.y * V.y);  // u_b conj(V)
      s.y -= c * (xb.y * V.x - xb.x * V.y);
      wa[e] = s;
    }
  }
}

template <int N>
static hipError_t kpair_round_t(const void* u_, void* spec_, const KPair* slots, int nslots, void* W_,
                                const void* tw_, const KernelParams& kp, double c, hipStream_t s) {
  const double2* u = static_cast<const double2*>(u_);
  double2* spec = static_cast<double2*>(spec_);
  double2* W = static_cast<double2*>(W_);
  const double2* tw = static_cast<const double2*>(tw_);
  constexpr int TX = pick_tx(N);
  constexpr int ROWS = pick_rows(N);
  constexpr int NTL = 256;
  if (nslots <= 0) return hipSuccess;
  const int nrb = N * N / ROWS;
  hipLaunchKernelGGL((k_kfwd_x<N, ROWS, NTL>), dim3(nrb, nslots), dim3(NTL), 0, s, u, spec, slots, tw);
  hipLaunchKernelGGL((k_kline_y<N, TX, NTL, -1>), dim3(N / TX, N, nslots), dim3(NTL), 0, s, spec, slots, tw);
  hipLaunchKernelGGL((k_kconv_z<N, TX, NTL>), dim3(N / TX, N, nslots), dim3(NTL), 0, s, spec, slots, tw, kp);
  hipLaunchKernelGGL((k_kline_y<N, TX, NTL, +1>), dim3(N / TX, N, nslots), dim3(NTL), 0, s, spec, slots, tw);
  hipLaunchKernelGGL((k_kinv_x<N, ROWS, NTL>), dim3(nrb, nslots), dim3(NTL), 0, s, u, spec, slots, W, tw, c);
  return hipGetLastError();
}

hipError_t kpair_round(int N, const void* u, void* spec, const KPair* slots, int nslots, void* W, const void* tw,
                       const KernelParams& kp, double c, hipStream_t s) {
  switch (N) {
#define X(n) case n: return kpair_round_t<n>(u, spec, slots, nslots, W, tw, kp, c, s);
    X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(80) X(96) X(100) X(108) X(120) X(160)
#undef X
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------ dense kernels

// Wm = -i W (elementwise), so that with the interleaved (re, im) layout read
// as real rows, u . W = Re sum conj(u) W and u . Wm = Im sum conj(u) W.
__global__ void k_times_minus_i(const double2* __restrict__ W, double2* __restrict__ Wm, int64_t n) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const double2 w = W[t];
    double2 r;
    r.x = w.y;
    r.y = -w.x;
    Wm[t] = r;
  }
}

// Per k-point block: M = (R + i I), made Hermitian, (M + M^H) / 2; writes it
// (nullable), and -M for the factorization.
__global__ void k_hermitize(const double* __restrict__ Re, const double* __restrict__ Im, int n,
                            double2* __restrict__ Mout, double2* __restrict__ negM) {
  const size_t off = size_t(blockIdx.y) * n * n;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n * n; t += gridDim.x * blockDim.x) {
    const int i = t / n, j = t % n;
    double2 m;
    m.x = 0.5 * (Re[off + size_t(i) * n + j] + Re[off + size_t(j) * n + i]);
    m.y = 0.5 * (Im[off + size_t(i) * n + j] - Im[off + size_t(j) * n + i]);
    if (Mout) Mout[off + t] = m;
    double2 q;
    q.x = -m.x;
    q.y = -m.y;
    negM[off + t] = q;
  }
}

// E_x = (1/N_k) sum_k sum_n Re M_k[n][n], in a fixed order (one thread).
__global__ void k_trace_avg(const double* __restrict__ Re, int n, int nk, double* __restrict__ ex) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < nk; ++q) {
      double t = 0.0;
      for (int i = 0; i < n; ++i) t += Re[size_t(q) * n * n + size_t(i) * n + i];
      s += t;
    }
    ex[0] = s / nk;
  }
}

// In-place lower Cholesky A = L L^H of each k-point's Hermitian matrix, one
// workgroup per k-point, column by column; info[k] = column + 1 where the
// pivot is not positive, -(column + 1) where it is not finite, 0 otherwise.
__global__ __launch_bounds__(256) void k_chol_c(double2* __restrict__ A, int n, int* __restrict__ info) {
  __shared__ double red[256];
  __shared__ double piv;
  double2* L = A + size_t(blockIdx.x) * n * n;
  const int tid = threadIdx.x;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int p = tid; p < j; p += 256) {
      const double2 l = L[size_t(j) * n + p];
      s += l.x * l.x + l.y * l.y;
    }
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) red[tid] += red[tid + h];
      __syncthreads();
    }
    if (tid == 0) {
      const double d = L[size_t(j) * n + j].x - red[0];
      piv = d;
      if (!(d > 0.0) || !isfinite(d)) {
        info[blockIdx.x] = isfinite(d) ? j + 1 : -(j + 1);
      } else {
        double2 r;
        r.x = sqrt(d);
        r.y = 0.0;
        L[size_t(j) * n + j] = r;
      }
    }
    __syncthreads();
    if (!(piv > 0.0) || !isfinite(piv)) return;
    const double ljj = sqrt(piv);
    for (int i = j + 1 + tid; i < n; i += 256) {
      double2 a = L[size_t(i) * n + j];
      for (int p = 0; p < j; ++p) {
        const double2 x = L[size_t(i) * n + p], y = L[size_t(j) * n + p];
        a.x -= x.x * y.x + x.y * y.y;  // x * conj(y)
        a.y -= x.y * y.x - x.x * y.y;
      }
      a.x /= ljj;
      a.y /= ljj;
      L[size_t(i) * n + j] = a;
    }
    __syncthreads();
  }
}

// X = L^-1 for each k-point (lower triangular, one thread per column, forward
// substitution), written as its real and imaginary parts Xr, Xi (zero above
// the diagonal).
__global__ void k_trinv_c(const double2* __restrict__ Lm, int n, double* __restrict__ Xr, double* __restrict__ Xi) {
  const size_t off = size_t(blockIdx.y) * n * n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double2* L = Lm + off;
  double* xr = Xr + off;
  double* xi = Xi + off;
  for (int i = 0; i < j; ++i) {
    xr[size_t(i) * n + j] = 0.0;
    xi[size_t(i) * n + j] = 0.0;
  }
  for (int i = j; i < n; ++i) {
    double sr = (i == j) ? 1.0 : 0.0, si = 0.0;
    for (int p = j; p < i; ++p) {
      const double2 l = L[size_t(i) * n + p];
      const double ar = xr[size_t(p) * n + j], ai = xi[size_t(p) * n + j];
      sr -= l.x * ar - l.y * ai;
      si -= l.x * ai + l.y * ar;
    }
    const double d = L[size_t(i) * n + i].x;
    xr[size_t(i) * n + j] = sr / d;
    xi[size_t(i) * n + j] = si / d;
  }
}

// |u| of every complex grid value (the screening integrand |psi_a psi_b*|
// is |u_a| |u_b|).
__global__ void k_cabs(const double2* __restrict__ u, double* __restrict__ a, int64_t n) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
    const double2 z = u[t];
    a[t] = sqrt(z.x * z.x + z.y * z.y);
  }
}

static unsigned grid_for(int64_t n, int bs) { return unsigned(std::min<int64_t>((n + bs - 1) / bs, 65536)); }

void launch_times_minus_i(const void* W, void* Wm, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_times_minus_i, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<const double2*>(W),
                     static_cast<double2*>(Wm), n);
}
void launch_hermitize(const double* Re, const double* Im, int n, int nk, void* Mout, void* negM, hipStream_t s) {
  hipLaunchKernelGGL(k_hermitize, dim3(grid_for(int64_t(n) * n, 256), nk), dim3(256), 0, s, Re, Im, n,
                     static_cast<double2*>(Mout), static_cast<double2*>(negM));
}
void launch_trace_avg(const double* Re, int n, int nk, double* ex, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_avg, dim3(1), dim3(64), 0, s, Re, n, nk, ex);
}
void launch_chol_c(void* A, int n, int nk, int* info, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_c, dim3(nk), dim3(256), 0, s, static_cast<double2*>(A), n, info);
}
void launch_trinv_c(const void* L, int n, int nk, double* Xr, double* Xi, hipStream_t s) {
  hipLaunchKernelGGL(k_trinv_c, dim3((n + 63) / 64, nk), dim3(64), 0, s, static_cast<const double2*>(L), n, Xr, Xi);
}
void launch_cabs(const void* u, double* a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_cabs, dim3(grid_for(n, 256)), dim3(256), 0, s, static_cast<const double2*>(u), a, n);
}

}  // namespace ace
