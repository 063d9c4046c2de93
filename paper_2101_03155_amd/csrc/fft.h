// Batched mixed-radix FFT building blocks for gfx950 (CDNA4), operating on
// lines held in LDS.
//
// The pair Poisson solve of Eq. (e:vij) transforms every orbital-pair density
// to reciprocal space and back.  A line of length N (N = 2^a 3^b 5^c) is
// transformed by a sequence of Stockham autosort passes with radices 8, 4, 2,
// 3 and 5; each pass reads R elements per butterfly into registers, applies
// the twiddles and a length-R DFT, and writes them back to their
// sorted-order positions in the same LDS buffer (a barrier separates the
// reads from the writes, so one buffer suffices).  The radix plan, the number
// of butterflies per thread and all strides are compile-time constants, so
// every register array is statically indexed.
//
// Sign convention: forward uses exp(-2 pi i jk/N), inverse exp(+2 pi i jk/N),
// both unnormalized (the 1/N^3 of the inverse is folded into the kernel v(G)).
#pragma once
#include <hip/hip_runtime.h>

namespace ace {

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using cplx = typename cplx_t<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// multiply by conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  C r; r.x = a.x * b.x + a.y * b.y; r.y = a.y * b.x - a.x * b.y; return r;
}
// multiply by s*i (s = +1 or -1)
template <int S, typename C> __device__ __forceinline__ C cmul_si(C a) {
  C r;
  if (S > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; }
  return r;
}
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }

// ---------------------------------------------------------------- radix plan
// 2^a is split into radix-8 passes with a 4,4 / 4 / 2 remainder; then one
// radix-3 pass per factor 3 and one radix-5 pass per factor 5.
constexpr int pow_of(int n, int p) { int a = 0; while (n % p == 0) { n /= p; ++a; } return a; }
constexpr bool smooth235(int n) {
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  while (n % 5 == 0) n /= 5;
  return n == 1;
}
// The grid sizes of the pair stage whose factors do not pair up into radix-8
// passes take composite radices 9, 10, 12 and 16 instead (two passes, so two
// LDS round trips per line rather than three or four).
constexpr int plan_fill(int n, int* r) {
  switch (n) {
    case 12: r[0] = 12; return 1;
    case 16: r[0] = 16; return 1;
    case 48: r[0] = 4; r[1] = 12; return 2;
    case 80: r[0] = 8; r[1] = 10; return 2;
    case 96: r[0] = 8; r[1] = 12; return 2;
    case 100: r[0] = 10; r[1] = 10; return 2;
    case 108: r[0] = 12; r[1] = 9; return 2;
    case 120: r[0] = 12; r[1] = 10; return 2;
    case 160: r[0] = 16; r[1] = 10; return 2;
    default: break;
  }
  int a = pow_of(n, 2), cnt = 0;
  while (a >= 3 && a != 4) { a -= 3; r[cnt++] = 8; }
  if (a == 4) { r[cnt++] = 4; r[cnt++] = 4; } else if (a == 2) r[cnt++] = 4; else if (a == 1) r[cnt++] = 2;
  for (int i = 0; i < pow_of(n, 3); ++i) r[cnt++] = 3;
  for (int i = 0; i < pow_of(n, 5); ++i) r[cnt++] = 5;
  return cnt;
}
constexpr int plan_len(int n) {
  int r[24] = {0};
  return plan_fill(n, r);
}
constexpr int plan_radix(int n, int p) {
  int r[24] = {0};
  plan_fill(n, r);
  return r[p];
}
// Plan variants: 0 takes the radices in the order above, 1 in reverse order
// (small radices first).  Both give the same transform; the tuner picks.
constexpr int plan_radix_v(int n, int p, int v) { return v == 0 ? plan_radix(n, p) : plan_radix(n, plan_len(n) - 1 - p); }
// product of the radices of passes 0..p-1
constexpr int plan_ns(int n, int p, int v = 0) {
  int s = 1;
  for (int i = 0; i < p; ++i) s *= plan_radix_v(n, i, v);
  return s;
}

// ---------------------------------------------------------------- small DFTs
// In-register DFT of length R with exponent sign S (-1 forward, +1 inverse).
template <int R, int S, typename C> struct Dft;

template <int S, typename C> struct Dft<2, S, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  }
};

template <int S, typename C> struct Dft<3, S, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T h = T(0.866025403784438646763723170752936183);  // sin(2 pi/3)
    C t1 = cadd(v[1], v[2]);
    C t2 = csub(v[0], cscale(t1, T(0.5)));
    C t3 = cmul_si<S>(cscale(csub(v[1], v[2]), h));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  }
};

template <int S, typename C> struct Dft<4, S, C> {
  static __device__ __forceinline__ void run(C* v) {
    C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
    C c = cadd(v[1], v[3]), d = cmul_si<S>(csub(v[1], v[3]));
    v[0] = cadd(a, c); v[2] = csub(a, c);
    v[1] = cadd(b, d); v[3] = csub(b, d);
  }
};

template <int S, typename C> struct Dft<5, S, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T c1 = T(0.309016994374947424102293417182819059);   // cos(2 pi/5)
    const T c2 = T(-0.809016994374947424102293417182819059);  // cos(4 pi/5)
    const T s1 = T(0.951056516295153572116439333379382143);   // sin(2 pi/5)
    const T s2 = T(0.587785252292473129168705954639072769);   // sin(4 pi/5)
    C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
    C t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
    C a1 = cadd(v[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    C a2 = cadd(v[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    C b1 = cmul_si<S>(cadd(cscale(t3, s1), cscale(t4, s2)));
    C b2 = cmul_si<S>(csub(cscale(t3, s2), cscale(t4, s1)));
    v[0] = cadd(v[0], cadd(t1, t2));
    v[1] = cadd(a1, b1); v[4] = csub(a1, b1);
    v[2] = cadd(a2, b2); v[3] = csub(a2, b2);
  }
};

template <int S, typename C> struct Dft<8, S, C> {
  static __device__ __forceinline__ void run(C* v) {
    using T = decltype(v[0].x);
    const T r2 = T(0.707106781186547524400844362104849039);
    C e[4] = {v[0], v[2], v[4], v[6]};
    C o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, S, C>::run(e);
    Dft<4, S, C>::run(o);
    // o[k] *= W8^k with W8 = (1 + S i)/sqrt 2
    C o1; o1.x = r2 * (o[1].x - S * o[1].y); o1.y = r2 * (o[1].y + S * o[1].x);
    C o2 = cmul_si<S>(o[2]);
    C o3; o3.x = r2 * (-o[3].x - S * o[3].y); o3.y = r2 * (-o[3].y + S * o[3].x);
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);   v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);   v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);   v[7] = csub(e[3], o3);
  }
};

// Composite lengths R = R1 R2 by one Cooley-Tukey step in registers:
// x[R2 n1 + n2] -> R2 DFTs of length R1 over n1, twiddles w^(n2 k1) with
// w = exp(S 2 pi i / R), then R1 DFTs of length R2 over n2, giving
// X[k1 + R1 k2].  The twiddles are compile-time constants.
constexpr double cx_sin_red(double x) {  // Taylor series, |x| <= pi/4
  double t = x, sum = x;
  for (int k = 1; k < 40; ++k) {
    t *= -x * x / double((2 * k) * (2 * k + 1));
    sum += t;
  }
  return sum;
}
constexpr double cx_cos_red(double x) {
  double t = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    t *= -x * x / double((2 * k - 1) * (2 * k));
    sum += t;
  }
  return sum;
}
// cos (c = true) or sin of 2 pi m / R: the angle is reduced to |x| <= pi/4
// by the half-turn and quarter-turn symmetries before the series
constexpr double root_cs(int m, int R, bool c) {
  const double pi = 3.141592653589793238462643383279502884;
  const int mm = ((m % R) + R) % R;
  double x = 2.0 * pi * double(2 * mm > R ? mm - R : mm) / double(R);  // in (-pi, pi]
  double sg = 1.0;
  if (x > pi / 2) { x -= pi; sg = -1.0; }
  else if (x < -pi / 2) { x += pi; sg = -1.0; }
  if (x > pi / 4) return sg * (c ? cx_sin_red(pi / 2 - x) : cx_cos_red(pi / 2 - x));
  if (x < -pi / 4) return sg * (c ? cx_sin_red(pi / 2 + x) : -cx_cos_red(pi / 2 + x));
  return sg * (c ? cx_cos_red(x) : cx_sin_red(x));
}
constexpr double root_cos(int m, int R) { return root_cs(m, R, true); }
constexpr double root_sin(int m, int R) { return root_cs(m, R, false); }

template <int M, int R, int S, typename C>
__device__ __forceinline__ C rotate(C a) {
  using T = decltype(a.x);
  constexpr int m = M % R;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (4 * m == R) {
    return cmul_si<S>(a);
  } else if constexpr (2 * m == R) {
    C r; r.x = -a.x; r.y = -a.y; return r;
  } else if constexpr (4 * m == 3 * R) {
    return cmul_si<-S>(a);
  } else {
    constexpr T c = T(root_cos(m, R)), sn = T(S * root_sin(m, R));
    // explicit fused multiply-adds: the rounding does not depend on how the
    // compiler contracts the expression in a given kernel
    C r; r.x = fma(a.x, c, -(a.y * sn)); r.y = fma(a.x, sn, a.y * c); return r;
  }
}

template <int R1, int R2, int S, typename C, int N2, int K = 0>
__device__ __forceinline__ void ct_twiddle_row(C (&y)[R2][R1]) {
  if constexpr (K < R1) {
    y[N2][K] = rotate<N2 * K, R1 * R2, S>(y[N2][K]);
    ct_twiddle_row<R1, R2, S, C, N2, K + 1>(y);
  }
}
template <int R1, int R2, int S, typename C, int N2 = 0>
__device__ __forceinline__ void ct_twiddle(C (&y)[R2][R1]) {
  if constexpr (N2 < R2) {
    ct_twiddle_row<R1, R2, S, C, N2>(y);
    ct_twiddle<R1, R2, S, C, N2 + 1>(y);
  }
}

template <int R1, int R2, int S, typename C>
__device__ __forceinline__ void dft_ct(C* v) {
  C y[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) y[n2][n1] = v[R2 * n1 + n2];
    Dft<R1, S, C>::run(y[n2]);
  }
  ct_twiddle<R1, R2, S, C>(y);
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    C z[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) z[n2] = y[n2][k1];
    Dft<R2, S, C>::run(z);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = z[k2];
  }
}

template <int S, typename C> struct Dft<9, S, C> {
  static __device__ __forceinline__ void run(C* v) { dft_ct<3, 3, S, C>(v); }
};
template <int S, typename C> struct Dft<10, S, C> {
  static __device__ __forceinline__ void run(C* v) { dft_ct<2, 5, S, C>(v); }
};
template <int S, typename C> struct Dft<12, S, C> {
  static __device__ __forceinline__ void run(C* v) { dft_ct<4, 3, S, C>(v); }
};
template <int S, typename C> struct Dft<16, S, C> {
  static __device__ __forceinline__ void run(C* v) { dft_ct<4, 4, S, C>(v); }
};

// ---------------------------------------------------------------- one pass
// LINES lines of length N in LDS; element p of line l at buf[l*LS + p*PS].
// JFAST: consecutive threads take consecutive butterflies of one line
// (unit-stride lines) rather than the same butterfly of consecutive lines.
// The pass's inputs come from load(l, p) (by default buf[l*LS + p*PS]); all
// of them are read before the barrier, so a first pass may read another
// layout of the same buffer than the one it writes, or global memory.  Its
// outputs go to store(l, p, value) (by default buf[l*LS + p*PS] = value),
// followed by a barrier unless END_SYNC is false (a last pass storing to
// global memory; the barrier between reads and writes stays, so the buffer's
// previous contents are read by all threads before a first pass writes it).
// WROT: threads whose butterfly index j has bit 2 set store their R outputs
// in an order rotated by WROT (same values, same places, other instructions),
// which moves their writes to other banks than those of threads j - 4.
template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, bool END_SYNC,
          int WROT = 0, typename L, typename St>
__device__ __forceinline__ void fft_pass_ls(cplx<T>* buf, const cplx<T>* tw, int tid, L load, St store);

template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, int WROT = 0,
          typename L>
__device__ __forceinline__ void fft_pass_l(cplx<T>* buf, const cplx<T>* tw, int tid, L load) {
  fft_pass_ls<T, N, P, LINES, LS, PS, NT, S, JFAST, V, true, WROT>(
      buf, tw, tid, load, [buf](int l, int p, cplx<T> x) { buf[l * LS + p * PS] = x; });
}

template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V>
__device__ __forceinline__ void fft_pass(cplx<T>* buf, const cplx<T>* tw, int tid) {
  fft_pass_l<T, N, P, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid,
                                                      [buf](int l, int p) { return buf[l * LS + p * PS]; });
}

template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, bool END_SYNC,
          int WROT, typename L, typename St>
__device__ __forceinline__ void fft_pass_ls(cplx<T>* buf, const cplx<T>* tw, int tid, L load, St store) {
  using C = cplx<T>;
  constexpr int R = plan_radix_v(N, P, V);
  constexpr int NS = plan_ns(N, P, V);
  constexpr int NB = N / R;
  constexpr int TOT = LINES * NB;
  constexpr int PER = (TOT + NT - 1) / NT;
  constexpr int TSTEP = N / (NS * R);
  C v[PER][R];
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if ((TOT % NT) == 0 || b < TOT) {
      const int l = JFAST ? b / NB : b % LINES;
      const int j = JFAST ? b % NB : b / LINES;
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = load(l, j + r * NB);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int b = tid + s * NT;
    if ((TOT % NT) == 0 || b < TOT) {
      const int l = JFAST ? b / NB : b % LINES;
      const int j = JFAST ? b % NB : b / LINES;
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const C w = tw[r * k * TSTEP];
          v[s][r] = (S < 0) ? cmul(v[s][r], w) : cmulc(v[s][r], w);
        }
      }
      Dft<R, S, C>::run(v[s]);
      const int o = (j / NS) * NS * R + k;
      const bool rot = WROT != 0 && (j & 4) != 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (WROT == 0) {
          store(l, o + r * NS, v[s][r]);
        } else {
          const int r2 = (r + WROT) % R;
          // (the empty asm keeps the two values in registers: a select of
          // the array elements themselves becomes an indexed load, which
          // moves the whole array to scratch memory)
          C a = v[s][r], b = v[s][r2];
          asm("" : "+v"(a.x), "+v"(a.y), "+v"(b.x), "+v"(b.y));
          C x;
          x.x = rot ? b.x : a.x;
          x.y = rot ? b.y : a.y;
          store(l, o + (rot ? r2 : r) * NS, x);
        }
      }
    }
  }
  if (END_SYNC) __syncthreads();
}

template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V>
__device__ __forceinline__ void fft_lines_from(cplx<T>* buf, const cplx<T>* tw, int tid) {
  if constexpr (P < plan_len(N)) {
    fft_pass<T, N, P, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid);
    fft_lines_from<T, N, P + 1, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid);
  }
}

// Full length-N transform of LINES lines held in LDS.  tw[m] = exp(-2 pi i m/N).
// Expects the caller to have synchronized after filling buf; ends synchronized.
template <typename T, int N, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V = 0>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, const cplx<T>* tw, int tid) {
  static_assert(smooth235(N), "FFT length must be 2^a 3^b 5^c");
  fft_lines_from<T, N, 0, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid);
}

// Passes P .. plan_len(N) - 2 in place, then the last pass through the storer
// (followed by a barrier if ES, for a storer that writes LDS).
template <typename T, int N, int P, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, bool ES = false,
          typename St>
__device__ __forceinline__ void fft_lines_to(cplx<T>* buf, const cplx<T>* tw, int tid, St store) {
  if constexpr (P + 1 < plan_len(N)) {
    fft_pass<T, N, P, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid);
    fft_lines_to<T, N, P + 1, LINES, LS, PS, NT, S, JFAST, V, ES>(buf, tw, tid, store);
  } else {
    fft_pass_ls<T, N, P, LINES, LS, PS, NT, S, JFAST, V, ES>(
        buf, tw, tid, [buf](int l, int p) { return buf[l * LS + p * PS]; }, store);
  }
}

// Full transform with the first pass reading through load(l, p) and the last
// writing through store(l, p, value) (to global memory: no closing barrier,
// unless ES).  Expects nothing of buf (the first pass fills it after a
// barrier); ends unsynchronized unless ES.
template <typename T, int N, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, bool ES = false,
          typename L, typename St>
__device__ __forceinline__ void fft_lines_ls(cplx<T>* buf, const cplx<T>* tw, int tid, L load, St store) {
  static_assert(smooth235(N), "FFT length must be 2^a 3^b 5^c");
  if constexpr (plan_len(N) == 1) {
    fft_pass_ls<T, N, 0, LINES, LS, PS, NT, S, JFAST, V, ES>(buf, tw, tid, load, store);
  } else {
    fft_pass_l<T, N, 0, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid, load);
    fft_lines_to<T, N, 1, LINES, LS, PS, NT, S, JFAST, V, ES>(buf, tw, tid, store);
  }
}

// The same, with the first pass reading its inputs through load(l, p) (an
// element-wise step fused into the transform's first LDS read).
template <typename T, int N, int LINES, int LS, int PS, int NT, int S, bool JFAST, int V, typename L>
__device__ __forceinline__ void fft_lines_load(cplx<T>* buf, const cplx<T>* tw, int tid, L load) {
  static_assert(smooth235(N), "FFT length must be 2^a 3^b 5^c");
  fft_pass_l<T, N, 0, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid, load);
  fft_lines_from<T, N, 1, LINES, LS, PS, NT, S, JFAST, V>(buf, tw, tid);
}

}  // namespace ace
