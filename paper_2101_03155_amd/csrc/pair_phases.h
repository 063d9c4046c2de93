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


// Copy E elements to LDS (dst[e] = src(e)) with every global load of a thread
// issued before its first LDS store, so a workgroup keeps all its loads in
// flight at once.
template <typename C, int E, int NT, typename F>
__device__ __forceinline__ void stage_in(C* dst, F src, int tid) {
  constexpr int LP = (E + NT - 1) / NT;
  C r[LP];
#pragma unroll
  for (int q = 0; q < LP; ++q) {
    const int e = tid + q * NT;
    if (E % NT == 0 || e < E) r[q] = src(e);
  }
#pragma unroll
  for (int q = 0; q < LP; ++q) {
    const int e = tid + q * NT;
    if (E % NT == 0 || e < E) dst[e] = r[q];
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


// ------------------------------------------------------------ real-to-complex path
// One orbital pair per workgroup and z-plane.  The x transform of the real
// pair density uses the two-for-one trick: rows y and y + N/2 form one
// complex line Z, and after its FFT the two half spectra are separated as
// X1[k] = (Z[k] + conj Z[N-k]) / 2, X2[k] = (Z[k] - conj Z[N-k]) / 2i for
// 0 <= k <= N/2.  The plane then holds N rows of XS = N/2 + 1 complex values
// (the non-negative x frequencies; the others follow by Hermitian symmetry)
// and the y and z transforms act on those columns only.  The spectrum of a
// pair is [z][y][kx], N * N * XS complex values, and the z pass runs over
// tiles of consecutive (y, kx) columns of the flattened planes.

template <int N> __host__ __device__ constexpr int r2c_xs() { return N / 2 + 1; }
// v(G) depends on ky and kz through ky^2 and kz^2 only, so its table holds the
// folded frequencies min(k, N - k) of y and z: [zq][yq][kx], each of y and z
// N/2 + 1 values, an eighth of the spectrum plane set, which stays in L2.
template <int N> __host__ __device__ constexpr int vt_half() { return N / 2 + 1; }
template <int N> __device__ __forceinline__ int vt_fold(int k) { return k <= N / 2 ? k : N - k; }
// LDS stride of the packed x lines of the in-plane transforms: one complex
// value of padding per line, so that consecutive lines start in different
// banks.  The passes that read their inputs from LDS give consecutive threads
// the same butterfly of consecutive lines, which then hit distinct banks.
// With unpadded lines and consecutive butterflies of one line per thread
// group, the Stockham writes of a line fall on a few banks: bank conflicts
// took over half of the LDS cycles of the owner pass and the forward at 96^3.
template <int N> __host__ __device__ constexpr int xls() { return N + 1; }
// position in buf of element e = l * N + x of the packed potential lines
template <int N> __device__ __forceinline__ int xpos(int e) { return e + e / N * (xls<N>() - N); }
// LDS layout of the inverse in-plane transforms (V: the y passes' plan order;
// the x passes take the other).  The y-transformed plane is [y][kx] at row
// stride XS, and the x passes' first pass re-packs rows l and l + N/2 into x
// line l (stride N + 1).  Where that pass has eight threads per line and N is
// a multiple of 32, the last y pass writes row y to row ysig(y), which
// interleaves each block of 32 rows so that the rows read by the 8-thread
// groups served in one LDS cycle start in disjoint bank ranges (rows l and
// l + 1 start one FP64 value apart, and their 8-value ranges overlapped).
// Its writes (element 12 j + r of a line from thread j, radix 12) hit each
// FP64 bank group twice, threads j and j + 4 alike; threads j >= 4 store in
// an order rotated by 2 (WROT), which puts them on the other half of the
// bank groups.  (Padding the x lines instead made the FP64 owner kernel
// spill registers.)  FP32 writes are conflict-free without the rotation.
template <typename T, int N, int V> struct InvLayout {
  static constexpr int XS = r2c_xs<N>();
  static constexpr int R0 = plan_radix_v(N, 0, V ^ 1);
  static constexpr bool SIG = N % 32 == 0 && N / R0 == 8;
  static constexpr int WROT = sizeof(T) == 8 && SIG && R0 == 12 ? 2 : 0;
  static constexpr int XL = xls<N>();
  static __host__ __device__ __forceinline__ int ysig(int y) {
    return SIG ? (y & ~31) | ((y & 3) << 3) | ((y & 31) >> 2) : y;
  }
  static __host__ __device__ __forceinline__ int xq(int l, int p) { return l * XL + p; }
};
template <int N> __host__ __device__ constexpr int r2c_tx() {
  return (N * r2c_xs<N>()) % 16 == 0 ? 16 : (N * r2c_xs<N>()) % 8 == 0 ? 8 : (N * r2c_xs<N>()) % 4 == 0 ? 4 : 2;
}
// z-pass tile of the owner paths: 32 columns of each plane row per tile (512
// bytes FP64, 256 bytes FP32; 16 FP64 columns measured 10% slower at 96^3,
// 64 columns or 512 threads slower in both precisions), the last tile of a
// slot ragged where the width does not divide N * XS.
template <typename T, int N> __host__ __device__ constexpr int own_tx() { return 32; }
template <typename T, int N> __host__ __device__ constexpr int own_ntile() {
  return (N * r2c_xs<N>() + own_tx<T, N>() - 1) / own_tx<T, N>();
}

// Pair density of plane z (phi_i, phi_j point at the plane) -> its half
// spectrum after the x and y transforms, stored to out (N * XS values).
template <typename T, int N, int NT, int V = 0>
__device__ __forceinline__ void body_fwd_xy_r(const T* __restrict__ pi_, const T* __restrict__ pj_, cplx<T>* out,
                                              cplx<T>* buf, const cplx<T>* tw, int tid) {
  using C = cplx<T>;
  constexpr int H = N / 2, XS = r2c_xs<N>();
  // The x transforms of the packed lines (line l: row l in .x, row l + H in
  // .y).  When the first pass has a butterfly for every thread it forms the
  // products from global memory itself (all of a thread's loads are issued
  // before the pass's barrier); otherwise (1024-thread workgroups) the
  // products are staged through LDS by all threads first, which keeps more
  // loads in flight (measured).
  auto prod = [pi_, pj_](int l, int p) {
    C v;
    v.x = pi_[l * N + p] * pj_[l * N + p];
    v.y = pi_[(l + H) * N + p] * pj_[(l + H) * N + p];
    return v;
  };
  // The lines sit at stride xls<N>() in LDS; the passes that read LDS give
  // consecutive threads the same butterfly of consecutive lines (distinct
  // banks), a first pass reading global memory consecutive butterflies of
  // one line (coalesced loads).  With 512 threads the radix order is
  // reversed: at 96^3 the larger first radix leaves fewer butterflies than
  // threads, so the products are staged and every pass reads LDS (8% faster;
  // slower with 1024 threads).
  constexpr int XL = xls<N>(), VX = NT <= 512 ? (V ^ 1) : V;
  if constexpr (H * (N / plan_radix_v(N, 0, VX)) >= NT) {
    fft_pass_l<T, N, 0, H, XL, 1, NT, -1, true, VX>(buf, tw, tid, prod);
    fft_lines_from<T, N, 1, H, XL, 1, NT, -1, false, VX>(buf, tw, tid);
  } else {
    constexpr int E = H * N, LP = (E + NT - 1) / NT;
    C r[LP];
#pragma unroll
    for (int q = 0; q < LP; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) r[q] = prod(e / N, e % N);
    }
#pragma unroll
    for (int q = 0; q < LP; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) buf[xpos<N>(e)] = r[q];
    }
    __syncthreads();
    fft_lines<T, N, H, XL, 1, NT, -1, false, VX>(buf, tw, tid);
  }
  // The y transforms of the half spectra, whose first pass separates the two
  // rows of each packed line on the way in: row y < H of column k is
  // X1 = (Z[k] + conj Z[N-k]) / 2 of line y, row y >= H is
  // X2 = (Z[k] - conj Z[N-k]) / 2i of line y - H (Z = line after the x
  // transform, still in the packed layout of buf); the last pass
  // stores the spectrum ([y][kx]) to global memory.
  auto sep = [buf](int k, int y) {
    const int l = y < H ? y : y - H;
    const C a = buf[l * XL + k], b = buf[l * XL + (k == 0 ? 0 : N - k)];
    C x;
    if (y < H) {
      x.x = T(0.5) * (a.x + b.x);
      x.y = T(0.5) * (a.y - b.y);
    } else {
      x.x = T(0.5) * (a.y + b.y);
      x.y = T(0.5) * (b.x - a.x);
    }
    return x;
  };
  fft_lines_ls<T, N, XS, 1, XS, NT, -1, false, V>(buf, tw, tid, sep,
                                                  [out](int l, int p, C x) { out[p * XS + l] = x; });
}

// z lines of the TX consecutive flattened columns starting at f0 of one
// pair's half spectrum: forward FFT, times v(G)/N^3, inverse FFT; in place.
// With active == false the caller's threads take part in the barriers only
// (no global loads or stores), so a workgroup can split into independent
// groups of NT threads working on different tiles.
// With eslot != nullptr the tile's share of sum_r rho v_ij is formed on the
// way (Parseval: sum_r rho v = sum_G (v(G)/N^3) |rho^(G)|^2, the half spectrum
// weighted 2 except at kx = 0 and N/2) and written to eslot[0]; red holds
// NT / 64 doubles.  vt (nullable): the kernel values v(G) of launch_vtable,
// [zq][yq][kx] over the folded z and y frequencies, read (before the forward
// transform, so the loads overlap it) instead of evaluated per element.
template <typename T, int N, int TX, int NT> __host__ __device__ constexpr int conv_lv() { return (N * TX + NT - 1) / NT; }

// The kernel values of the TX columns starting at f0 for the elements this
// thread multiplies in body_conv_z_r_v, from the folded table vt.
template <typename T, int N, int TX, int NT>
__device__ __forceinline__ void load_vtile(const T* __restrict__ vt, int f0, int tid, T (&vv)[conv_lv<T, N, TX, NT>()]) {
  constexpr int XS = r2c_xs<N>(), PL = N * XS, E = N * TX, LV = conv_lv<T, N, TX, NT>();
  const int ncol = PL - f0 < TX ? PL - f0 : TX;
#pragma unroll
  for (int q = 0; q < LV; ++q) {
    const int e = tid + q * NT;
    if ((E % NT == 0 || e < E) && (PL % TX == 0 || e % TX < ncol)) {
      const int f = f0 + e % TX;
      vv[q] = vt[(size_t(vt_fold<N>(e / TX)) * vt_half<N>() + vt_fold<N>(f / XS)) * XS + f % XS];
    }
  }
}

// body_conv_z_r with the tile's kernel values already in registers (usev) or
// evaluated per element (kp).
template <typename T, int N, int TX, int NT, int V = 0>
__device__ __forceinline__ void body_conv_z_r_v(cplx<T>* spec_p, int f0, const KernelParams& kp, cplx<T>* buf,
                                                const cplx<T>* tw, int tid, bool active, double* eslot,
                                                double* red, bool usev, const T (&vv)[conv_lv<T, N, TX, NT>()]) {
  using C = cplx<T>;
  constexpr int XS = r2c_xs<N>(), PL = N * XS, LV = conv_lv<T, N, TX, NT>(), E = N * TX;
  C* base = spec_p + f0;
  // columns of this tile inside the plane (fewer than TX in a ragged last
  // tile, whose other columns are transformed as zeros and not stored)
  const int ncol = PL - f0 < TX ? PL - f0 : TX;
  // forward z transforms, the first pass reading the tile from global memory
  fft_lines_load<T, N, TX, 1, TX, NT, -1, false, V>(buf, tw, tid, [=](int l, int p) {
    if (active && (PL % TX == 0 || l < ncol)) return base[size_t(p) * PL + l];
    C zr;
    zr.x = T(0);
    zr.y = T(0);
    return zr;
  });
  double es = 0.0;
#pragma unroll
  for (int q = 0; q < LV; ++q) {
    const int e = tid + q * NT;
    if (E % NT != 0 && e >= E) continue;
    if (PL % TX != 0 && e % TX >= ncol) continue;
    const int f = f0 + e % TX;
    const int kx = f % XS;
    const T v = usev ? vv[q] : kernel_value<T, N>(kp, kx, f / XS, e / TX);
    C c = buf[e];
    if (eslot) es += double((kx == 0 || kx == N / 2) ? 1 : 2) * double(v) * (double(c.x) * c.x + double(c.y) * c.y);
    c.x *= v;
    c.y *= v;
    buf[e] = c;
  }
  if (eslot) {
    for (int off = 32; off > 0; off >>= 1) es += __shfl_down(es, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = es;
  }
  __syncthreads();
  if (eslot && tid == 0) {
    double sx = 0.0;
    for (int w = 0; w < NT / 64; ++w) sx += red[w];
    eslot[0] = sx;
  }
  // inverse z transforms, the last pass storing the tile to global memory
  fft_lines_to<T, N, 0, TX, 1, TX, NT, +1, false, V>(buf, tw, tid, [=](int l, int p, C x) {
    if (active && (PL % TX == 0 || l < ncol)) base[size_t(p) * PL + l] = x;
  });
}

template <typename T, int N, int TX, int NT, int V = 0>
__device__ __forceinline__ void body_conv_z_r(cplx<T>* spec_p, int f0, const KernelParams& kp, cplx<T>* buf,
                                              const cplx<T>* tw, int tid, bool active = true,
                                              double* eslot = nullptr, double* red = nullptr,
                                              const T* __restrict__ vt = nullptr) {
  T vv[conv_lv<T, N, TX, NT>()];
  // the table loads are issued before the forward transform, so they overlap it
  if (vt) load_vtile<T, N, TX, NT>(vt, f0, tid, vv);
  body_conv_z_r_v<T, N, TX, NT, V>(spec_p, f0, kp, buf, tw, tid, active, eslot, red, vt != nullptr, vv);
}

// Half spectrum of plane z -> the real potential of the plane, left in buf as
// H complex lines, element x of line l at buf[InvLayout<T, N, V>::xq(l, x)]:
// line l holds row l in .x and row l + N/2 in .y.
// body_inv_xy_t: the same on a plane already staged in buf (and synchronized).
template <typename T, int N, int NT, int V = 0>
__device__ __forceinline__ void body_inv_xy_t(cplx<T>* buf, const cplx<T>* tw, int tid);

template <typename T, int N, int NT, int V = 0>
__device__ __forceinline__ void body_inv_xy_r(const cplx<T>* in, cplx<T>* buf, const cplx<T>* tw, int tid) {
  stage_in<cplx<T>, N * r2c_xs<N>(), NT>(buf, [&](int e) { return in[e]; }, tid);
  __syncthreads();
  body_inv_xy_t<T, N, NT, V>(buf, tw, tid);
}

// The x transforms of body_inv_xy_t (buf holds the y-transformed plane).
template <typename T, int N, int NT, int V>
__device__ __forceinline__ void inv_x_repacked(cplx<T>* buf, const cplx<T>* tw, int tid);

template <typename T, int N, int NT, int V>
__device__ __forceinline__ void body_inv_xy_t(cplx<T>* buf, const cplx<T>* tw, int tid) {
  using Lay = InvLayout<T, N, V>;
  constexpr int XS = r2c_xs<N>();
  fft_lines_ls<T, N, XS, 1, XS, NT, +1, false, V, true>(
      buf, tw, tid, [buf](int l, int p) { return buf[l + p * XS]; },
      [buf](int l, int p, cplx<T> x) { buf[l + Lay::ysig(p) * XS] = x; });
  inv_x_repacked<T, N, NT, V>(buf, tw, tid);
}

// The same from the half-spectrum plane in global memory: the first pass of
// the y transforms reads it directly (no staging copy).  Needs no barrier
// before it: the first pass reads before its barrier and writes after.
template <typename T, int N, int NT, int V = 0>
__device__ __forceinline__ void body_inv_xy_g(const cplx<T>* __restrict__ in, cplx<T>* buf, const cplx<T>* tw,
                                              int tid) {
  using Lay = InvLayout<T, N, V>;
  constexpr int XS = r2c_xs<N>();
  fft_lines_ls<T, N, XS, 1, XS, NT, +1, false, V, true>(
      buf, tw, tid, [in](int l, int p) { return in[p * XS + l]; },
      [buf](int l, int p, cplx<T> x) { buf[l + Lay::ysig(p) * XS] = x; });
  inv_x_repacked<T, N, NT, V>(buf, tw, tid);
}

template <typename T, int N, int NT, int V>
__device__ __forceinline__ void inv_x_repacked(cplx<T>* buf, const cplx<T>* tw, int tid) {
  using C = cplx<T>;
  constexpr int H = N / 2, XS = r2c_xs<N>();
  // The x transforms, whose first pass re-packs rows l and l + H into line
  // l on the way in: Z[k] = X1[k] + i X2[k] and Z[N-k] = conj X1[k] +
  // i conj X2[k] for k <= H (X1, X2 = rows l, l + H of the [y][kx] layout);
  // the zero and Nyquist bins of a real row are real, as a c2r transform
  // takes them.  This pass keeps consecutive butterflies of one line on
  // consecutive threads (with consecutive lines its re-pack spills registers
  // in FP64), with the radix order reversed: the larger first radix spreads
  // its writes over more banks.  The later passes take consecutive lines.
  using Lay = InvLayout<T, N, V>;
  fft_pass_l<T, N, 0, H, Lay::XL, 1, NT, +1, true, V ^ 1, Lay::WROT>(buf, tw, tid, [buf](int l, int p) {
    const bool lowk = p <= H;
    const int k = lowk ? p : N - p;
    C x1 = buf[Lay::ysig(l) * XS + k], x2 = buf[Lay::ysig(l + H) * XS + k];
    if (k == 0 || k == H) {
      x1.y = T(0);
      x2.y = T(0);
    }
    C z;
    if (lowk) {
      z.x = x1.x - x2.y;
      z.y = x1.y + x2.x;
    } else {
      z.x = x1.x + x2.y;
      z.y = x2.x - x1.y;
    }
    return z;
  });
  fft_lines_from<T, N, 1, H, Lay::XL, 1, NT, +1, false, V ^ 1>(buf, tw, tid);
}

// W_i -= v phi_j and (i != j) W_j -= v phi_i over plane z for one pair, with
// v from the packed lines of body_inv_xy_r; optional partial sum of v rho.
template <typename T, int N, int NT, bool EN>
__device__ __forceinline__ void accumulate_w_r(const T* __restrict__ pi_, const T* __restrict__ pj_, T* wi, T* wj,
                                               bool off, double* eslot, const cplx<T>* buf, double* red, int tid) {
  constexpr int HN = (N / 2) * N;
  T ea = T(0);
  if (wi) {
    // batches of U elements per thread: all global loads of a batch first
    constexpr int U = 3;
    constexpr int LP = (HN + NT - 1) / NT;
#pragma unroll
    for (int q0 = 0; q0 < LP; q0 += U) {
      T fi0[U], fj0[U], fi1[U], fj1[U], w0[U], w1[U], u0[U], u1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = tid + (q0 + u) * NT;
        if (q0 + u < LP && (HN % NT == 0 || e < HN)) {
          fi0[u] = pi_[e]; fj0[u] = pj_[e]; fi1[u] = pi_[e + HN]; fj1[u] = pj_[e + HN];
          w0[u] = wi[e]; w1[u] = wi[e + HN];
          if (off) { u0[u] = wj[e]; u1[u] = wj[e + HN]; }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = tid + (q0 + u) * NT;
        if (q0 + u < LP && (HN % NT == 0 || e < HN)) {
          const cplx<T> v = buf[xpos<N>(e)];
          wi[e] = w0[u] - v.x * fj0[u];
          wi[e + HN] = w1[u] - v.y * fj1[u];
          if (off) {
            wj[e] = u0[u] - v.x * fi0[u];
            wj[e + HN] = u1[u] - v.y * fi1[u];
          }
          if (EN) ea += v.x * fi0[u] * fj0[u] + v.y * fi1[u] * fj1[u];
        }
      }
    }
  } else if (EN) {
    for (int e = tid; e < HN; e += NT) {
      const cplx<T> v = buf[xpos<N>(e)];
      ea += v.x * pi_[e] * pj_[e] + v.y * pi_[e + HN] * pj_[e + HN];
    }
  }
  if (EN) {
    double x = ea;
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sx = 0;
      for (int w = 0; w < NT / 64; ++w) sx += red[w];
      eslot[0] = sx;
    }
  }
}


// W_k of plane z from all pairs containing orbital k (the owner of row k):
// W_k = -sum_j v_kj phi_j.  For each adjacency entry (pair slot p, partner j)
// the pair's half-spectrum plane is transformed back and v_kj phi_j is added
// to an accumulator in registers; the row is written once, never read.
template <typename T, int N, int NT, int V = 0>
__device__ __forceinline__ void body_inv_owner_r(const T* __restrict__ phi, const cplx<T>* __restrict__ spec,
                                                 const int32_t* __restrict__ adj, int a0, int a1, size_t zo,
                                                 T* __restrict__ wk, cplx<T>* buf, const cplx<T>* tw, int tid) {
  constexpr int XS = r2c_xs<N>(), HN = (N / 2) * N;
  constexpr size_t NG = size_t(N) * N * N, PL = size_t(N) * XS;
  constexpr int LP = (HN + NT - 1) / NT;
  T acc0[LP], acc1[LP];
#pragma unroll
  for (int q = 0; q < LP; ++q) { acc0[q] = T(0); acc1[q] = T(0); }
  const size_t zp = zo / (size_t(N) * N) * PL;  // plane offset in a pair's half spectrum
  for (int a = a0; a < a1; ++a) {
    // an opaque copy of the thread index keeps the transform's index
    // arithmetic inside the loop (hoisted, it would all stay live)
    int t = tid;
    asm volatile("" : "+v"(t));
    const int p = adj[2 * a], j = adj[2 * a + 1];
    // (the first pass's barrier also orders the previous entry's reads of buf
    // before this entry's writes)
    body_inv_xy_g<T, N, NT, V>(spec + size_t(p) * N * PL + zp, buf, tw, t);
    const T* fj = phi + size_t(j) * NG + zo;
    // partner row in batches of U elements per thread, loads first
    constexpr int U = 3;
#pragma unroll
    for (int q0 = 0; q0 < LP; q0 += U) {
      T f0[U], f1[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = t + (q0 + u) * NT;
        if (q0 + u < LP && (HN % NT == 0 || e < HN)) { f0[u] = fj[e]; f1[u] = fj[e + HN]; }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = t + (q0 + u) * NT;
        if (q0 + u < LP && (HN % NT == 0 || e < HN)) {
          const cplx<T> v = buf[xpos<N>(e)];
          acc0[q0 + u] += v.x * f0[u];
          acc1[q0 + u] += v.y * f1[u];
        }
      }
    }
  }
#pragma unroll
  for (int q = 0; q < LP; ++q) {
    const int e = tid + q * NT;
    if (HN % NT == 0 || e < HN) { wk[e] = -acc0[q]; wk[e + HN] = -acc1[q]; }
  }
}

}  // namespace ace
