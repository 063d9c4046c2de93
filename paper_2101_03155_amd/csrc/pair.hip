// Pair Poisson solves and W accumulation (step (c) of the ACE build).
//
// For every kept orbital pair (i, j) the exchange operator of Eq. (vx) needs
// v_ij = K * (phi_i phi_j), the periodic convolution of the pair density with
// the interaction kernel, computed in reciprocal space as in Eq. (e:vij):
// forward 3D FFT, multiplication by v(G), inverse 3D FFT.  The contribution
// -v_ij phi_j is added to W_i and, for i != j, -v_ij phi_i to W_j.
//
// Two real pair densities are packed into one complex field (real part pair
// a, imaginary part pair b).  Because v(G) is real and even in G, the product
// v(G) * FFT(rho_a + i rho_b) transforms back to v_a + i v_b exactly, so one
// complex 3D FFT pair serves two orbital pairs.
//
// Data layout: grids are [z][y][x] with x fastest; the spectrum of a pack is
// N^3 complex values in the same [z][y][x] order (in place through all
// passes).  A round of packs is conflict-free (no orbital appears twice), so
// the W read-modify-writes of one launch never collide: no atomics, and the
// result does not depend on scheduling.
//
// Two launch paths:
//  * fused: (product + x FFT + y FFT) per z-plane in one workgroup with the
//    plane in LDS; (z FFT, v(G), inverse z FFT) per x-tile column block;
//    (inverse y FFT + inverse x FFT + accumulate) per z-plane.  Three
//    HBM round trips of the spectrum per direction pair.
//  * split (planes larger than LDS): x, y and z passes as separate kernels.
#include <algorithm>

#include "ace_internal.h"
#include "fft.h"
#include "pair_phases.h"

namespace ace {


template <typename T, int N>
constexpr bool fused_fits_t() {
  return (size_t(N) * N + N) * sizeof(cplx<T>) + 1024 <= 163840;
}

// ------------------------------------------------------------ fused path

template <typename T, int N, int NT>
__global__ __launch_bounds__(NT) void k_fwd_xy(const T* __restrict__ phi, cplx<T>* __restrict__ spec,
                                               const Pack* __restrict__ packs,
                                               const cplx<T>* __restrict__ twg) {
  using C = cplx<T>;
  constexpr int P2 = N * N;
  constexpr size_t NG = size_t(N) * N * N;
  __shared__ C buf[P2];
  __shared__ C tw[N];
  const int tid = threadIdx.x, z = blockIdx.x, p = blockIdx.y;
  const Pack pk = packs[p];
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const size_t zo = size_t(z) * P2;
  const T* pia = phi + size_t(pk.ia) * NG + zo;
  const T* pja = phi + size_t(pk.ja) * NG + zo;
  if (pk.jb >= 0) {
    const T* pib = phi + size_t(pk.ib) * NG + zo;
    const T* pjb = phi + size_t(pk.jb) * NG + zo;
    for (int e = tid; e < P2; e += NT) {
      C v; v.x = pia[e] * pja[e]; v.y = pib[e] * pjb[e];
      buf[e] = v;
    }
  } else {
    for (int e = tid; e < P2; e += NT) {
      C v; v.x = pia[e] * pja[e]; v.y = T(0);
      buf[e] = v;
    }
  }
  __syncthreads();
  fft_lines<T, N, N, N, 1, NT, -1, true>(buf, tw, tid);   // x: rows
  fft_lines<T, N, N, 1, N, NT, -1, false>(buf, tw, tid);  // y: columns
  C* out = spec + size_t(p) * NG + zo;
  for (int e = tid; e < P2; e += NT) out[e] = buf[e];
}

template <typename T, int N, int NT, bool EN>
__global__ __launch_bounds__(NT) void k_inv_xy(const T* __restrict__ phi, const cplx<T>* __restrict__ spec,
                                               const Pack* __restrict__ packs, T* __restrict__ W,
                                               double* __restrict__ epart,
                                               const cplx<T>* __restrict__ twg) {
  using C = cplx<T>;
  constexpr int P2 = N * N;
  constexpr size_t NG = size_t(N) * N * N;
  __shared__ C buf[P2];
  __shared__ C tw[N];
  __shared__ double red[2 * (NT / 64)];
  const int tid = threadIdx.x, z = blockIdx.x, p = blockIdx.y;
  const Pack pk = packs[p];
  for (int i = tid; i < N; i += NT) tw[i] = twg[i];
  const size_t zo = size_t(z) * P2;
  const C* in = spec + size_t(p) * NG + zo;
  for (int e = tid; e < P2; e += NT) buf[e] = in[e];
  __syncthreads();
  fft_lines<T, N, N, 1, N, NT, +1, false>(buf, tw, tid);  // y
  fft_lines<T, N, N, N, 1, NT, +1, true>(buf, tw, tid);   // x
  accumulate_w<T, NT, EN>(phi, pk, NG, zo, P2, W, EN ? epart + 2 * (size_t(p) * N + z) : nullptr, buf, red, tid);
}

// ------------------------------------------------------------ z pass (both paths)

template <typename T, int N, int TX, int NT>
__global__ __launch_bounds__(NT) void k_conv_z(cplx<T>* __restrict__ spec, const cplx<T>* __restrict__ twg,
                                               KernelParams kp) {
  __shared__ cplx<T> buf[N * TX];
  __shared__ cplx<T> tw[N];
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  body_conv_z<T, N, TX, NT>(spec + size_t(blockIdx.z) * N * N * N, blockIdx.x * TX, blockIdx.y, kp, buf, tw,
                            threadIdx.x);
}

// ------------------------------------------------------------ split path

template <typename T, int N, int ROWS, int NT>
__global__ __launch_bounds__(NT) void k_fwd_x(const T* __restrict__ phi, cplx<T>* __restrict__ spec,
                                              const Pack* __restrict__ packs,
                                              const cplx<T>* __restrict__ twg) {
  __shared__ cplx<T> buf[ROWS * N];
  __shared__ cplx<T> tw[N];
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  const int p = blockIdx.y;
  body_fwd_x<T, N, ROWS, NT>(phi, spec + size_t(p) * N * N * N, packs[p], size_t(blockIdx.x) * ROWS * N, buf, tw,
                             threadIdx.x);
}

template <typename T, int N, int TX, int NT, int S>
__global__ __launch_bounds__(NT) void k_line_y(cplx<T>* __restrict__ spec, const cplx<T>* __restrict__ twg) {
  __shared__ cplx<T> buf[N * TX];
  __shared__ cplx<T> tw[N];
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  body_line_y<T, N, TX, NT, S>(spec + size_t(blockIdx.z) * N * N * N, blockIdx.x * TX, blockIdx.y, buf, tw,
                               threadIdx.x);
}

template <typename T, int N, int ROWS, int NT, bool EN>
__global__ __launch_bounds__(NT) void k_inv_x(const T* __restrict__ phi, const cplx<T>* __restrict__ spec,
                                              const Pack* __restrict__ packs, T* __restrict__ W,
                                              double* __restrict__ epart,
                                              const cplx<T>* __restrict__ twg) {
  __shared__ cplx<T> buf[ROWS * N];
  __shared__ cplx<T> tw[N];
  __shared__ double red[2 * (NT / 64)];
  for (int i = threadIdx.x; i < N; i += NT) tw[i] = twg[i];
  const int p = blockIdx.y;
  body_inv_x<T, N, ROWS, NT, EN>(phi, spec + size_t(p) * N * N * N, packs[p], size_t(blockIdx.x) * ROWS * N, W,
                                 epart ? epart + 2 * (size_t(p) * gridDim.x + blockIdx.x) : nullptr, buf, tw, red,
                                 threadIdx.x);
}


// ------------------------------------------------------------ real-to-complex path
// One pair per workgroup: blockIdx.y = 2 * pack + (0: pair a, 1: pair b); the
// spectrum of slot y is N * N * XS complex values at spec + y * N * N * XS.

template <typename T, int N>
constexpr bool r2c_fits_t() {
  return (size_t(N) * r2c_xs<N>() + N) * sizeof(cplx<T>) + 1024 <= 163840;
}

// ZFAST: blockIdx.x = z-plane, blockIdx.y = pair slot; otherwise the slot
// runs fastest, so the workgroups in flight share a few z-planes and the
// phi rows of those planes stay in the caches (dealing the planes to the
// XCDs, as the owner pass does, measured no faster here: the pass is bound
// by its spectrum writes).
template <typename T, int N, int NT, bool ZFAST = true>
__global__ __launch_bounds__(NT) void k_fwd_xy_r(const T* __restrict__ phi, cplx<T>* __restrict__ spec,
                                                 const Pack* __restrict__ packs,
                                                 const cplx<T>* __restrict__ twg) {
  using C = cplx<T>;
  constexpr int XS = r2c_xs<N>();
  constexpr size_t NG = size_t(N) * N * N, PL = size_t(N) * XS;
  __shared__ C buf[N * XS];
  __shared__ C tw[N];
  const int tid = threadIdx.x;
  const int z = ZFAST ? blockIdx.x : blockIdx.y, slot = ZFAST ? blockIdx.y : blockIdx.x;
  const Pack pk = packs[slot >> 1];
  const int i = (slot & 1) ? pk.ib : pk.ia, j = (slot & 1) ? pk.jb : pk.ja;
  if (j < 0) return;
  for (int t = tid; t < N; t += NT) tw[t] = twg[t];
  const size_t zo = size_t(z) * N * N;
  body_fwd_xy_r<T, N, NT>(phi + size_t(i) * NG + zo, phi + size_t(j) * NG + zo,
                          spec + size_t(slot) * N * PL + size_t(z) * PL, buf, tw, tid);
}

// epart != nullptr: per-tile partial sums of sum_r rho v for the pair
// energies, epart[2 * (pack * ntile + tile) + (slot & 1)].  SPW slots per
// workgroup (blockIdx.y = slot group): the tile's slice of the v(G) table is
// then fetched from memory once and re-read from L2 for the other slots.
template <typename T, int N, int TX, int NT, int SPW = 1>
__global__ __launch_bounds__(NT) void k_conv_z_r(cplx<T>* __restrict__ spec, const Pack* __restrict__ packs,
                                                 int nslots, const cplx<T>* __restrict__ twg, KernelParams kp,
                                                 double* __restrict__ epart, const T* __restrict__ vt) {
  constexpr size_t PL = size_t(N) * r2c_xs<N>();
  __shared__ cplx<T> buf[N * TX];
  __shared__ cplx<T> tw[N];
  __shared__ double red[NT / 64];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = twg[t];
  // the tile's kernel values serve every slot of the workgroup
  T vv[conv_lv<T, N, TX, NT>()];
  if (vt) load_vtile<T, N, TX, NT>(vt, blockIdx.x * TX, threadIdx.x, vv);
  for (int q = 0; q < SPW; ++q) {
    const int slot = blockIdx.y * SPW + q;
    if (slot >= nslots) break;
    if ((slot & 1) && packs[slot >> 1].jb < 0) continue;
    double* es = epart ? epart + 2 * (size_t(slot >> 1) * gridDim.x + blockIdx.x) + (slot & 1) : nullptr;
    // (each body's first barrier orders the previous body's reads of buf,
    // tw and red before its writes)
    body_conv_z_r_v<T, N, TX, NT>(spec + size_t(slot) * N * PL, blockIdx.x * TX, kp, buf, tw, threadIdx.x, true, es,
                                  red, vt != nullptr, vv);
  }
}

// Owner-computes W: one workgroup per (z-plane, orbital k), walking the
// adjacency entries adj_ptr[k] .. adj_ptr[k + 1] of (pair slot, partner).
// Without XCD: blockIdx.x = z-plane, blockIdx.y = orbital k (measured faster
// than the orbital-fastest order over the whole device).  With XCD (N a
// multiple of 8, one-dimensional grid of N * norb): workgroups are dealt to
// the eight XCDs in turn, so XCD x is given the planes z = x mod 8 with the
// orbital fastest; the owners in flight on an XCD then share the partner
// planes and spectra they read in that XCD's L2 (3-6% faster at 32 waters).
template <typename T, int N, int NT, bool XCD = false>
__global__ __launch_bounds__(NT, 4) void k_inv_owner_r(const T* __restrict__ phi, const cplx<T>* __restrict__ spec,
                                                    const int32_t* __restrict__ adj_ptr,
                                                    const int32_t* __restrict__ adj,
                                                    const int32_t* __restrict__ operm, T* __restrict__ W,
                                                    const cplx<T>* __restrict__ twg) {
  constexpr size_t NG = size_t(N) * N * N;
  __shared__ cplx<T> buf[N * r2c_xs<N>()];
  __shared__ cplx<T> tw[N];
  int z, k;
  if (!XCD) {
    z = blockIdx.x;
    k = blockIdx.y;
  } else {
    const int i = blockIdx.x, l = i >> 3;
    const int norb = int(gridDim.x) / N;
    z = (l / norb) * 8 + (i & 7);
    k = l % norb;
  }
  if (operm) k = operm[k];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = twg[t];
  const size_t zo = size_t(z) * N * N;
  body_inv_owner_r<T, N, NT>(phi, spec, adj, adj_ptr[k], adj_ptr[k + 1], zo,
                                                W + size_t(k) * NG + zo, buf, tw, threadIdx.x);
}

template <typename T, int N, int NT, bool EN>
__global__ __launch_bounds__(NT) void k_inv_xy_r(const T* __restrict__ phi, const cplx<T>* __restrict__ spec,
                                                 const Pack* __restrict__ packs, T* __restrict__ W,
                                                 double* __restrict__ epart,
                                                 const cplx<T>* __restrict__ twg) {
  using C = cplx<T>;
  constexpr int XS = r2c_xs<N>();
  constexpr size_t NG = size_t(N) * N * N, PL = size_t(N) * XS;
  __shared__ C buf[N * XS];
  __shared__ C tw[N];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x, z = blockIdx.x, slot = blockIdx.y;
  const Pack pk = packs[slot >> 1];
  const int i = (slot & 1) ? pk.ib : pk.ia, j = (slot & 1) ? pk.jb : pk.ja;
  if (j < 0) return;
  for (int t = tid; t < N; t += NT) tw[t] = twg[t];
  body_inv_xy_r<T, N, NT>(spec + size_t(slot) * N * PL + size_t(z) * PL, buf, tw, tid);
  const size_t zo = size_t(z) * N * N;
  T* wi = W ? W + size_t(i) * NG + zo : nullptr;
  T* wj = W ? W + size_t(j) * NG + zo : nullptr;
  accumulate_w_r<T, N, NT, EN>(phi + size_t(i) * NG + zo, phi + size_t(j) * NG + zo, wi, wj, i != j,
                               EN ? epart + 2 * (size_t(slot >> 1) * N + z) + (slot & 1) : nullptr, buf, red, tid);
}

// ------------------------------------------------------------ dispatch

template <typename T, int N>
static hipError_t pair_round_t(const PairShape& sh, const void* phi_, void* spec_, const Pack* packs,
                               int npacks, int npairs, void* W_, double* epart, const void* tw_,
                               const KernelParams& kp, hipStream_t s, EventRecorder* rec) {
  using C = cplx<T>;
  const T* phi = static_cast<const T*>(phi_);
  T* W = static_cast<T*>(W_);
  C* spec = static_cast<C*>(spec_);
  const C* tw = static_cast<const C*>(tw_);
  constexpr int TX = pick_tx(N);
  constexpr int NTL = 256;
  if (npacks <= 0) return hipSuccess;
  // algorithmic HBM bytes per orbital pair, in units of N^3 * sizeof(T):
  // read phi_i, phi_j (2) + spectrum write (1) | spectrum read + write (2) |
  // spectrum read (1) + phi re-read (2) + W_i, W_j read-modify-write (4)
  const double u = double(npairs) * double(N) * N * N * sizeof(T);
  if constexpr (r2c_fits_t<T, N>()) {
    if (sh.fused_xy == 2) {
      constexpr int NTR = 512;
      constexpr int TXR = r2c_tx<N>();
      rec_begin(rec, KC_FWD_XY, s);
      hipLaunchKernelGGL((k_fwd_xy_r<T, N, NTR>), dim3(N, 2 * npacks), dim3(NTR), 0, s, phi, spec, packs, tw);
      rec_end(rec, KC_FWD_XY, s, 3 * u);
      rec_begin(rec, KC_CONV_Z, s);
      hipLaunchKernelGGL((k_conv_z_r<T, N, TXR, NTL>), dim3(N * r2c_xs<N>() / TXR, 2 * npacks), dim3(NTL), 0, s, spec,
                         packs, 2 * npacks, tw, kp, nullptr, static_cast<const T*>(nullptr));
      rec_end(rec, KC_CONV_Z, s, 2 * u);
      rec_begin(rec, KC_INV_XY, s);
      if (epart)
        hipLaunchKernelGGL((k_inv_xy_r<T, N, NTR, true>), dim3(N, 2 * npacks), dim3(NTR), 0, s, phi, spec, packs, W,
                           epart, tw);
      else
        hipLaunchKernelGGL((k_inv_xy_r<T, N, NTR, false>), dim3(N, 2 * npacks), dim3(NTR), 0, s, phi, spec, packs, W,
                           epart, tw);
      rec_end(rec, KC_INV_XY, s, 7 * u);
      return hipGetLastError();
    }
  }
  if constexpr (fused_fits_t<T, N>()) {
    if (sh.fused_xy) {
      constexpr int NTP = 512;
      rec_begin(rec, KC_FWD_XY, s);
      hipLaunchKernelGGL((k_fwd_xy<T, N, NTP>), dim3(N, npacks), dim3(NTP), 0, s, phi, spec, packs, tw);
      rec_end(rec, KC_FWD_XY, s, 3 * u);
      rec_begin(rec, KC_CONV_Z, s);
      hipLaunchKernelGGL((k_conv_z<T, N, TX, NTL>), dim3(N / TX, N, npacks), dim3(NTL), 0, s, spec, tw, kp);
      rec_end(rec, KC_CONV_Z, s, 2 * u);
      rec_begin(rec, KC_INV_XY, s);
      if (epart)
        hipLaunchKernelGGL((k_inv_xy<T, N, NTP, true>), dim3(N, npacks), dim3(NTP), 0, s, phi, spec, packs, W, epart, tw);
      else
        hipLaunchKernelGGL((k_inv_xy<T, N, NTP, false>), dim3(N, npacks), dim3(NTP), 0, s, phi, spec, packs, W, epart, tw);
      rec_end(rec, KC_INV_XY, s, 7 * u);
      return hipGetLastError();
    }
  }
  constexpr int ROWS = pick_rows(N);
  const int nrb = N * N / ROWS;
  rec_begin(rec, KC_FWD_X, s);
  hipLaunchKernelGGL((k_fwd_x<T, N, ROWS, NTL>), dim3(nrb, npacks), dim3(NTL), 0, s, phi, spec, packs, tw);
  rec_end(rec, KC_FWD_X, s, 3 * u);
  rec_begin(rec, KC_FWD_Y, s);
  hipLaunchKernelGGL((k_line_y<T, N, TX, NTL, -1>), dim3(N / TX, N, npacks), dim3(NTL), 0, s, spec, tw);
  rec_end(rec, KC_FWD_Y, s, 2 * u);
  rec_begin(rec, KC_CONV_Z, s);
  hipLaunchKernelGGL((k_conv_z<T, N, TX, NTL>), dim3(N / TX, N, npacks), dim3(NTL), 0, s, spec, tw, kp);
  rec_end(rec, KC_CONV_Z, s, 2 * u);
  rec_begin(rec, KC_INV_Y, s);
  hipLaunchKernelGGL((k_line_y<T, N, TX, NTL, +1>), dim3(N / TX, N, npacks), dim3(NTL), 0, s, spec, tw);
  rec_end(rec, KC_INV_Y, s, 2 * u);
  rec_begin(rec, KC_INV_X, s);
  if (epart)
    hipLaunchKernelGGL((k_inv_x<T, N, ROWS, NTL, true>), dim3(nrb, npacks), dim3(NTL), 0, s, phi, spec, packs, W, epart, tw);
  else
    hipLaunchKernelGGL((k_inv_x<T, N, ROWS, NTL, false>), dim3(nrb, npacks), dim3(NTL), 0, s, phi, spec, packs, W, epart, tw);
  rec_end(rec, KC_INV_X, s, 7 * u);
  return hipGetLastError();
}

// ------------------------------------------------------------ owner-computes W
// All pairs are transformed forward (packs of consecutive pairs, no conflict
// constraints: only phi is read) and convolved, with every pair's half
// spectrum kept in HBM; then one workgroup per (z-plane, orbital k) forms W_k
// from k's adjacency list and writes it once.  Algorithmic bytes per pair:
// forward 3, z pass 2 (N^3 s units, as for the other paths); the owner pass
// reads each adjacency entry's spectrum plane and partner row (2 per
// off-diagonal pair, 1 per diagonal one) and writes each W row once.
template <typename T, int N>
static hipError_t pair_owner_t(const void* phi_, void* spec_, const Pack* packs, int npacks, int npairs,
                               const int32_t* adj_ptr, const int32_t* adj, const int32_t* operm, int norb,
                               int64_t nadj, void* W_,
                               double* epart, const void* tw_, const KernelParams& kp, const void* vt_, int chunk,
                               hipStream_t s, EventRecorder* rec) {
  if constexpr (!r2c_fits_t<T, N>()) {
    return hipErrorInvalidValue;
  } else {
    using C = cplx<T>;
    const T* phi = static_cast<const T*>(phi_);
    T* W = static_cast<T*>(W_);
    C* spec = static_cast<C*>(spec_);
    const C* tw = static_cast<const C*>(tw_);
    // planes too large for two workgroups per CU take 1024 threads, so that
    // one workgroup still runs four waves per SIMD
    constexpr int NTR = size_t(N) * r2c_xs<N>() * sizeof(C) > 81920 ? 1024 : 512;
    constexpr int NTL = 256, TXR = own_tx<T, N>();
    constexpr int NTILE = own_ntile<T, N>();
    constexpr size_t SLOT = size_t(N) * N * r2c_xs<N>();  // complex values per pair slot
    const double u3 = double(N) * N * N * sizeof(T);
    // forward and z pass in launches of at most `chunk` packs (grid y = 2 *
    // packs <= 65534); one launch each over all pairs measured fastest
    const int CH = chunk < 1 ? 1 : (chunk > 32767 ? 32767 : chunk);
    for (int c0 = 0; c0 < npacks; c0 += CH) {
      const int nc = (npacks - c0 < CH) ? npacks - c0 : CH;
      const int pc = (2 * c0 + 2 * nc <= npairs) ? 2 * nc : npairs - 2 * c0;  // pairs in this chunk
      rec_begin(rec, KC_FWD_XY, s);
      hipLaunchKernelGGL((k_fwd_xy_r<T, N, NTR, false>), dim3(2 * nc, N), dim3(NTR), 0, s, phi,
                         spec + 2 * size_t(c0) * SLOT, packs + c0, tw);
      rec_end(rec, KC_FWD_XY, s, 3 * u3 * pc);
      rec_begin(rec, KC_CONV_Z, s);
      // FP64: four slots per workgroup share the table slice (z pass 5% faster
      // at 32 waters); FP32 (half the table) measured faster with one
      if (sizeof(T) == 8)
        hipLaunchKernelGGL((k_conv_z_r<T, N, TXR, NTL, 4>), dim3(NTILE, (2 * nc + 3) / 4), dim3(NTL), 0, s,
                           spec + 2 * size_t(c0) * SLOT, packs + c0, 2 * nc, tw, kp,
                           epart ? epart + 2 * size_t(c0) * NTILE : nullptr, static_cast<const T*>(vt_));
      else
        hipLaunchKernelGGL((k_conv_z_r<T, N, TXR, NTL>), dim3(NTILE, 2 * nc), dim3(NTL), 0, s,
                           spec + 2 * size_t(c0) * SLOT, packs + c0, 2 * nc, tw, kp,
                           epart ? epart + 2 * size_t(c0) * NTILE : nullptr, static_cast<const T*>(vt_));
      rec_end(rec, KC_CONV_Z, s, 2 * u3 * pc);
    }
    if (W) {
      rec_begin(rec, KC_INV_XY, s);
      if (N % 8 == 0)
        hipLaunchKernelGGL((k_inv_owner_r<T, N, NTR, true>), dim3(N * norb), dim3(NTR), 0, s, phi, spec, adj_ptr, adj,
                           operm, W, tw);
      else
        hipLaunchKernelGGL((k_inv_owner_r<T, N, NTR>), dim3(N, norb), dim3(NTR), 0, s, phi, spec, adj_ptr, adj, operm,
                           W, tw);
      rec_end(rec, KC_INV_XY, s, double(nadj) * (2.0 * SLOT * sizeof(T) + u3) + double(norb) * u3);
    }
    return hipGetLastError();
  }
}

#define ACE_PAIR_SIZES(X) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(80) X(96) X(100) X(108) X(120) X(160)

bool pair_supported(int N) {
  switch (N) {
#define X(n) case n: return true;
    ACE_PAIR_SIZES(X)
#undef X
    default: return false;
  }
}

hipError_t pair_owner(int prec, int N, const void* phi, void* spec, const Pack* packs, int npacks, int npairs,
                      const int32_t* adj_ptr, const int32_t* adj, const int32_t* operm, int norb, int64_t nadj,
                      void* W, double* epart, const void* tw, const KernelParams& kp, const void* vt, int chunk,
                      hipStream_t s, EventRecorder* rec) {
  switch (N) {
#define X(n)                                                                                                       \
  case n:                                                                                                          \
    return prec == 0 ? pair_owner_t<double, n>(phi, spec, packs, npacks, npairs, adj_ptr, adj, operm, norb, nadj, \
                                               W, epart, tw, kp, vt, chunk, s, rec)                                \
                     : pair_owner_t<float, n>(phi, spec, packs, npacks, npairs, adj_ptr, adj, operm, norb, nadj, W, \
                                              epart, tw, kp, vt, chunk, s, rec);
    ACE_PAIR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// v(G) of the half spectrum, [z][y][kx], in the pair-stage precision: the
// same values the z pass would evaluate per element (kernel_value).
template <typename T, int N>
__global__ void k_vtable(KernelParams kp, T* __restrict__ vt) {
  constexpr int XS = r2c_xs<N>(), H = vt_half<N>();
  constexpr int64_t TOT = int64_t(H) * H * XS;
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < TOT; e += int64_t(gridDim.x) * blockDim.x) {
    const int kx = int(e % XS), y = int((e / XS) % H), z = int(e / (int64_t(XS) * H));
    vt[e] = kernel_value<T, N>(kp, kx, y, z);
  }
}

hipError_t launch_vtable(int prec, int N, const KernelParams& kp, void* vt, hipStream_t s) {
  const int64_t tot = int64_t(N / 2 + 1) * (N / 2 + 1) * (N / 2 + 1);
  const unsigned g = unsigned(std::min<int64_t>((tot + 255) / 256, 2048));
  switch (N) {
#define X(n)                                                                                                   \
  case n:                                                                                                      \
    if (prec == 0)                                                                                             \
      hipLaunchKernelGGL((k_vtable<double, n>), dim3(g), dim3(256), 0, s, kp, static_cast<double*>(vt));       \
    else                                                                                                       \
      hipLaunchKernelGGL((k_vtable<float, n>), dim3(g), dim3(256), 0, s, kp, static_cast<float*>(vt));         \
    return hipGetLastError();
    ACE_PAIR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

int pair_owner_ntile(int prec, int N) {
  switch (N) {
#define X(n) case n: return prec == 0 ? own_ntile<double, n>() : own_ntile<float, n>();
    ACE_PAIR_SIZES(X)
#undef X
    default:
      return 0;
  }
}

bool pair_r2c_fits(int prec, int N) {
  switch (N) {
#define X(n) case n: return prec == 0 ? r2c_fits_t<double, n>() : r2c_fits_t<float, n>();
    ACE_PAIR_SIZES(X)
#undef X
    default: return false;
  }
}

// Complex spectrum elements per pack (two pairs) for a launch shape.
size_t pair_spec_elems(int prec, int N, const PairShape& sh) {
  if (sh.fused_xy >= 2 && pair_r2c_fits(prec, N)) return 2 * size_t(N) * N * (N / 2 + 1);
  return size_t(N) * N * N;
}

bool pair_fused_fits(int prec, int N) {
  switch (N) {
#define X(n) case n: return prec == 0 ? fused_fits_t<double, n>() : fused_fits_t<float, n>();
    ACE_PAIR_SIZES(X)
#undef X
    default: return false;
  }
}

// The owner-computes path (real-to-complex transforms) is the default wherever
// its half-spectrum plane fits in LDS: measured faster than the split passes
// even at one workgroup per CU (120^3 FP64, 160^3 FP32).
PairShape pair_default_shape(int prec, int N) {
  PairShape sh;
  sh.fused_xy = pair_r2c_fits(prec, N) ? 3 : 0;
  sh.nt_xy = 512;
  sh.tx = pick_tx(N);
  return sh;
}

int pair_energy_blocks(int N, const PairShape& sh) {
  if (sh.fused_xy) return N;
  return N * N / pick_rows(N);
}

hipError_t pair_round(int prec, int N, const PairShape& sh, const void* phi, void* spec,
                      const Pack* packs, int npacks, int npairs, void* W, double* epart, const void* tw,
                      const KernelParams& kp, hipStream_t s, EventRecorder* rec) {
  PairShape use = sh;
  if (use.fused_xy == 3) use.fused_xy = 2;  // owner path over budget: real-to-complex rounds
  if ((use.fused_xy == 1 && !pair_fused_fits(prec, N)) || (use.fused_xy == 2 && !pair_r2c_fits(prec, N)))
    use.fused_xy = 0;
  switch (N) {
#define X(n)                                                                                          \
  case n:                                                                                             \
    return prec == 0 ? pair_round_t<double, n>(use, phi, spec, packs, npacks, npairs, W, epart, tw, kp, s, rec) \
                     : pair_round_t<float, n>(use, phi, spec, packs, npacks, npairs, W, epart, tw, kp, s, rec);
    ACE_PAIR_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace ace
