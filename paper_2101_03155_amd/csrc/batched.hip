// Batched pair stage: the pair Poisson solves of many independent systems of
// uneven size (grids 16^3 .. 96^3, different orbital counts, pair lists and
// interaction kernels) sharing launches.
//
// The pair list of every system is split into conflict-free rounds (as for a
// single build); super-round r gathers round r of every system, and a
// segment is the part of a super-round whose systems share one grid size N.
// The five passes of the split path (x forward with the pair product,
// y forward, z forward + v(G) + z inverse, y inverse, x inverse with the W
// update) are "phases"; a work item is one workgroup's share of one phase of
// one pack, and the items of a segment cover packs of different systems,
// kernels and pair-list lengths.  Kernels are specialized per N (mixing sizes
// in one kernel would size its registers for the largest case).
//
// Two launch forms:
//  * one launch per (segment, phase), captured with everything else of the
//    batched build in a hipGraph;
//  * one cooperative (persistent) launch per grid size that walks all its
//    segments and phases with a grid-wide barrier after each phase, so the
//    data a phase reads was completely written by the previous one.
#include <hip/hip_cooperative_groups.h>

#include "ace_internal.h"
#include "fft.h"
#include "pair_phases.h"

namespace ace {

namespace cg = cooperative_groups;

constexpr int BNT = 256;

template <int TXV>
__host__ __device__ constexpr int btx(int n) { return pick_tx(n) < TXV ? pick_tx(n) : TXV; }

__host__ __device__ inline int64_t batched_items(int n, int phase, int txv) {
  const int rows = pick_rows(n);
  const int tx = txv == 8 ? btx<8>(n) : btx<16>(n);
  return (phase == 0 || phase == 4) ? int64_t(n) * n / rows : int64_t(n / tx) * n;
}

template <typename T, int N, int TXV, int V>
__device__ __forceinline__ void run_phase(int p, int64_t b, const BSys& sy, const BPack& bp, cplx<T>* buf,
                                          const cplx<T>* tw, double* red, int tid) {
  constexpr int TX = btx<TXV>(N);
  constexpr int ROWS = pick_rows(N);
  constexpr int NXT = N / TX;
  cplx<T>* spec = static_cast<cplx<T>*>(bp.spec);
  const T* phi = static_cast<const T*>(sy.phi);
  if (p == 0) {
    body_fwd_x<T, N, ROWS, BNT, V>(phi, spec, bp.pk, size_t(b) * ROWS * N, buf, tw, tid);
  } else if (p == 1) {
    body_line_y<T, N, TX, BNT, -1, V>(spec, int(b % NXT) * TX, int(b / NXT), buf, tw, tid);
  } else if (p == 2) {
    KernelParams kp;
    kp.kind = sy.kind;
    kp.omega = sy.omega;
    kp.inv_ng = sy.inv_ng;
    kp.g[0] = sy.g[0]; kp.g[1] = sy.g[1]; kp.g[2] = sy.g[2];
    body_conv_z<T, N, TX, BNT, V>(spec, int(b % NXT) * TX, int(b / NXT), kp, buf, tw, tid);
  } else if (p == 3) {
    body_line_y<T, N, TX, BNT, +1, V>(spec, int(b % NXT) * TX, int(b / NXT), buf, tw, tid);
  } else {
    body_inv_x<T, N, ROWS, BNT, false, V>(phi, spec, bp.pk, size_t(b) * ROWS * N, static_cast<T*>(sy.W), nullptr,
                                          buf, tw, red, tid);
  }
}

// Item j of phase p of segment sg (all packs of one grid size N).
template <typename T, int N, int TXV, int V>
__device__ __forceinline__ void run_item(int p, int64_t j, const BRound& sg, const BSys* __restrict__ sys,
                                         const BPack* __restrict__ packs, const int64_t* __restrict__ starts,
                                         cplx<T>* buf, cplx<T>* tw, double* red) {
  const int tid = threadIdx.x;
  // pack q with starts[q] <= j < starts[q + 1]
  const int64_t* st = starts + sg.start_off[p];
  int lo = 0, hi = sg.npacks;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] <= j) lo = mid; else hi = mid;
  }
  const BPack bp = packs[sg.pack0 + lo];
  const BSys& sy = sys[bp.sys];
  const int64_t b = j - st[lo];
  const cplx<T>* twg = static_cast<const cplx<T>*>(sy.tw);
  __syncthreads();  // the previous item's last reads of buf/tw are done
  for (int i = tid; i < N; i += BNT) tw[i] = twg[i];
  run_phase<T, N, TXV, V>(p, b, sy, bp, buf, tw, red, tid);
}

template <typename T, int N, int TXV, int V>
__global__ __launch_bounds__(BNT) void k_batched_phase(int p, BRound sg, const BSys* __restrict__ sys,
                                                       const BPack* __restrict__ packs,
                                                       const int64_t* __restrict__ starts) {
  constexpr int E = (N * btx<TXV>(N) > pick_rows(N) * N) ? N * btx<TXV>(N) : pick_rows(N) * N;
  __shared__ cplx<T> buf[E];
  __shared__ cplx<T> tw[N];
  __shared__ double red[2 * (BNT / 64)];
  for (int64_t j = blockIdx.x; j < sg.nitems[p]; j += gridDim.x)
    run_item<T, N, TXV, V>(p, j, sg, sys, packs, starts, buf, tw, red);
}

// One launch for every segment of one grid size: all super-rounds, all five
// phases, a grid-wide barrier after each phase.
template <typename T, int N, int TXV, int V>
__global__ __launch_bounds__(BNT) void k_batched_persistent(int nseg, const BRound* __restrict__ segs,
                                                            const BSys* __restrict__ sys,
                                                            const BPack* __restrict__ packs,
                                                            const int64_t* __restrict__ starts) {
  constexpr int E = (N * btx<TXV>(N) > pick_rows(N) * N) ? N * btx<TXV>(N) : pick_rows(N) * N;
  __shared__ cplx<T> buf[E];
  __shared__ cplx<T> tw[N];
  __shared__ double red[2 * (BNT / 64)];
  cg::grid_group grid = cg::this_grid();
  for (int r = 0; r < nseg; ++r) {
    const BRound sg = segs[r];
    for (int p = 0; p < 5; ++p) {
      for (int64_t j = blockIdx.x; j < sg.nitems[p]; j += gridDim.x)
        run_item<T, N, TXV, V>(p, j, sg, sys, packs, starts, buf, tw, red);
      grid.sync();
    }
  }
}

// ------------------------------------------------------------ real-to-complex layout
// Three phases per segment: (0) product + x and y transforms per (pair,
// z-plane), (1) z lines + v(G) over tiles of flattened half-spectrum columns,
// (2) inverse y and x transforms + W update per (pair, z-plane).  A pack has
// one or two pair slots, each with its own N * N * (N/2 + 1) half spectrum.
constexpr int BNTR = 512;

// LDS buffer of the three phases: the in-plane bodies use N * XS values, the
// z pass two tiles of N * TX (TX can exceed XS on small grids, e.g. 16 > 9 at
// N = 16).
template <int N>
__host__ __device__ constexpr int r2c_buf_elems() {
  return 2 * N * r2c_tx<N>() > N * r2c_xs<N>() ? 2 * N * r2c_tx<N>() : N * r2c_xs<N>();
}

// Items per pair slot: one per z-plane in phases 0 and 2; in phase 1 one per
// tpi z-pass tiles: 1 for the per-phase launches (256-thread workgroups), 2
// in the persistent launch (each half of a 512-thread workgroup transforms one
// tile).
template <int N>
__host__ __device__ constexpr int64_t r2c_slot_items(int phase, int tpi) {
  return phase == 1 ? (int64_t(N) * r2c_xs<N>() / r2c_tx<N>() + tpi - 1) / tpi : int64_t(N);
}

// Item j of phase p, which belongs to pack q of the segment (the caller has
// located q).  tw holds the twiddles of system *tw_sys (-1: none yet).
template <typename T, int N, int V, int NT>
__device__ __forceinline__ void run_item_r(int p, int64_t j, int q, const BRound& sg, const BSys* __restrict__ sys,
                                           const BPack* __restrict__ packs, const int64_t* __restrict__ st,
                                           cplx<T>* buf, cplx<T>* tw, int& tw_sys, double* red) {
  constexpr int XS = r2c_xs<N>();
  constexpr size_t NG = size_t(N) * N * N, PL = size_t(N) * XS;
  // an opaque copy of the thread index: keeps the per-thread index arithmetic
  // of the three phase bodies inside this item instead of hoisted out of the
  // item loop (where it would all stay live at once)
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const BPack bp = packs[sg.pack0 + q];
  const BSys& sy = sys[bp.sys];
  const int64_t b = j - st[q];
  constexpr int TPI = NT == BNTR ? 2 : 1;
  const int64_t per = r2c_slot_items<N>(p, TPI);
  const int slot = int(b / per);
  const int sub = int(b % per);
  const int oi = slot ? bp.pk.ib : bp.pk.ia, oj = slot ? bp.pk.jb : bp.pk.ja;
  cplx<T>* spec = static_cast<cplx<T>*>(bp.spec) + size_t(slot) * N * PL;
  const T* phi = static_cast<const T*>(sy.phi);
  __syncthreads();  // the previous item's last reads of buf/tw are done
  if (bp.sys != tw_sys) {
    const cplx<T>* twg = static_cast<const cplx<T>*>(sy.tw);
    for (int i = tid; i < N; i += NT) tw[i] = twg[i];
    tw_sys = bp.sys;
  }
  if (NT != BNTR) {
    // per-phase launch of the z pass with 256-thread workgroups: one tile per item
    KernelParams kp;
    kp.kind = sy.kind;
    kp.omega = sy.omega;
    kp.inv_ng = sy.inv_ng;
    kp.g[0] = sy.g[0]; kp.g[1] = sy.g[1]; kp.g[2] = sy.g[2];
    body_conv_z_r<T, N, r2c_tx<N>(), NT, V>(spec, sub * r2c_tx<N>(), kp, buf, tw, tid);
  } else if (p == 0) {
    const size_t zo = size_t(sub) * N * N;
    body_fwd_xy_r<T, N, BNTR, V>(phi + size_t(oi) * NG + zo, phi + size_t(oj) * NG + zo, spec + size_t(sub) * PL,
                                 buf, tw, tid);
  } else if (p == 1) {
    KernelParams kp;
    kp.kind = sy.kind;
    kp.omega = sy.omega;
    kp.inv_ng = sy.inv_ng;
    kp.g[0] = sy.g[0]; kp.g[1] = sy.g[1]; kp.g[2] = sy.g[2];
    constexpr int TXR = r2c_tx<N>(), NTILE = N * XS / TXR, HALF = BNTR / 2;
    const int half = tid >= HALF ? 1 : 0;
    const int tile = 2 * sub + half;
    // each half has its own N * TXR slice of the LDS buffer
    body_conv_z_r<T, N, TXR, HALF, V>(spec, (tile < NTILE ? tile : NTILE - 1) * TXR, kp, buf + half * N * TXR, tw,
                                      tid - half * HALF, tile < NTILE);
  } else {
    const size_t zo = size_t(sub) * N * N;
    body_inv_xy_r<T, N, BNTR, V>(spec + size_t(sub) * PL, buf, tw, tid);
    T* W = static_cast<T*>(sy.W);
    accumulate_w_r<T, N, BNTR, false>(phi + size_t(oi) * NG + zo, phi + size_t(oj) * NG + zo,
                                      W + size_t(oi) * NG + zo, W + size_t(oj) * NG + zo, oi != oj, nullptr, buf,
                                      red, tid);
  }
}

// The items of phase p of one segment, split into contiguous ranges, one per
// workgroup: the pack of the first item is found by bisection, then the pack
// index only moves forward.
template <typename T, int N, int V, int NT>
__device__ __forceinline__ void run_range_r(int p, const BRound& sg, const BSys* __restrict__ sys,
                                            const BPack* __restrict__ packs, const int64_t* __restrict__ starts,
                                            cplx<T>* buf, cplx<T>* tw, int& tw_sys, double* red) {
  const int64_t total = sg.nitems[p];
  const int64_t per = (total + gridDim.x - 1) / gridDim.x;
  int64_t j = int64_t(blockIdx.x) * per;
  const int64_t jend = (j + per < total) ? j + per : total;
  if (j >= jend) return;
  const int64_t* st = starts + sg.start_off[p];
  int lo = 0, hi = sg.npacks;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] <= j) lo = mid; else hi = mid;
  }
  int q = lo;
  for (; j < jend; ++j) {
    while (q + 1 < sg.npacks && st[q + 1] <= j) ++q;
    run_item_r<T, N, V, NT>(p, j, q, sg, sys, packs, st, buf, tw, tw_sys, red);
  }
}

// One phase P of one segment (the phase is a template parameter so that each
// launch carries only its own body).
template <typename T, int N, int V, int P>
__global__ __launch_bounds__(BNTR, 4) void k_batched_phase_r(BRound sg, const BSys* __restrict__ sys,
                                                          const BPack* __restrict__ packs,
                                                          const int64_t* __restrict__ starts) {
  __shared__ cplx<T> buf[N * r2c_xs<N>()];
  __shared__ cplx<T> tw[N];
  __shared__ double red[BNTR / 64];
  int tw_sys = -1;
  run_range_r<T, N, V, BNTR>(P, sg, sys, packs, starts, buf, tw, tw_sys, red);
}

// The z pass as its own per-phase launch: 256-thread workgroups, one tile each.
template <typename T, int N, int V>
__global__ __launch_bounds__(256) void k_batched_conv_r(BRound sg, const BSys* __restrict__ sys,
                                                        const BPack* __restrict__ packs,
                                                        const int64_t* __restrict__ starts) {
  __shared__ cplx<T> buf[N * r2c_tx<N>()];
  __shared__ cplx<T> tw[N];
  __shared__ double red[4];
  int tw_sys = -1;
  run_range_r<T, N, V, 256>(1, sg, sys, packs, starts, buf, tw, tw_sys, red);
}

template <typename T, int N, int V>
__global__ __launch_bounds__(BNTR, 4) void k_batched_persistent_r(int nseg, const BRound* __restrict__ segs,
                                                               const BSys* __restrict__ sys,
                                                               const BPack* __restrict__ packs,
                                                               const int64_t* __restrict__ starts) {
  __shared__ cplx<T> buf[r2c_buf_elems<N>()];
  __shared__ cplx<T> tw[N];
  __shared__ double red[BNTR / 64];
  cg::grid_group grid = cg::this_grid();
  int tw_sys = -1;
  for (int r = 0; r < nseg; ++r) {
    const BRound sg = segs[r];
    for (int p = 0; p < 3; ++p) {
      run_range_r<T, N, V, BNTR>(p, sg, sys, packs, starts, buf, tw, tw_sys, red);
      grid.sync();
    }
  }
}

template <typename T, int N, int V>
static hipError_t launch_seg_r(int mode, int nseg, const BRound* h_segs, const BRound* d_segs, const BSys* sys,
                               const BPack* packs, const int64_t* starts, int blocks_per_cu, hipStream_t s) {
  if (mode == 1) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batched_persistent_r<T, N, V>, BNTR, 0);
    if (e != hipSuccess) return e;
    if (per < 1) return hipErrorInvalidConfiguration;
    const int use = (blocks_per_cu > 0 && blocks_per_cu < per) ? blocks_per_cu : per;
    dim3 grid(unsigned(ncu * use)), block(BNTR);
    void* args[] = {&nseg, (void*)&d_segs, (void*)&sys, (void*)&packs, (void*)&starts};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batched_persistent_r<T, N, V>), grid, block,
                                      args, 0, s);
  }
  const int grid_cap = 256 * (blocks_per_cu > 0 ? blocks_per_cu : 8);
  for (int r = 0; r < nseg; ++r)
    for (int p = 0; p < 3; ++p) {
      const int64_t n = h_segs[r].nitems[p];
      if (n == 0) continue;
      // one workgroup per item: the dispatcher overlaps the item prologues
      // (blocks_per_cu > 8 caps the grid and loops instead)
      const unsigned g = unsigned(blocks_per_cu > 8 && n > grid_cap ? grid_cap : n);
      if (p == 0)
        hipLaunchKernelGGL((k_batched_phase_r<T, N, V, 0>), dim3(g), dim3(BNTR), 0, s, h_segs[r], sys, packs, starts);
      else if (p == 1)
        hipLaunchKernelGGL((k_batched_conv_r<T, N, V>), dim3(unsigned(n)), dim3(256), 0, s, h_segs[r], sys,
                           packs, starts);
      else
        hipLaunchKernelGGL((k_batched_phase_r<T, N, V, 2>), dim3(g), dim3(BNTR), 0, s, h_segs[r], sys, packs, starts);
    }
  return hipGetLastError();
}

// ---- owner layout: the spectra of every pair of the segment's systems are
// resident, so the forward and z passes run over all pairs in one launch each
// and W_k of each system is formed once per (orbital, plane) from the pairs
// that contain k (no rounds, no read-modify-write of W).

// Forward: grid (pair slots, N), slot fastest so that the planes of the
// orbitals of one system are read by neighbouring workgroups.
template <typename T, int N, int V>
__global__ __launch_bounds__(BNTR, 4) void k_batched_owner_fwd_r(const BSys* __restrict__ sys,
                                                              const BPack* __restrict__ packs) {
  constexpr size_t NG = size_t(N) * N * N, PL = size_t(N) * r2c_xs<N>();
  __shared__ cplx<T> buf[N * r2c_xs<N>()];
  __shared__ cplx<T> tw[N];
  const int slot = blockIdx.x, z = blockIdx.y;
  const BPack bp = packs[slot >> 1];
  const int i = (slot & 1) ? bp.pk.ib : bp.pk.ia, j = (slot & 1) ? bp.pk.jb : bp.pk.ja;
  if (j < 0) return;
  const BSys& sy = sys[bp.sys];
  const cplx<T>* twg = static_cast<const cplx<T>*>(sy.tw);
  for (int t = threadIdx.x; t < N; t += BNTR) tw[t] = twg[t];
  const T* phi = static_cast<const T*>(sy.phi);
  const size_t zo = size_t(z) * N * N;
  cplx<T>* spec = static_cast<cplx<T>*>(bp.spec) + size_t(slot & 1) * N * PL + size_t(z) * PL;
  body_fwd_xy_r<T, N, BNTR, V>(phi + size_t(i) * NG + zo, phi + size_t(j) * NG + zo, spec, buf, tw, threadIdx.x);
}

// z pass: one 256-thread workgroup per (pair slot, tile), tiles of a slot adjacent.
template <typename T, int N, int V>
__global__ __launch_bounds__(256) void k_batched_owner_conv_r(const BSys* __restrict__ sys,
                                                              const BPack* __restrict__ packs) {
  constexpr int TXR = own_tx<T, N>(), NTILE = own_ntile<T, N>();
  constexpr size_t PL = size_t(N) * r2c_xs<N>();
  __shared__ cplx<T> buf[N * TXR];
  __shared__ cplx<T> tw[N];
  const int64_t g = blockIdx.x;
  const int slot = int(g / NTILE), tile = int(g % NTILE);
  const BPack bp = packs[slot >> 1];
  if ((slot & 1) && bp.pk.jb < 0) return;
  const BSys& sy = sys[bp.sys];
  const cplx<T>* twg = static_cast<const cplx<T>*>(sy.tw);
  for (int t = threadIdx.x; t < N; t += 256) tw[t] = twg[t];
  KernelParams kp;
  kp.kind = sy.kind;
  kp.omega = sy.omega;
  kp.inv_ng = sy.inv_ng;
  kp.g[0] = sy.g[0]; kp.g[1] = sy.g[1]; kp.g[2] = sy.g[2];
  cplx<T>* spec = static_cast<cplx<T>*>(bp.spec) + size_t(slot & 1) * N * PL;
  body_conv_z_r<T, N, TXR, 256, V>(spec, tile * TXR, kp, buf, tw, threadIdx.x, true, nullptr, nullptr,
                                   static_cast<const T*>(sy.vt));
}

// W_k of plane z of one system: one workgroup per (system, orbital, plane)
// item.  The items are dealt to the eight XCDs in turn: XCD x is given the
// planes z = x mod 8, with the orbitals of all systems fastest (as in the
// single-build owner pass); the system is found by bisection over the orbital
// offsets.  Adjacency entries (slot, partner) index the slots of the
// segment's spectra.
template <typename T, int N, int V>
__global__ __launch_bounds__(BNTR, 4) void k_batched_owner_r(int nown, const BOwner* __restrict__ own,
                                                          const BSys* __restrict__ sys,
                                                          const int32_t* __restrict__ adj,
                                                          const cplx<T>* __restrict__ spec) {
  constexpr size_t NG = size_t(N) * N * N;
  __shared__ cplx<T> buf[N * r2c_xs<N>()];
  __shared__ cplx<T> tw[N];
  const int64_t g = blockIdx.x, l = g >> 3;
  const int64_t norb_all = int64_t(gridDim.x) / N;
  const int z = int(l / norb_all) * 8 + int(g & 7);
  const int64_t j = l % norb_all;
  int lo = 0, hi = nown;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (own[mid].orb0 <= j) lo = mid; else hi = mid;
  }
  const BOwner o = own[lo];
  const BSys& sy = sys[o.sys];
  const int k = o.operm ? o.operm[j - o.orb0] : int(j - o.orb0);
  const cplx<T>* twg = static_cast<const cplx<T>*>(sy.tw);
  for (int t = threadIdx.x; t < N; t += BNTR) tw[t] = twg[t];
  const size_t zo = size_t(z) * N * N;
  T* W = static_cast<T*>(sy.W) + size_t(k) * NG + zo;
  body_inv_owner_r<T, N, BNTR, V>(static_cast<const T*>(sy.phi), spec, adj, o.adj_ptr[k], o.adj_ptr[k + 1], zo, W,
                                  buf, tw, threadIdx.x);
}

template <typename T, int N, int V>
static hipError_t launch_owner_t(int nslots, int nown, int64_t items, const BSys* sys, const BPack* packs,
                                 const BOwner* own, const int32_t* adj, const void* spec, hipStream_t s) {
  constexpr int64_t NTILE = own_ntile<T, N>();
  if (NTILE * nslots > int64_t(0x7fffffff) || items > int64_t(0x7fffffff)) return hipErrorInvalidValue;
  if (nslots > 0) {
    hipLaunchKernelGGL((k_batched_owner_fwd_r<T, N, V>), dim3(unsigned(nslots), N), dim3(BNTR), 0, s, sys, packs);
    hipLaunchKernelGGL((k_batched_owner_conv_r<T, N, V>), dim3(unsigned(NTILE * nslots)), dim3(256), 0, s, sys,
                       packs);
  }
  if (items > 0)
    hipLaunchKernelGGL((k_batched_owner_r<T, N, V>), dim3(unsigned(items)), dim3(BNTR), 0, s, nown, own, sys, adj,
                       static_cast<const cplx<T>*>(spec));
  return hipGetLastError();
}

hipError_t batched_owner(int prec, int n, int plan_v, int nslots, int nown, int64_t items, const BSys* sys,
                         const BPack* packs, const BOwner* own, const int32_t* adj, const void* spec, hipStream_t s) {
  switch (n) {
#define X(nn)                                                                                                  \
  case nn:                                                                                                     \
    if (prec == 0)                                                                                             \
      return plan_v ? launch_owner_t<double, nn, 1>(nslots, nown, items, sys, packs, own, adj, spec, s)         \
                    : launch_owner_t<double, nn, 0>(nslots, nown, items, sys, packs, own, adj, spec, s);        \
    return plan_v ? launch_owner_t<float, nn, 1>(nslots, nown, items, sys, packs, own, adj, spec, s)            \
                  : launch_owner_t<float, nn, 0>(nslots, nown, items, sys, packs, own, adj, spec, s);
    X(16) X(24) X(32) X(48) X(64) X(80) X(96)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

bool batched_r2c_fits(int prec, int n) {
  switch (n) {
#define X(nn) case nn: return (size_t(r2c_buf_elems<nn>()) + nn) * (prec == 0 ? 16 : 8) + 1024 <= 163840;
    X(16) X(24) X(32) X(48) X(64) X(80) X(96)
#undef X
    default: return false;
  }
}

int64_t batched_r2c_slot_items(int n, int phase, bool persistent) {
  switch (n) {
#define X(nn) case nn: return r2c_slot_items<nn>(phase, persistent ? 2 : 1);
    X(16) X(24) X(32) X(48) X(64) X(80) X(96)
#undef X
    default: return 0;
  }
}

bool batched_supported(int n) {
  return n == 16 || n == 24 || n == 32 || n == 48 || n == 64 || n == 80 || n == 96;
}

int64_t batched_phase_items(int n, int phase, int txv) { return batched_items(n, phase, txv); }

template <typename T, int N, int TXV, int V>
static hipError_t launch_seg_t(int mode, int nseg, const BRound* h_segs, const BRound* d_segs, const BSys* sys,
                               const BPack* packs, const int64_t* starts, int blocks_per_cu, hipStream_t s) {
  if (mode == 1) {
    int dev = 0, ncu = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_batched_persistent<T, N, TXV, V>, BNT, 0);
    if (e != hipSuccess) return e;
    if (per < 1) return hipErrorInvalidConfiguration;
    const int use = (blocks_per_cu > 0 && blocks_per_cu < per) ? blocks_per_cu : per;
    dim3 grid(unsigned(ncu * use)), block(BNT);
    void* args[] = {&nseg, (void*)&d_segs, (void*)&sys, (void*)&packs, (void*)&starts};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_batched_persistent<T, N, TXV, V>), grid, block,
                                      args, 0, s);
  }
  const int grid_cap = 256 * (blocks_per_cu > 0 ? blocks_per_cu : 8);
  for (int r = 0; r < nseg; ++r)
    for (int p = 0; p < 5; ++p) {
      const int64_t n = h_segs[r].nitems[p];
      if (n == 0) continue;
      const unsigned g = unsigned(n < grid_cap ? n : grid_cap);
      hipLaunchKernelGGL((k_batched_phase<T, N, TXV, V>), dim3(g), dim3(BNT), 0, s, p, h_segs[r], sys, packs, starts);
    }
  return hipGetLastError();
}

template <typename T, int N>
static hipError_t launch_seg_n(int mode, int txv, int plan_v, int nseg, const BRound* h, const BRound* d,
                               const BSys* sys, const BPack* packs, const int64_t* starts, int bpc, hipStream_t s) {
  if (txv == 8)
    return plan_v ? launch_seg_t<T, N, 8, 1>(mode, nseg, h, d, sys, packs, starts, bpc, s)
                  : launch_seg_t<T, N, 8, 0>(mode, nseg, h, d, sys, packs, starts, bpc, s);
  return plan_v ? launch_seg_t<T, N, 16, 1>(mode, nseg, h, d, sys, packs, starts, bpc, s)
                : launch_seg_t<T, N, 16, 0>(mode, nseg, h, d, sys, packs, starts, bpc, s);
}

// Launch the segments [h_segs, h_segs + nseg), all of grid size n.
hipError_t batched_segments(int prec, int n, int mode, int txv, int plan_v, int blocks_per_cu, int nseg,
                            const BRound* h_segs, const BRound* d_segs, const BSys* sys, const BPack* packs,
                            const int64_t* starts, bool r2c, hipStream_t s) {
  if (r2c) {
    switch (n) {
#define X(nn)                                                                                                   \
  case nn:                                                                                                      \
    if (prec == 0)                                                                                              \
      return plan_v ? launch_seg_r<double, nn, 1>(mode, nseg, h_segs, d_segs, sys, packs, starts, blocks_per_cu, s) \
                    : launch_seg_r<double, nn, 0>(mode, nseg, h_segs, d_segs, sys, packs, starts, blocks_per_cu, s); \
    return plan_v ? launch_seg_r<float, nn, 1>(mode, nseg, h_segs, d_segs, sys, packs, starts, blocks_per_cu, s)    \
                  : launch_seg_r<float, nn, 0>(mode, nseg, h_segs, d_segs, sys, packs, starts, blocks_per_cu, s);
      X(16) X(24) X(32) X(48) X(64) X(80) X(96)
#undef X
      default:
        return hipErrorInvalidValue;
    }
  }
  switch (n) {
#define X(nn)                                                                                                  \
  case nn:                                                                                                     \
    return prec == 0 ? launch_seg_n<double, nn>(mode, txv, plan_v, nseg, h_segs, d_segs, sys, packs, starts,   \
                                                blocks_per_cu, s)                                              \
                     : launch_seg_n<float, nn>(mode, txv, plan_v, nseg, h_segs, d_segs, sys, packs, starts,    \
                                               blocks_per_cu, s);
    X(16) X(24) X(32) X(48) X(64) X(80) X(96)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// Zero fill without memset nodes (kept out of captured graphs).
__global__ void k_zero(uint32_t* __restrict__ p, int64_t n) {
  for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < n; e += int64_t(gridDim.x) * blockDim.x)
    p[e] = 0u;
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n = int64_t(bytes / 4);
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_zero, dim3(unsigned(g)), dim3(256), 0, s, static_cast<uint32_t*>(p), n);
}

}  // namespace ace
