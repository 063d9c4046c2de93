// Internal declarations shared by the host layer and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ace {

// One unit of pair work: two orbital pairs whose densities are transformed
// together as the real and imaginary parts of one complex field.  jb < 0 marks
// a pack that carries a single pair.
struct Pack {
  int ia, ja, ib, jb;
};

// One pair slot of the k-point pair stage: Bloch orbitals a <= b and the
// shift d = k_b - k_a (bohr^-1) of the kernel; b < 0 marks an empty slot.
struct KPair {
  int a, b;
  double d[3];
};

// Interaction kernel in reciprocal space: v(G) for the bare Coulomb 1/r
// (kind 0, v(0)=0) or erfc(omega r)/r (kind 1, v(0)=pi/omega^2).
struct KernelParams {
  int kind;
  double omega;
  double inv_ng;   // 1 / (grid size), folded into v(G)
  double g[3];     // 2 pi / L along x, y, z
};

// Batched form: one system, one pack of a super-round, one super-round.
struct BSys {
  int N;
  int kind;
  double omega;
  double inv_ng;
  double g[3];
  const void* phi;  // [norb][N^3] in the pair-stage precision
  void* W;          // [norb][N^3] in the pair-stage precision
  const void* tw;   // N twiddles
  const void* vt;   // v(G) table of launch_vtable (owner layout) or null
};
struct BPack {
  int sys;
  int pad;
  Pack pk;
  void* spec;       // N^3 complex values of this pack
};
struct BRound {                // one segment: the packs of one grid size in one super-round
  int pack0, npacks;         // packs [pack0, pack0 + npacks) of the BPack table
  int64_t start_off[5];      // per phase: offset of the item prefix table (npacks + 1 entries)
  int64_t nitems[5];         // per phase: number of work items
};

// Owner layout of the batched form: one system of a grid-size segment.
struct BOwner {
  int sys;                   // index into the BSys table
  int norb;
  int64_t orb0;              // offset of the system's orbitals among those of the segment
  const int32_t* adj_ptr;    // [norb + 1] absolute offsets into the entry table
  const int32_t* operm;      // [norb] dispatch order of the owners (nullable: index order)
};

// Kernel launch shape of the pair stage, chosen by the tuner.
struct PairShape {
  int fused_xy;    // 0: split passes; 1: one workgroup per (plane, pack) does both in-plane FFTs;
                   // 2: real-to-complex, one workgroup per (plane, pair) on the half spectrum;
                   // 3: real-to-complex with all spectra resident and W formed per owner row
  int nt_xy;       // threads of the in-plane kernels (fused path)
  int tx;          // x-tile of the strided line kernels
};

// Timing hook: when non-null, each pair-stage launch of kernel class `cls`
// is bracketed by events appended to the recorder.
struct EventRecorder;
void rec_begin(EventRecorder* r, int cls, hipStream_t s);
void rec_end(EventRecorder* r, int cls, hipStream_t s, double units = 0.0);

enum KernelClass {
  KC_FWD_XY = 0,   // pair product + forward in-plane FFTs
  KC_CONV_Z = 1,   // forward z FFT, multiply by v(G), inverse z FFT
  KC_INV_XY = 2,   // inverse in-plane FFTs + W accumulation
  KC_FWD_X = 3, KC_FWD_Y = 4, KC_INV_Y = 5, KC_INV_X = 6,
  KC_GEMM_NT = 7, KC_GEMM_TN = 8, KC_QRCP = 9,
  ST_LOCALIZE = 10, ST_PAIRLIST = 11, ST_PAIRS = 12, ST_TAIL = 13, ST_BUILD = 14,
  KC_COUNT = 15
};

// Pair stage: process `npacks` packs (a conflict-free round) for an N^3 grid.
// phi, W are [norb][N^3] in precision `prec` (0 = FP64, 1 = FP32).
// spec is scratch of npacks * N^3 complex values.  epart (nullable) receives
// per-(pack, block) partial sums of v * rho for the pair energies; the number
// of blocks per pack is returned by pair_energy_blocks().
// npairs: orbital pairs carried by the packs (for the timing units).
hipError_t pair_round(int prec, int N, const PairShape& sh, const void* phi, void* spec,
                      const Pack* packs, int npacks, int npairs, void* W, double* epart,
                      const void* tw, const KernelParams& kp, hipStream_t s, EventRecorder* rec);
int pair_energy_blocks(int N, const PairShape& sh);
bool pair_supported(int N);
bool pair_r2c_fits(int prec, int N);
int pair_owner_ntile(int prec, int N);  // z-pass tiles per pair slot of the owner path
// Owner-computes W over all pairs (spectra of every pair resident); operm
// (nullable) is the order the owners are dispatched in; W may be
// null (energies only); epart: per (pack, tile) partial energies or null; vt:
// the table of launch_vtable or null (v(G) evaluated per element).
hipError_t pair_owner(int prec, int N, const void* phi, void* spec, const Pack* packs, int npacks, int npairs,
                      const int32_t* adj_ptr, const int32_t* adj, const int32_t* operm, int norb, int64_t nadj,
                      void* W, double* epart,
                      const void* tw, const KernelParams& kp, const void* vt, int chunk, hipStream_t s,
                      EventRecorder* rec);
// v(G) / N^3 over the folded frequencies, [zq][yq][kx] with zq, yq, kx in
// [0, N/2] ((N/2 + 1)^3 values in the pair-stage precision): v depends on
// ky and kz only through their squares.
hipError_t launch_vtable(int prec, int N, const KernelParams& kp, void* vt, hipStream_t s);
size_t pair_spec_elems(int prec, int N, const PairShape& sh);

// Dense kernels (gemm.hip, linalg.hip).
// op: 0 A B^T, 1 |A| |B|^T, 2 (A.A)(B.B)^T  (FP64 only for op != 0)
// sym: A == B (same rows, same op) and M == Nn; only the upper triangle of
// 128 x 128 tiles is computed and mirrored (FP64 only).
hipError_t gemm_nt(int prec, int op, const void* A, int64_t lda, const void* B, int64_t ldb, int M,
                   int Nn, int64_t K, double alpha, double* Cpart, double* C, hipStream_t s,
                   EventRecorder* rec, bool sym = false, int64_t max_split = 0);
// Split count of gemm_nt; the default (sym = true) is the largest count any
// product of this shape uses, for sizing the partial-sum buffer.  max_split > 0
// caps the count (K is then cut into longer chunks).
int64_t gemm_nt_nsplit(int M, int Nn, int64_t K, int64_t* kchunk_out, bool sym = true, int64_t max_split = 0);
hipError_t gemm_ls(int bprec, bool trans, bool lower, const double* S, int lds, const void* B, int64_t ldb,
                   double* C, int64_t ldc, int M, int K, int64_t R, double alpha, hipStream_t s,
                   EventRecorder* rec);
// res[r] -= sum_m (sum_k Q[m][k] Psi[k][r])^2 for r < R, over M <= 128 rows
// of Q (row pitch ldq) and K rows of Psi (row pitch ldp), in one launch.
hipError_t refresh_bounds(const double* Q, int ldq, const double* Psi, int64_t ldp, int M, int K, int64_t R,
                          double* res, hipStream_t s);
void launch_symmetrize(const double* M, int n, double* out, double* negM, double* ex, double* asym, hipStream_t s);
void launch_neg_sumsq(const double* c, int64_t n, double* out, hipStream_t s);
// Blocked Cholesky of the lower triangle of A (n <= 512) in place; info must
// be zero on entry; tinv is 64 x 64 doubles of scratch.
void launch_cholesky(double* A, int n, int* info, double* tinv, hipStream_t s);
void launch_trinv(const double* L, int n, double* X, hipStream_t s);
// -A = L L^T and X = L^-1 (zeros above the diagonal); info zero on entry, set
// as by launch_cholesky.  A holds L afterwards only where n > 128.
void launch_chol_inv(double* A, int n, int* info, double* X, double* tinv, hipStream_t s);
void launch_colnorm(const double* A, int n, int64_t ng, double* res, hipStream_t s);
int qrcp_blocks(int64_t ng);
void launch_qrcp_update(const double* A, int n, int64_t ng, const double* q, double* res, double* pv, int64_t* pi,
                        const int* stop, hipStream_t s);
int qrcp_pool_blocks(int P);
void launch_qrcp_update_r(double* R, int n, int P, const double* q, double* res, double* pv, int64_t* pi,
                          const int* stop, hipStream_t s);
void launch_qrcp_select_r(const double* R, int n, int P, int* kdev, const double* pv, const int64_t* pi,
                          double* Q, double* res, int32_t* piv, double* qout, const int32_t* pool,
                          const double* t_out, int* stop, hipStream_t s);
// Selection and update of one pool step in one launch (candidates read from
// pv_in/pi_in, written to pv_out/pi_out; n <= 1024).
void launch_qrcp_step_r(double* R, int n, int P, int* kdev, const double* pv_in, const int64_t* pi_in, double* Q,
                        double* res, int32_t* piv, const int32_t* pool, const double* t_out, int* stop,
                        double* pv_out, int64_t* pi_out, hipStream_t s);
void launch_add_inplace(double* a, const double* b, int64_t cnt, hipStream_t s);
void launch_qrcp_select(const double* A, int n, int64_t ng, int* kdev, const double* pv, const int64_t* pi,
                        int nblk, double* Q, double* res, int32_t* piv, double* qout, const int32_t* pool,
                        const double* t_out, int* stop, hipStream_t s);
int pool_blocks(int64_t ng);
void launch_pool_build(const double* res, int64_t ng, int pmax, unsigned* hist, double* t, int64_t* cnt,
                       double* tmax, int* total, double* t_out, hipStream_t s);
void launch_pool_write(const double* res, int64_t ng, const double* t, const int64_t* off, int32_t* pool,
                       double* pres, hipStream_t s);
void launch_pool_gather(const double* A, int n, int64_t ng, const int32_t* pool, int np, double* Apool,
                        hipStream_t s);
void launch_refresh_res(const double* L, int k, int64_t rc, const double* norm0, double* res, hipStream_t s);
void launch_retire(const int32_t* piv, int k, double* res, hipStream_t s);
void launch_gather_cols(const double* A, int n, int64_t ng, const int32_t* piv, double* AC, hipStream_t s);
void launch_scale_inf(double* X, const double* G, int n, hipStream_t s);
void launch_ns_combine(const double* X, const double* Z, double* Y, int64_t cnt, hipStream_t s);
void launch_dev_identity(const double* G, int n, double* out, hipStream_t s);
void launch_compact_pairs(const double* O, int n, double rho_cut, int64_t cap, int32_t* pairs, double* ov,
                          int64_t* count, hipStream_t s);
void launch_pair_energy(const double* epart, int npacks, int nblk, const Pack* packs, const int64_t* pidx, double dV,
                        double* e, hipStream_t s);
void launch_d2f(const double* a, float* b, int64_t n, hipStream_t s);
void launch_f2d(const float* a, double* b, int64_t n, hipStream_t s);
void launch_nonfinite(const double* a, int64_t n, int* flag, hipStream_t s);
bool pair_fused_fits(int prec, int N);
bool batched_supported(int n);
int64_t batched_phase_items(int n, int phase, int txv);
// Segments of one grid size n.  mode 0: one launch per (segment, phase);
// mode 1: one cooperative launch for all the segments.
hipError_t batched_segments(int prec, int n, int mode, int txv, int plan_v, int blocks_per_cu, int nseg,
                            const BRound* h_segs, const BRound* d_segs, const BSys* sys, const BPack* packs,
                            const int64_t* starts, bool r2c, hipStream_t s);
bool batched_r2c_fits(int prec, int n);
// Owner layout for the systems of grid size n: forward and z pass over the
// nslots pair slots of packs (whose spectra are all resident), then W of
// every system from its adjacency entries (slot, partner) in adj; items is the
// sum over the systems of norb * n (n a multiple of 8).
hipError_t batched_owner(int prec, int n, int plan_v, int nslots, int nown, int64_t items, const BSys* sys,
                         const BPack* packs, const BOwner* own, const int32_t* adj, const void* spec, hipStream_t s);
// work items per pair slot of phase 0..2 (the z pass packs two tiles per item
// in the persistent launch, one in the per-phase launches)
int64_t batched_r2c_slot_items(int n, int phase, bool persistent);
void launch_zero(void* p, size_t bytes, hipStream_t s);

// Learned screener (screener.hip).
void launch_marginals(const double* phi, int norb, int n, double* pz, double* py, double* px, hipStream_t s);
void launch_subsample(const double* phi, int norb, int n, int st, double* out, hipStream_t s);
void launch_centroids(const double* pz, const double* py, const double* px, int norb, int n, double L, double dV,
                      double* cen, double* spr, hipStream_t s);
void launch_pair_features(const int32_t* pairs, int64_t np, int norb, const double* cen, const double* spr,
                          const double* O, const double* P, double L, float* f, hipStream_t s);
void launch_mlp_init(float* m, uint64_t seed, hipStream_t s);
int stats_blocks(int64_t n);
void launch_mlp_stats(const float* x, const float* t, int64_t n, double* part, float* m, hipStream_t s);
void launch_mlp_forward(const float* m, const float* x, int64_t n, int clamp, float* y, hipStream_t s);
int mlp_grad_blocks(int bsz);
void launch_mlp_grad_partial(const float* m, const float* x, const float* t, int64_t n, int64_t off, int64_t stride,
                             int64_t b0, int bsz, float* gpart, float* lpart, hipStream_t s);
void launch_mlp_reduce(const float* gpart, const float* lpart, int nb, float* grad, float* loss, hipStream_t s);
void launch_mlp_adam(const float* gpart, const float* lpart, int nb, float* m, float* mom, float* vel, int step,
                     float lr, float b1, float b2, float eps, float* loss_acc, hipStream_t s);
void launch_select(const float* pred, const float* feats, int64_t np, int norb, const float* model, double budget,
                   const double* O, double rho_cut, float ood_tol, int* ood, double* tau, uint8_t* keep, int64_t cap,
                   int32_t* pairs, int64_t* count, float* q, double* w, hipStream_t s);
PairShape pair_default_shape(int prec, int N);

// k-point build (kpoint.hip): complex fields as interleaved (re, im) doubles.
hipError_t kpair_round(int N, const void* u, void* spec, const KPair* slots, int nslots, void* W, const void* tw,
                       const KernelParams& kp, double c, hipStream_t s);
void launch_times_minus_i(const void* W, void* Wm, int64_t n, hipStream_t s);
void launch_hermitize(const double* Re, const double* Im, int n, int nk, void* Mout, void* negM, hipStream_t s);
void launch_trace_avg(const double* Re, int n, int nk, double* ex, hipStream_t s);
void launch_chol_c(void* A, int n, int nk, int* info, hipStream_t s);
void launch_trinv_c(const void* L, int n, int nk, double* Xr, double* Xi, hipStream_t s);
void launch_cabs(const void* u, double* a, int64_t n, hipStream_t s);

}  // namespace ace
