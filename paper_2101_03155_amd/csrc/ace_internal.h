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

// Interaction kernel in reciprocal space: v(G) for the bare Coulomb 1/r
// (kind 0, v(0)=0) or erfc(omega r)/r (kind 1, v(0)=pi/omega^2).
struct KernelParams {
  int kind;
  double omega;
  double inv_ng;   // 1 / (grid size), folded into v(G)
  double g[3];     // 2 pi / L along x, y, z
};

// Kernel launch shape of the pair stage, chosen by the tuner.
struct PairShape {
  int fused_xy;    // 1: one workgroup per (plane, pack) does both in-plane FFTs
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

// Dense kernels (gemm.hip, linalg.hip).
hipError_t gemm_nt(int prec, bool abs_ops, const void* A, int64_t lda, const void* B, int64_t ldb, int M,
                   int Nn, int64_t K, double alpha, double* Cpart, double* C, hipStream_t s,
                   EventRecorder* rec);
int64_t gemm_nt_nsplit(int M, int Nn, int64_t K, int64_t* kchunk_out);
hipError_t gemm_ls(int bprec, bool trans, bool lower, const double* S, int lds, const void* B, int64_t ldb,
                   double* C, int64_t ldc, int M, int K, int64_t R, double alpha, hipStream_t s,
                   EventRecorder* rec);
void launch_symmetrize(const double* M, int n, double* out, double* negM, double* ex, double* asym, hipStream_t s);
void launch_cholesky(double* A, int n, int* info, hipStream_t s);
void launch_trinv(const double* L, int n, double* X, hipStream_t s);
void launch_colnorm(const double* A, int n, int64_t ng, double* res, hipStream_t s);
int qrcp_blocks(int64_t ng);
void launch_qrcp_update(const double* A, int n, int64_t ng, const double* q, double* res, double* pv, int64_t* pi,
                        hipStream_t s);
void launch_qrcp_select(const double* A, int n, int64_t ng, int k, const double* pv, const int64_t* pi, int nblk,
                        double* Q, double* res, int32_t* piv, double* qout, hipStream_t s);
void launch_gather_cols(const double* A, int n, int64_t ng, const int32_t* piv, double* AC, hipStream_t s);
void launch_scale_frob(double* X, int64_t cnt, hipStream_t s);
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
PairShape pair_default_shape(int prec, int N);

}  // namespace ace
