/*
 * libace — screened adaptively compressed exchange (ACE) build on AMD MI355X.
 *
 * C ABI.  Every array argument is DEVICE memory owned by the caller (for
 * example torch tensors); the library never frees it and keeps no pointer to
 * it after a call returns.  Work is issued on the context's HIP stream.
 *
 * Units and layout (all entry points):
 *   - Hartree atomic units (bohr, Hartree);
 *   - a grid function is stored [z][y][x], x fastest, FP64, over an
 *     n[0] x n[1] x n[2] (= nx, ny, nz) periodic grid of an orthorhombic box
 *     with edges L[0..2] (bohr); N_G = nx*ny*nz, dV = Lx*Ly*Lz / N_G;
 *   - a set of orbitals is [norb][N_G] (orbital-major);
 *   - orbitals are real and orthonormal on the grid: sum_r phi_i phi_j dV = d_ij;
 *   - the Fourier convention is G = 2 pi k / L with k in FFT order over the
 *     full FFT box (no spherical cutoff).
 *
 * Errors: every call returns an ace_status; on failure ace_last_error() holds
 * a message and the outputs are unspecified.  Argument checks are done on the
 * host before any work is queued.  Supported grids: cubic, n = 8, 12, 16, 24,
 * 32, 48, 64, 80, 96, 100, 108, 120 or 160; 1 <= norb <= 512.
 *
 * Calls that must return a count or a factorization status to the host
 * (ace_pairlist, ace_build, ace_localize) synchronize the stream once.
 */
#ifndef ACE_H
#define ACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ace_ctx ace_ctx;

typedef enum {
  ACE_OK = 0,
  ACE_E_ARG = -1,         /* invalid argument (message names it)                 */
  ACE_E_HIP = -2,         /* HIP runtime error                                    */
  ACE_E_NOMEM = -3,       /* workspace allocation failed or above ACE_WORKSPACE_MAX */
  ACE_E_NOT_PD = -4,      /* -M not positive definite (message names the column) */
  ACE_E_CAPACITY = -5,    /* output capacity too small (required count returned) */
  ACE_E_NONFINITE = -6,   /* NaN/Inf met in M                                     */
  ACE_E_UNSUPPORTED = -7  /* grid size / shape not supported                      */
} ace_status;

typedef enum {
  ACE_KERNEL_COULOMB = 0, /* v(G) = 4 pi / G^2, v(0) = 0                            */
  ACE_KERNEL_ERFC = 1     /* erfc(omega r)/r: 4 pi/G^2 (1 - exp(-G^2/4 omega^2)),
                             v(0) = pi / omega^2                                    */
} ace_kernel;

typedef enum {
  ACE_FP64 = 0, /* every step in FP64                                            */
  ACE_FP32 = 1  /* pair products, FFTs and W in FP32; Phi^T W on FP32 matrix cores
                   with compensated summation; Cholesky, L^-1 and xi in FP64     */
} ace_precision;

typedef struct {
  int32_t n[3]; /* grid points along x, y, z */
  double L[3];  /* box edges along x, y, z (bohr) */
} ace_grid;

/* Library version string. */
const char* ace_version(void);

/* Create a context issuing work on `hip_stream` (a hipStream_t; NULL = the
 * default stream) on the current device.  The context owns workspaces, FFT
 * twiddle tables, pair schedules and timing events. */
int ace_create(ace_ctx** ctx, void* hip_stream);
int ace_destroy(ace_ctx* ctx);
const char* ace_last_error(const ace_ctx* ctx);
int ace_set_stream(ace_ctx* ctx, void* hip_stream);

/* Free every workspace the context has grown (device buffers of earlier
 * calls) and the batched graphs that refer to them; the next call allocates
 * again.  Synchronizes the context's streams first. */
int ace_release_workspace(ace_ctx* ctx);

/*
 * (a) Localization by selected columns of the density matrix (SCDM), the
 * unitary rotation of Eq. (unit), as used in the SCDM paragraph of Sec. Theory.
 *
 *   psi    [norb][N_G]  canonical orbitals (input)
 *   phi    [norb][N_G]  localized orbitals phi_k = sum_i psi_i U_ik (output)
 *   pivots [norb] int32 grid indices c_k picked by greedy QR with column
 *                        pivoting of A[i][r] = psi_i(r) (output)
 *   U      [norb][norb] orthogonal rotation, row i = psi index (output, nullable)
 *
 * Pivot k maximizes the residual norm of column r after projection onto the
 * previously picked columns; the 8 best downdated candidates are re-ranked by
 * explicitly projected residuals; ties go to the smaller grid index.
 * U = A_C (A_C^T A_C)^-1/2 with A_C = A[:, pivots] (Loewdin orthonormalization
 * of the selected density-matrix columns).  phi[k] belongs to pivots[k].
 */
int ace_localize(ace_ctx* ctx, const ace_grid* grid, int norb, const double* psi, double* phi,
                 int32_t* pivots, double* U);

/*
 * (a) on given columns: the Loewdin step of SCDM (Eq. unit) only,
 *   U = A_C (A_C^T A_C)^-1/2,  A_C = A[:, pivots],  phi_k = sum_i psi_i U_ik,
 * with no pivot search.  For MD, where the ACE operator is rebuilt every step
 * and the orbitals move little between steps, the columns ace_localize picked
 * at the previous step can be reused: any columns with a nonsingular A_C give
 * an orthonormal phi spanning the same occupied space.
 *   psi    [norb][N_G] (input)
 *   pivots [norb] int32 distinct grid indices in [0, N_G), device memory
 *          (input; copied to the host and checked before any kernel runs)
 *   phi    [norb][N_G] (output);  U [norb][norb] (output, nullable)
 * Errors: ACE_E_ARG for a repeated or out-of-range column, ACE_E_NONFINITE
 * when the polar iteration does not converge (A_C singular or nearly so:
 * call ace_localize for fresh columns).
 */
int ace_localize_pivots(ace_ctx* ctx, const ace_grid* grid, int norb, const double* psi, const int32_t* pivots,
                        double* phi, double* U);

/*
 * (b) without a host synchronization: as ace_pairlist, but the kept count is
 * written to npairs (DEVICE int64) and nothing waits for it, so a caller can
 * queue the screening and the following work without a round trip (or
 * capture them in a graph after one call has grown the workspaces).  Pairs
 * beyond capacity are not written; the caller compares *npairs with capacity.
 */
int ace_pairlist_device(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, double rho_cut,
                        int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs);

/*
 * (a) at the next MD step, with the previous step's columns as the warm start
 * (the ACE operator is rebuilt at least once per MD step, Sec. Theory).
 *   pivots  [norb] int32, device (in: the previous step's columns; out: the
 *           columns used at this step)
 *   cond_max >= 1: the previous columns are kept when (max_k R_kk / min_k R_kk)^2,
 *           with A_C = Q R the QR factorization of this step's A[:, pivots] in
 *           pivot order (read from the Cholesky factor of A_C^T A_C), is at most
 *           cond_max; then only the Loewdin step of Eq. (unit) runs, as in
 *           ace_localize_pivots.  Otherwise (or when the polar iteration fails)
 *           a fresh SCDM (ace_localize) picks new columns.
 *   phi, U  as ace_localize;  info (HOST): reused_columns, gram_cond.
 * Greedy pivoting keeps that ratio small, so the fresh columns' ratio is the
 * natural reference for cond_max.  Errors as ace_localize_pivots.
 */
typedef struct {
  int32_t reused_columns; /* 1: previous columns kept (Loewdin only); 0: fresh SCDM      */
  double gram_cond;       /* (max R_kk / min R_kk)^2 of the previous columns (inf if singular) */
  int64_t pairs_added;    /* ace_pairlist_step: kept now, not in the previous list        */
  int64_t pairs_removed;  /* ace_pairlist_step: in the previous list, not kept now        */
} ace_step_info;

int ace_localize_step(ace_ctx* ctx, const ace_grid* grid, int norb, const double* psi, int32_t* pivots,
                      double cond_max, double* phi, double* U, ace_step_info* info);

/*
 * (b) at the next MD step: ace_pairlist on this step's orbitals, compared
 * pair by pair with the previous step's list (meaningful when the columns
 * were kept, so orbital k continues orbital k): info->pairs_added and
 * info->pairs_removed count the pairs whose overlap crossed rho_cut upward
 * and downward.  prev_pairs [nprev][2] int32 device, sorted by (i, j) (as
 * ace_pairlist writes them); the other arguments and errors as ace_pairlist.
 */
int ace_pairlist_step(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, double rho_cut,
                      const int32_t* prev_pairs, int64_t nprev, int64_t capacity, int32_t* pairs, double* overlap,
                      int64_t* npairs, ace_step_info* info);

/*
 * (b) Pair screening (criterion in the SCDM paragraph of Sec. Theory): keep
 * (i, j), i <= j, when  O_ij = dV sum_r |phi_i(r)| |phi_j(r)|  >= rho_cut;
 * diagonal pairs are always kept.
 *
 *   pairs    [capacity][2] int32 (i, j) sorted by i then j (output)
 *   overlap  [capacity] FP64 O_ij of each kept pair (output, nullable)
 *   npairs   HOST pointer: number of kept pairs (output)
 *
 * If more than `capacity` pairs are kept, returns ACE_E_CAPACITY with the
 * required count in *npairs.
 */
int ace_pairlist(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, double rho_cut,
                 int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs);

/*
 * (c)-(e) ACE build over a pair list (Appendix A applied to the screened
 * exchange of Eq. (vx)):
 *   (c) for each pair (i, j): v_ij = K * (phi_i phi_j) by FFT (Eq. e:vij),
 *       W_i -= v_ij phi_j and, if i != j, W_j -= v_ij phi_i;
 *   (d) M = dV Phi W^T, symmetrized (M + M^T)/2; -M = L L^T (Cholesky);
 *   (e) xi = L^-1 W, i.e. the projectors P = W L^-T, so V_ACE = -xi^T xi dV.
 *
 *   phi     [norb][N_G] orthonormal orbitals (input)
 *   pairs   [npairs][2] int32, 0 <= i <= j < norb, no duplicates (input)
 *   kernel  ace_kernel; omega used for ACE_KERNEL_ERFC (bohr^-1)
 *   prec    ace_precision
 *   xi      [norb][N_G] projectors (output)
 *   M       [norb][norb] symmetrized M (output, nullable)
 *   W       [norb][N_G] FP64 copy of W (output, nullable)
 *   ex      [1] E_x = tr M, Hartree (output, nullable)
 *   pair_energy [npairs] e_ij = -(2 - d_ij) dV sum_r phi_i phi_j v_ij
 *           (output, nullable); sum of e_ij equals E_x
 *
 * Returns ACE_E_NOT_PD when -M is not positive definite (a screened list that
 * dropped too much); rebuilding with the full pair list is the remedy.
 */
int ace_build(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, const int32_t* pairs,
              int64_t npairs, int kernel, double omega, int prec, double* xi, double* M, double* W,
              double* ex, double* pair_energy);

/*
 * ACE application (Sec. Theory, equation after Eq. e:vij; Appendix A):
 *   y_a = V_ACE x_a = -sum_k xi_k <xi_k | x_a>,  <f|g> = dV sum_r f g.
 *   xi [norb][N_G], x [nvec][N_G] (inputs), y [nvec][N_G] (output).
 */
int ace_apply(ace_ctx* ctx, const ace_grid* grid, int norb, const double* xi, int nvec, const double* x,
              double* y);

/*
 * ACE application fused with the exchange energy of the functions it is
 * applied to (Appendix A, projector form; with x the occupied orbitals this is
 * one SCF cycle's application and E_x).  Both results come from the same
 * coefficients c_ka = <xi_k | x_a>:
 *   y_a = -sum_k c_ka xi_k,   ex = sum_a <x_a | V_ACE x_a> = -sum_ka c_ka^2.
 *   xi [norb][N_G], x [nvec][N_G] (inputs), y [nvec][N_G] (output),
 *   ex [1] Hartree, device memory (output, required).
 * Arguments and errors as ace_apply; the energy is summed in a fixed order.
 */
int ace_apply_energy(ace_ctx* ctx, const ace_grid* grid, int norb, const double* xi, int nvec, const double* x,
                     double* y, double* ex);

/*
 * ace_apply_energy for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results as ace_apply_energy (to the rounding of a different
 * split-K summation order), with its scratch (the split-K partial sums and
 * the coefficients c_ka) in a fixed device array of ACE_NOALLOC_SCRATCH_BYTES
 * that the library holds on each device until the process ends.  The call
 * allocates nothing and frees nothing; the caller passes every input and
 * output.  Limits: norb <= 512, nvec <= 512 (ACE_E_ARG beyond); the split
 * count of the product is capped so the partial sums fit.  Every call on a
 * device shares that device's array: calls that overlap on one device (two
 * streams, two contexts) race, so serialize them.
 */
#define ACE_NOALLOC_SCRATCH_BYTES ((4 * 1048576 + 512 * 512) * 8)
int ace_apply_energy_noalloc(ace_ctx* ctx, const ace_grid* grid, int norb, const double* xi, int nvec,
                             const double* x, double* y, double* ex);

/*
 * Exact exchange on the orbitals themselves (Eq. vx over every pair, no
 * screening and no localization): the full-rank operator behind the exact
 * force of the multiple-time-step force splitting (Sec. Theory).
 *   W_i = V_X psi_i = -sum_j v_ij psi_j   (steps (c) of ace_build, all pairs)
 *   M_kl = <psi_k | W_l>, symmetrized;  ex = tr M.
 *   psi  [norb][N_G] orthonormal orbitals (input)
 *   kernel, omega, prec as ace_build (prec sets the pair stage; W is returned
 *        in FP64 either way)
 *   W    [norb][N_G] (output, required)
 *   M    [norb][norb] (output, nullable)
 *   ex   [1] Hartree, device memory (output, nullable)
 * The pair list i <= j is generated internally (norb (norb + 1) / 2 pairs).
 * No Cholesky or projectors are formed.  Errors as ace_build.
 */
int ace_exact_exchange(ace_ctx* ctx, const ace_grid* grid, int norb, const double* psi, int kernel, double omega,
                       int prec, double* W, double* M, double* ex);

/*
 * Complex orbitals with k-points (the screening criterion of Sec. Theory is
 * written with phi_j*; Eq. (vx) and Appendix A with conjugates).  The
 * orbitals are Bloch functions psi_a(r) = exp(i k_a.r) u_a(r) on an N_k-point
 * sampling of the Brillouin zone, given by their cell-periodic parts u.
 * Complex arrays are interleaved (re, im) FP64 pairs.
 *
 *   norb    bands per k-point;  nk  k-points (nk * norb <= 2048)
 *   kvec    HOST [nk][3] k-point coordinates kx, ky, kz (bohr^-1)
 *   u       [nk * norb][N_G] complex: u_a, a = q * norb + m (k-point q, band m);
 *           orthonormal within each k-point: dV sum_r conj(u_a) u_b = d_ab
 *   pairs   [npairs][2] int32 over a: 0 <= a <= b < nk * norb, no duplicates
 *   xi      [nk * norb][N_G] complex projectors (output)
 *   M       [nk][norb][norb] complex, each Hermitian (output, nullable)
 *   W       [nk * norb][N_G] complex (output, nullable)
 *   ex      [1] E_x = (1/N_k) sum_k tr M_k, Hartree (output, nullable)
 *
 * For a pair (a, b), d = k_b - k_a and
 *   V = IFFT( v(|G + d|) FFT(conj(u_a) u_b) )   (Eq. e:vij with the Bloch phase),
 *   w_b -= V u_a / N_k  and, if a != b,  w_a -= conj(V) u_b / N_k,
 * i.e. W = V_X psi on the periodic parts, with the Brillouin-zone average.
 * The operator is block-diagonal in k: per k-point M = dV U^H W made
 * Hermitian, -M = L L^H, and P = W L^-H (Appendix A), returned by rows as
 * xi = conj(L)^-1 W, so that V_ACE x = -sum_j xi_j <xi_j|x> dV.  FP64 only.
 * Errors as ace_build; ACE_E_NOT_PD names the k-point and the column.
 */
int ace_build_kpoints(ace_ctx* ctx, const ace_grid* grid, int norb, int nk, const double* kvec, const double* u,
                      const int32_t* pairs, int64_t npairs, int kernel, double omega, double* xi, double* M,
                      double* W, double* ex);

/*
 * Screening of Bloch orbitals (criterion of Sec. Theory with phi_j*): keep
 * (a, b), a <= b, when  dV sum_r |u_a| |u_b|  (= the integral of |psi_a psi_b*|,
 * |exp(i k.r)| = 1)  >= rho_cut; diagonal pairs always kept.  u as for
 * ace_build_kpoints with ntot = nk * norb rows; the other arguments and the
 * errors as ace_pairlist.
 */
int ace_pairlist_kpoints(ace_ctx* ctx, const ace_grid* grid, int ntot, const double* u, double rho_cut,
                         int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs);

/*
 * Timing.  While enabled, every launch of the hot kernels and every stage of
 * the calls above is bracketed by HIP events on the context stream.
 * ace_profile_read synchronizes and returns, for class `cls`, the number of
 * bracketed launches, their summed milliseconds and their summed algorithmic
 * work `units` (HBM bytes for the pair-stage and pivot-search classes, flops
 * for the GEMM classes; 0 for stages), then clears the class if reset != 0.
 * Classes:
 *   0 pair product + forward in-plane FFTs      (3 N^3 s bytes per pair)
 *   1 z FFT, v(G) multiply, inverse z FFT        (2 N^3 s bytes per pair)
 *   2 inverse in-plane FFTs + W update           (7 N^3 s bytes per pair)
 *   3..6 split path: forward x, forward y, inverse y, inverse x passes
 *   7 split-K GEMM (2 M N K flops), 8 left-small GEMM (2 M K R flops)
 *   9 pivot-search update pass ((norb + 2) N_G 8 bytes)
 *   10 localize, 11 pairlist, 12 pair stage, 13 M + Cholesky + projectors,
 *   14 whole ace_build
 * (s = 8 bytes in FP64, 4 in FP32.)
 */
int ace_profile_enable(ace_ctx* ctx, int enable);
int ace_profile_read(ace_ctx* ctx, int cls, int64_t* launches, double* total_ms, double* units, int reset);
/* Restrict the bracketing to the classes whose bit (1 << cls) is set in mask
 * (default: all); the others cost no events.  Lets a caller time a run
 * without bracketing its many small launches (e.g. the pivot-search steps)
 * while still timing the stages and the dominant kernels.  ACE_E_ARG for bits
 * beyond the last class. */
int ace_profile_classes(ace_ctx* ctx, unsigned mask);

/*
 * Pair-stage launch shape for one (precision, grid size), set by the autotuner:
 *   fused = 0  separate x, y and z passes over the complex field of a pack of
 *              two pairs (16 N^3 s algorithmic bytes per pair);
 *   fused = 1  one workgroup per (z-plane, pack) does both in-plane FFTs with
 *              the plane in LDS (12 N^3 s per pair);
 *   fused = 2  real-to-complex: one workgroup per (z-plane, pair) on the half
 *              spectrum N x N x (N/2 + 1) (12 N^3 s per pair, half the LDS);
 *   fused = 3  real-to-complex with the half spectra of all pairs resident and
 *              W formed per owner row: one workgroup per (z-plane, orbital k)
 *              sums v_kj phi_j over k's pairs and writes W_k once (about
 *              9 N^3 s per pair; no conflict-free rounds).  The owners run in
 *              a reverse Cuthill-McKee order of the pair graph (in index
 *              order when the environment sets ACE_OWNER_ORDER=0 before
 *              ace_create; results agree to rounding).  When the spectra
 *              exceed ACE_OWNER_SPECTRA_MAX bytes (default 96 GiB) the build
 *              uses fused = 2 instead.  The default where two real-to-complex
 *              planes fit in one CU's LDS.
 * A path whose plane does not fit in LDS for this size falls back to 0; other
 * values of fused are ACE_E_ARG.
 * max_packs (>= 1) caps the packs per launch.  Results agree between paths to
 * rounding.
 */
int ace_set_pair_shape(ace_ctx* ctx, int prec, int n, int fused, int max_packs);
int ace_get_pair_shape(ace_ctx* ctx, int prec, int n, int* fused, int* max_packs);

/*
 * Batched form: many independent ACE builds (uneven orbital counts, grids,
 * pair lists and kernels) in shared launches.  Each system is what ace_build
 * takes; its pair list is split into conflict-free rounds, round r of every
 * system forms super-round r, and the pair-stage passes of a super-round run
 * in launches shared by all its systems of one grid size.
 *
 *   grid, norb, kernel, omega, phi, pairs, npairs  as for ace_build (inputs)
 *   xi, M (nullable), ex (nullable)                 as for ace_build (outputs)
 *   status, fail_column  HOST fields written by the call: ACE_OK, or
 *                        ACE_E_NOT_PD / ACE_E_NONFINITE with the column
 *
 * prec: ace_precision (the precision form runs the pair stage in FP32).
 * mode 0: the whole batched build (pair stage and every system's M, Cholesky
 *         and projectors) is captured in a hipGraph on a private stream and
 *         replayed when the same inputs come back;
 * mode 1: one persistent cooperative launch per grid size runs all its
 *         super-rounds and passes, with grid-wide barriers between passes;
 * mode 2: the launches of mode 0 issued directly.
 * Grid sizes: 16, 24, 32, 48, 64, 80 or 96.  Returns ACE_E_NOT_PD if any
 * system failed its factorization (the others are complete).
 */
typedef struct {
  ace_grid grid;
  int32_t norb;
  int32_t kernel;
  double omega;
  const double* phi;
  const int32_t* pairs;
  int64_t npairs;
  double* xi;
  double* M;
  double* ex;
  int32_t status;
  int32_t fail_column;
} ace_system;

int ace_build_batched(ace_ctx* ctx, int nsys, ace_system* systems, int prec, int mode);

/* Batched launch shape (set by the autotuner): x-tile width of the line
 * passes of the split layout (8 or 16), radix order of the FFT plans (0 large
 * radices first, 1 small first), workgroups per compute unit of the
 * persistent launch (1..32), and the layout of the pair stage: 0 the five
 * split passes over packed complex fields in conflict-free rounds, 2
 * real-to-complex half spectra in three phases per round, 3 (the default) the
 * owner layout: the half spectra of all pairs of a grid size stay resident,
 * the forward and z passes run over all of them in one launch each, and each
 * row of W is formed once from the pairs that contain its orbital.  Layouts
 * 2 and 3 apply to every grid size whose half-spectrum plane fits in LDS (all
 * supported sizes).  Layout 3 needs the spectra within the budget of the
 * owner path of ace_build (ACE_OWNER_SPECTRA_MAX bytes, and 60% of the free
 * device memory) and is not used by the persistent launch (mode 1); in those
 * cases layout 2 runs instead.  ACE_E_ARG for other values. */
int ace_set_batched_shape(ace_ctx* ctx, int txv, int plan_variant, int blocks_per_cu, int layout);

/*
 * Learned pair screener (the learned replacement of the screening criterion
 * of Sec. Theory).  It predicts log10 |e_ij| from five pair features and
 * drops the pairs with the smallest predicted |e_ij| while their predicted
 * sum stays within an E_x budget.
 */

/* Features of each pair, float32 [npairs][5]: minimum-image distance of the
 * periodic centroids of |phi_i|^2 and |phi_j|^2 (bohr); the smaller and the
 * larger spread sqrt(dV sum |phi|^2 |r - c|^2) (bohr); log10 of
 * dV sum |phi_i||phi_j|; log10 of dV sum phi_i^2 phi_j^2.  With stride s > 1
 * the two overlap sums run over the grid points whose indices are multiples
 * of s (weight dV s^3; s must divide the grid size).  pairs == NULL means
 * every pair i <= j in row-major triangle order (npairs must then be
 * norb(norb+1)/2).  Cubic boxes. */
int ace_pair_features(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, const int32_t* pairs,
                      int64_t npairs, float* feats, int stride);

/* Exact pair energies e_ij = -(2 - d_ij) dV sum_r phi_i phi_j v_ij (Eq. e:vij)
 * of a pair list, without building W or the ACE operator: the training
 * targets of the screener.  Arguments as for ace_build. */
int ace_pair_energies(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, const int32_t* pairs,
                      int64_t npairs, int kernel, double omega, int prec, double* e);

/* MLP model: float32 device array of ACE_MLP_NMODEL values: W1[64][5], b1[64],
 * W2[64][64], b2[64], w3[64], b3 (ACE_MLP_NPARAM trainable values), then
 * xmean[5], xstd[5], tmean, tstd, xmin[5], xmax[5].  Network: standardize,
 * tanh(W1 x + b1), tanh(W2 h + b2), w3 . h + b3; prediction tmean + tstd *
 * output (the target is log10 |e_ij|). */
#define ACE_MLP_NPARAM 4609
#define ACE_MLP_NMODEL 4631

typedef struct {
  float lr, beta1, beta2, eps; /* Adam */
  int32_t batch;               /* minibatch size */
  int32_t epochs;
  int32_t step0;               /* Adam steps taken before this call */
  uint64_t seed;               /* sample order */
} ace_mlp_hparams;

/* Glorot-uniform weights from a counter-based generator (splitmix64 of seed
 * and index), zero biases, unit standardization. */
int ace_mlp_init(ace_ctx* ctx, float* model, uint64_t seed);
/* Standardization statistics and feature ranges of a training set
 * x [n][5], t [n]. */
int ace_mlp_fit_norm(ace_ctx* ctx, float* model, const float* x, const float* t, int64_t n);
/* Predictions y [n] (log10 |e|); clamp != 0 clips the features to the
 * training ranges first (as the screening does). */
int ace_mlp_forward(ace_ctx* ctx, const float* model, const float* x, int64_t n, int clamp, float* y);
/* Gradient grad [ACE_MLP_NPARAM] of the mean squared error of the
 * standardized targets over all n samples, and the loss (nullable). */
int ace_mlp_grad(ace_ctx* ctx, const float* model, const float* x, const float* t, int64_t n, float* grad,
                 float* loss);
/* Adam training: epochs over the samples in a seeded order, minibatches of
 * hp->batch; adam_m, adam_v [ACE_MLP_NPARAM] persist between calls;
 * loss_curve [epochs] (nullable) receives the sum of the minibatch losses of
 * each epoch.  Deterministic for a given seed. */
int ace_mlp_train(ace_ctx* ctx, float* model, float* adam_m, float* adam_v, const float* x, const float* t, int64_t n,
                  const ace_mlp_hparams* hp, float* loss_curve);

/* Training and inference of the screener on one state array: the model
 * (ACE_MLP_NMODEL floats, standardization set, e.g. by ace_mlp_fit_norm)
 * followed by the Adam moments m and v (ACE_MLP_NPARAM floats each).
 * ace_screener_train: ace_mlp_train on that state (feats [n][5], target [n]
 * log10 |e_ij|).  ace_screener_predict: predictions pred [n] (log10 |e_ij|)
 * with the features clipped to the training ranges, as the screening uses
 * them (ace_mlp_forward with clamp = 1). */
int ace_screener_train(ace_ctx* ctx, const float* feats, const float* target, int64_t n, const ace_mlp_hparams* hp,
                       float* state);
int ace_screener_predict(ace_ctx* ctx, const float* state, const float* feats, int64_t n, float* pred);

/* Learned screening: features and predictions for every pair i <= j, then
 * off-diagonal pairs are dropped in ascending order of predicted |e_ij| while
 * their predicted sum stays <= budget (Hartree); diagonal pairs are kept.
 * If any off-diagonal pair lies outside the model's training range (widened
 * by ood_tol times each span) on the interacting side (closer centroids,
 * larger overlaps, unseen spreads), the overlap rule O_ij >= rho_cut_fallback
 * is used instead and *used_fallback is set; pairs beyond the range on the far
 * side are predicted with clipped features.  stride: the feature stride the
 * model was trained with (see ace_pair_features); the fallback always
 * evaluates O_ij on the full grid.  pairs [capacity][2] sorted by (i, j);
 * *npairs (HOST) as for ace_pairlist. */
int ace_screen_learned(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, const float* model,
                       double budget, double rho_cut_fallback, double ood_tol, int64_t capacity, int32_t* pairs,
                       int64_t* npairs, int* used_fallback, int stride);

/*
 * Both screening rules behind one record (the screening criterion of Sec.
 * Theory, or its learned replacement):
 *   mode 0: the overlap rule at rho_cut (ace_pairlist; overlap nullable);
 *   mode 1: the learned rule under ex_budget (Hartree) with model, ood_tol and
 *           the feature stride, and the overlap rule at rho_cut as the
 *           fallback (ace_screen_learned; overlap must be NULL).
 * pairs, capacity and *npairs (HOST) as for ace_pairlist; *used_fallback
 * (nullable) is set when the learned rule fell back.
 */
typedef struct {
  int32_t mode;
  double rho_cut;
  double ex_budget;
  const float* model;
  double ood_tol;
  int32_t stride;
} ace_screen_spec;

int ace_screen(ace_ctx* ctx, const ace_grid* grid, int norb, const double* phi, const ace_screen_spec* screen,
               int64_t capacity, int32_t* pairs, double* overlap, int64_t* npairs, int* used_fallback);

#ifdef __cplusplus
}
#endif

#endif /* ACE_H */
