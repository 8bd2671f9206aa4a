// Launchers of the block kernels (blas.hip) and the small-matrix kernels
// (smallmat.hip) used by the solver.
#pragma once

#include "internal.h"

#define UPDATE_NCH 4   // row chunks per work-group in the fused update
#define MAX_RED_BLOCKS 1024  // blocks of a grid reduction at most

template <typename T, typename TX>
struct UpdateArgs {
  int rows, n, ns;
  cplx<T>* Q;                 // [rows][n]  Q_{k-1} in, Q_k out (vector update, in place)
  cplx<T>* Qring;             // matrix-core update: [win][rows][n], Q_j in buffer j % win
  const cplx<T>* W;           // [rows][n]  (A + s0) P^(0)
  const double2* alpha;       // n x n FP64
  const double2* rhoinv;      // n x n FP64
  cplx<T>* P;                 // [ns][rows][n] search directions, sorted shift order
  cplx<TX>* X;                // solutions; shift s at X + xidx[s]*rows*n
  const cplx<T>* Mx;          // [ns][n][n]
  const cplx<T>* Mp;          // [ns][n][n]
  const cplx<T>* Wm;          // [ns][2][BMS_MAX_WIN][n][n] window coefficients (matrix cores)
  const double2* wst;         // FP64 window state [2][ns][2][BMS_MAX_WIN][n][n] (drain)
  int win;                    // window length of the shifts s >= 1 (1: every iteration)
  SolverFlags* flags;         // read; the matrix-core update also sets upd_done, upd_stop
  int xidx[BMS_MAX_SHIFTS];
};

// run_if: the kernel does nothing unless *run_if is non-zero (NULL: always runs)
template <typename T>
hipError_t launch_cholqr_gram(hipStream_t st, int rows, int n, const void* Q, const void* W,
                              const double2* alpha, double2* G, double2* partials, int nb,
                              const int* run_if);
template <typename T, typename TX>
hipError_t launch_update(hipStream_t st, const UpdateArgs<T, TX>& a);
// variant 0: both coefficient columns in registers; 1: one at a time
template <typename T, typename TX>
hipError_t launch_update_fast(hipStream_t st, const UpdateArgs<T, TX>& a, int variant);
// update on the matrix cores (update_mfma.hip), for n = 8 and 16, with one or
// two 16-row tiles per wave; F = double or float (the Q step is FP64 in both)
bool update_mfma_supported(int n);
// The shifts s >= 1 are updated in windows of SmallParams::win iterations
// (the small step gathers each window's coefficients, see SmallState::wst);
// after the last iteration launch_update_drain applies every window still
// open (Q, W, alpha, rhoinv, Mx and Mp are not used there).
template <typename F>
hipError_t launch_update_mfma(hipStream_t st, const UpdateArgs<F, F>& a, bool two_tiles);
template <typename F>
hipError_t launch_update_drain(hipStream_t st, const UpdateArgs<F, F>& a);
// longest window the matrix-core update of precision F stages in LDS
template <typename F>
int update_mfma_max_win();
hipError_t launch_resid_norms(hipStream_t st, int rows, int n, const void* B, const void* Y,
                              double2* out, double2* partials, int nb);
hipError_t launch_action(hipStream_t st, int rows, int n, int ns, double a0, const double* alpha,
                         const void* B, const void* X, double2* out, double2* partials, int nb);
// out[p] = sum over b < nb of partials[b * P + p] (in a fixed order), unless
// *skip is non-zero or *run_if is zero (either may be NULL)
hipError_t launch_sum_partials(hipStream_t st, const double2* partials, int nb, int P,
                               double2* out, const int* skip, const int* run_if);

hipError_t launch_resid_block(hipStream_t st, int rows, int n, const void* B, const void* Y,
                              const double* cs, const double* cb, void* R, const int* skip);
hipError_t launch_axpy_cols(hipStream_t st, int rows, int n, void* X, const void* E,
                            const double* cs);
// out = a0 B + sum_s alpha[s] X[s] over blk complex elements (alpha host array)
hipError_t launch_rational_combine(hipStream_t st, size_t blk, int ns, double a0,
                                   const double* alpha, const void* B, const void* X, void* out);
hipError_t launch_gather_col(hipStream_t st, int rows, int n, int col, const void* src, void* dst);
hipError_t launch_scatter_axpy_col(hipStream_t st, int rows, int n, int col, void* X,
                                   const void* e, double scale);
hipError_t launch_flush(hipStream_t st, int rows, int n, int ns, void* X32, void* X64,
                        const int* xmap, const int* skip);
template <typename TO>
hipError_t launch_block_matmul_d(hipStream_t st, int rows, int n, const void* X, const double2* M,
                                 void* Y, const int* skip);

// ---- small n x n FP64 state of the solver (device) ----------------------
// All matrices are row-major n x n double2. Double-buffered entries are
// indexed by iteration parity (flags->iter & 1).
struct SmallState {
  double2* Gb;      // [2][n*n]  G_k = P^H (A+s0) P  (= alpha_k^-1)
  double2* rhob;    // [2][n*n]  rho_k
  double2* alpha;   // [n*n]     alpha_k
  double2* rhoinv;  // [n*n]     rho_k^-1
  double2* delta;   // [n*n]     delta_k (unshifted residual coefficients)
  double2* beta_s;  // [ns][n*n] beta^(s)
  double2* alpha_s; // [ns][n*n] alpha^(s)
  double* norm0;    // [n]       |b_i|
  double2* G4;      // [4][n*n]  P^H W, Q^H W, W^H W, Q^H Q of the iteration
  double2* Gqr;     // [n*n]     output of the V^H V Gram
  double2* tmp;     // [n*n]     scratch
  double* rel_last; // smallest max relative true residual of sigma_0 at a reliable update
  int* counter;     // grid-completion counter of the rho kernel
  int* upd_log;    // [max_iter] block vectors the update of each iteration moves
  // Window state of the deferred shift update, [2][ns][2][BMS_MAX_WIN][n*n]:
  // per slot and shift the X family (Cx, Ex_0, Ex_1, ...) and the P family
  // (Cp, Ep_0, ...) of the open window started at iteration k0, such that after
  // iteration k (j = k - k0 + 1 iterations gathered)
  //   X_{k+1} = X_k0 + P_k0 Cx + sum_{i < j-1} Q_{k0+1+i} Ex_i
  //   P_{k+1} = Q_{k+1} + P_k0 Cp + sum_{i < j-1} Q_{k0+1+i} Ep_i
  double2* wst;
};

struct SmallParams {
  int n, ns, max_iter;
  double tol, freeze_tol, breakdown_tol;
  double sigma[BMS_MAX_SHIFTS];  // sorted shifts
  int win;  // window of the shifts s >= 1 (matrix-core update; 1 = every iteration)
};

// initial QR of B: from G = B^H B, delta_0 = chol(G)^H, out Rinv = delta_0^-1;
// initialises every piece of state and the flags
hipError_t launch_small_init(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             const double2* Gb_in, double2* Rinv_out);
hipError_t launch_small_init_pass2(hipStream_t st, const SmallParams& p, SmallState s,
                                   SolverFlags* fl, const double2* Gb_in, double2* Rinv_out);
// reliable update: from G = R0^H R0 of the true residual, delta_k = chol(G)^H
// and Rinv_out = delta_k^-1 (so that Q_k = R0 Rinv_out)
hipError_t launch_small_reliable(hipStream_t st, const SmallParams& p, SmallState s,
                                 SolverFlags* fl, const double2* Gin, double2* Rinv_out);
// Wm: the window coefficients of every shift in the block precision, for the
// matrix-core update ([ns][2][BMS_MAX_WIN][n*n], the layout of SmallState::wst)
template <typename T>
hipError_t launch_small_iter(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             cplx<T>* Mx, cplx<T>* Mp, cplx<T>* Wm);
template <typename T>
hipError_t launch_small_rho_explicit(hipStream_t st, const SmallParams& p, SmallState s,
                                     SolverFlags* fl, cplx<T>* Mp, cplx<T>* Wm);
// variant 0: vector kernel; 1, 2 and the default: matrix cores, every wave
// streaming its own rows with 4 or 8 steps in flight; 3, 4, 5: matrix cores,
// rows staged through LDS with 1, 2 or 4 chunks in flight (n = 8, 16; other n
// take the vector kernel). nb blocks at most (the size of partials); given the
// compute-unit count, the matrix-core kernels launch one round of resident
// blocks. A second kernel sums the blocks' partials into G4.
template <typename T>
hipError_t launch_gram4(hipStream_t st, int rows, int n, const void* P, const void* Q,
                        const void* W, double2* G4, double2* partials, int nb,
                        const int* skip, int variant = -1, int num_cu = 0);
bool gram4_mfma_supported(int n);
