// Launchers of the block kernels (blas.hip) and the small-matrix kernels
// (smallmat.hip) used by the solver.
#pragma once

#include "internal.h"

#define UPDATE_NCH 4   // row chunks per work-group in the fused update
#define MAX_RED_BLOCKS 1024  // blocks of a grid reduction at most

template <typename T, typename TX>
struct UpdateArgs {
  int rows, n, ns;
  cplx<T>* Q;                 // [rows][n]  Q_{k-1} in, Q_k out
  const cplx<T>* W;           // [rows][n]  (A + s0) P^(0)
  const double2* alpha;       // n x n FP64
  const double2* rhoinv;      // n x n FP64
  cplx<T>* P;                 // [ns][rows][n] search directions, sorted shift order
                              // (the matrix-core update: [2][ns][rows][n], buffer pp_cur[s])
  cplx<TX>* X;                // solutions; shift s at X + xidx[s]*rows*n
  const cplx<T>* Mx;          // [ns][n][n]
  const cplx<T>* Mp;          // [ns][n][n]
  const cplx<T>* Mxd;         // [ns][n][n] the deferred Mx (matrix-core update)
  SolverFlags* flags;         // read; the matrix-core update also sets upd_done
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
// With SmallParams::pingpong the shifts s >= 1 follow the PP_* modes the small
// step sets; after the last iteration launch_update_drain adds every increment
// still pending (Q, W, alpha, rhoinv and Mp are not used there).
template <typename F>
hipError_t launch_update_mfma(hipStream_t st, const UpdateArgs<F, F>& a, bool two_tiles);
template <typename F>
hipError_t launch_update_drain(hipStream_t st, const UpdateArgs<F, F>& a);
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
};

struct SmallParams {
  int n, ns, max_iter;
  double tol, freeze_tol, breakdown_tol;
  double sigma[BMS_MAX_SHIFTS];  // sorted shifts
  int pingpong;  // shifts s >= 1 take the two-iteration X update (matrix-core update)
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
template <typename T>
hipError_t launch_small_iter(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             cplx<T>* Mx, cplx<T>* Mp, cplx<T>* Mxd);
template <typename T>
hipError_t launch_small_rho_explicit(hipStream_t st, const SmallParams& p, SmallState s,
                                     SolverFlags* fl, cplx<T>* Mp);
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
