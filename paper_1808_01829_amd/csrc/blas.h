// Launchers of the block kernels (blas.hip) and the small-matrix kernels
// (smallmat.hip) used by the solver.
#pragma once

#include "internal.h"

#define UPDATE_NCH 4  // row chunks per work-group in the fused update

template <typename T, typename TX>
struct UpdateArgs {
  int rows, n, ns;
  cplx<T>* Q;                 // [rows][n]  Q_{k-1} in, Q_k out
  const cplx<T>* W;           // [rows][n]  (A + s0) P^(0)
  const double2* alpha;       // n x n FP64
  const double2* rhoinv;      // n x n FP64
  cplx<T>* P;                 // [ns][rows][n] search directions, sorted shift order
  cplx<TX>* X;                // solutions; shift s at X + xidx[s]*rows*n
  const cplx<T>* Mx;          // [ns][n][n]
  const cplx<T>* Mp;          // [ns][n][n]
  const SolverFlags* flags;
  int xidx[BMS_MAX_SHIFTS];
};

template <typename T>
hipError_t launch_cholqr_gram(hipStream_t st, int rows, int n, const void* Q, const void* W,
                              const double2* alpha, double2* G, double2* partials, int* counter,
                              int nb, const int* skip);
template <typename T, typename TX>
hipError_t launch_update(hipStream_t st, const UpdateArgs<T, TX>& a);
hipError_t launch_resid_norms(hipStream_t st, int rows, int n, const void* B, const void* Y,
                              double2* out, double2* partials, int* counter, int nb);
hipError_t launch_action(hipStream_t st, int rows, int n, int ns, double a0, const double* alpha,
                         const void* B, const void* X, double2* out, double2* partials,
                         int* counter, int nb);

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
  double2* Ggram;   // [n*n]     output of the P^H W Gram
  double2* Gqr;     // [n*n]     output of the V^H V Gram
  double2* tmp;     // [n*n]     scratch
  int* counter;     // grid-completion counter of the rho kernel
  int* nact_log;    // [max_iter] active shifts in each completed iteration
};

struct SmallParams {
  int n, ns, max_iter;
  double tol, freeze_tol, breakdown_tol;
  double sigma[BMS_MAX_SHIFTS];  // sorted shifts
};

// initial QR of B: from G = B^H B, delta_0 = chol(G)^H, out Rinv = delta_0^-1;
// initialises every piece of state and the flags
hipError_t launch_small_init(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             const double2* Gb_in, double2* Rinv_out);
hipError_t launch_small_init_pass2(hipStream_t st, const SmallParams& p, SmallState s,
                                   SolverFlags* fl, const double2* Gb_in, double2* Rinv_out);
template <typename T>
hipError_t launch_small_alpha(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                              cplx<T>* Mx);
template <typename T>
hipError_t launch_small_rho(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                            cplx<T>* Mp);
