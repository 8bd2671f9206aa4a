// The n_pf x n_pf FP64 algebra of Algorithm 1 on the device: Cholesky-QR
// factors, alpha_k = (P^H (A+s0) P)^-1, and the two coupled two-term
// recurrences of the shifted systems (Algorithm 1, the shift-recurrence steps):
//   beta^(s)_k  = (1 + (s_s - s_0) alpha_k
//                  + alpha_k rho_{k-1} alpha_{k-1}^-1 (1 - beta^(s)_{k-1}) rho_{k-1}^dag)^-1
//   alpha^(s)_k = beta^(s)_k alpha_k rho_{k-1} alpha_{k-1}^-1 alpha^(s)_{k-1}
// with the shifted residual coefficients delta^(s)_k = rho_k alpha_k^-1 alpha^(s)_k
// (Sec. III, the paragraph after eq. convergence_bound_shifts). alpha_{k-1}^-1
// is the previous Gram G_{k-1}, kept instead of inverting alpha again.
//
// One work-group of 256 threads per shift; matrices live in LDS (n <= 32).
#include "blas.h"

#define NMAX BMS_MAX_RHS
#define NN (NMAX * NMAX)

namespace {

__device__ __forceinline__ double2 cdiv_real(double2 a, double d) { return make_double2(a.x / d, a.y / d); }
__device__ __forceinline__ double2 crecip(double2 a) {
  double m = a.x * a.x + a.y * a.y;
  return make_double2(a.x / m, -a.y / m);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// C = op(A) op(B), op 0 = identity, 1 = conjugate transpose. C must not alias.
// The k loops of these helpers are unrolled so that several LDS loads are in
// flight (their latency, not arithmetic, sets the time of the small step);
// the order of the additions is unchanged.
__device__ void sm_mm(double2* C, const double2* A, int ta, const double2* B, int tb, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    const int a0 = ta ? i : i * n, as = ta ? n : 1;
    const int b0 = tb ? j * n : j, bs = tb ? 1 : n;
    double2 s = make_double2(0, 0);
#pragma unroll 4
    for (int k = 0; k < n; ++k) {
      double2 a = A[a0 + k * as], b = B[b0 + k * bs];
      if (ta) a = cconj(a);
      if (tb) b = cconj(b);
      s = cfma(a, b, s);
    }
    C[e] = s;
  }
  __syncthreads();
}

__device__ void sm_load(double2* dst, const double2* src, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) dst[e] = src[e];
  __syncthreads();
}

__device__ void sm_store(double2* dst, const double2* src, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) dst[e] = src[e];
}

template <typename C>
__device__ void sm_store_t(C* dst, const double2* src, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) dst[e] = from_d<C>(src[e]);
}

__device__ void sm_identity(double2* A, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    A[e] = make_double2(i == j ? 1.0 : 0.0, 0);
  }
  __syncthreads();
}

// G = R^H R with R upper triangular and a real positive diagonal (so that
// {Q, R} = qr(V) has Q = V R^-1 for G = V^H V). Returns 0, or BMS_EBREAKDOWN
// when a pivot is <= tol * trace(G), or BMS_ENAN.
// Right-looking in place: R starts as the upper triangle of G; step j takes
// the square root of the pivot, scales row j, and subtracts row j's outer
// product from the trailing rows. Every entry sees the same operations in
// the same order as the dot-product (left-looking) form, so the factor is
// the same bit for bit, with no one-thread loops between the barriers. Every
// thread reads the pivot (the previous step's barrier made it final) and
// takes the same decision, so a step needs two barriers: one after the row
// is scaled, one after the trailing update (which does not read the pivot;
// the square root replaces it there).
__device__ int sm_chol_upper(double2* R, const double2* G, int n, double tol) {
  __shared__ double trace;
  if (threadIdx.x == 0) {
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += G[i * n + i].x;
    trace = tr;
  }
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
    int i = e / n, l = e - (e / n) * n;
    R[e] = l >= i ? G[e] : make_double2(0, 0);
  }
  __syncthreads();
  const double tr = trace;
  for (int j = 0; j < n; ++j) {
    const double d = R[j * n + j].x;
    if (!(d == d) || !(tr == tr) || !(fabs(tr) < 1e300)) return BMS_ENAN;
    if (!(d > tol * tr)) return BMS_EBREAKDOWN;
    const double djj = sqrt(d);
    for (int l = j + 1 + threadIdx.x; l < n; l += BMS_WG) R[j * n + l] = cdiv_real(R[j * n + l], djj);
    __syncthreads();
    if (threadIdx.x == 0) R[j * n + j] = make_double2(djj, 0);
    const int m = n - j - 1;
    for (int e = threadIdx.x; e < m * m; e += BMS_WG) {
      const int i = j + 1 + e / m, l = j + 1 + (e - (e / m) * m);
      if (l >= i) R[i * n + l] = csub(R[i * n + l], cmul(cconj(R[j * n + i]), R[j * n + l]));
    }
    __syncthreads();
  }
  return 0;
}

// X = R^-1 for upper triangular R, one row of X per step (from the last),
// the columns of a row in parallel
__device__ void sm_triinv_upper(double2* X, const double2* R, int n) {
  for (int i = n - 1; i >= 0; --i) {
    for (int j = threadIdx.x; j < n; j += BMS_WG) {
      if (j < i) {
        X[i * n + j] = make_double2(0, 0);
        continue;
      }
      double2 s = make_double2(i == j ? 1.0 : 0.0, 0);
#pragma unroll 4
      for (int k = i + 1; k <= j; ++k) s = csub(s, cmul(R[i * n + k], X[k * n + j]));
      X[i * n + j] = cdiv_real(s, R[i * n + i].x);
    }
    __syncthreads();
  }
}

// Ainv = A^-1 by Gauss-Jordan elimination with partial pivoting; A is
// destroyed. Returns 0 or BMS_ENAN (singular / non-finite).
// Column c: the pivot search, a row swap when the pivot is off the diagonal,
// then in one phase the pivot row scaled and the multipliers (column c) read,
// then the elimination, each phase ended by a barrier. The columns of A up
// to c are not updated in step c: nothing reads them afterwards (the pivot
// search and the multipliers use the columns beyond), so Ainv is the same
// bit for bit as with every column updated.
__device__ int sm_inv_general(double2* Ainv, double2* A, int n) {
  __shared__ int status;
  __shared__ int piv;
  __shared__ double2 fac[NMAX];
  sm_identity(Ainv, n);
  if (threadIdx.x == 0) status = 0;
  for (int c = 0; c < n; ++c) {
    // pivot: the first row r >= c of largest |A[r][c]| (the diagonal's own
    // value decides a NaN there; NaN below it is never taken), by a
    // reduction over the first wave
    if (threadIdx.x < 64) {
      const int r = c + (int)threadIdx.x;
      double v = r < n ? cabs2(A[r * n + c]) : -1.0;
      if (r > c && !(v == v)) v = -1.0;
      int idx = r;
      for (int off = 32; off > 0; off >>= 1) {
        const double v2 = __shfl_down(v, off);
        const int i2 = __shfl_down(idx, off);
        if (v2 > v || (v2 == v && i2 < idx)) {
          v = v2;
          idx = i2;
        }
      }
      if (threadIdx.x == 0) {
        if (!(v > 0) || !(v < 1e300)) status = BMS_ENAN;
        piv = idx;
      }
    }
    __syncthreads();
    if (status) return status;
    int p = piv;
    if (p != c) {
      for (int k = threadIdx.x; k < n; k += BMS_WG) {
        double2 t = A[p * n + k];
        A[p * n + k] = A[c * n + k];
        A[c * n + k] = t;
        t = Ainv[p * n + k];
        Ainv[p * n + k] = Ainv[c * n + k];
        Ainv[c * n + k] = t;
      }
      __syncthreads();
    }
    // the pivot itself is not written in this phase (column c of A is not
    // updated), so every thread reads it
    const double2 inv = crecip(A[c * n + c]);
    for (int k = threadIdx.x; k < n; k += BMS_WG) {
      if (k > c) A[c * n + k] = cmul(A[c * n + k], inv);
      Ainv[c * n + k] = cmul(Ainv[c * n + k], inv);
    }
    for (int r = threadIdx.x; r < n; r += BMS_WG) fac[r] = A[r * n + c];
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
      int r = e / n, k = e - (e / n) * n;
      if (r == c) continue;
      double2 f = fac[r];
      if (k > c) A[e] = csub(A[e], cmul(f, A[c * n + k]));
      Ainv[e] = csub(Ainv[e], cmul(f, Ainv[c * n + k]));
    }
    __syncthreads();
  }
  return 0;
}

__device__ void raise_error(SolverFlags* fl, int code) {
  if (threadIdx.x == 0) {
    atomicCAS(&fl->error, 0, code);
    fl->stop = 1;
    fl->halted = 1;
  }
}

// Initial thin QR of B (pass 0) or its re-orthogonalisation (pass 1):
// from G = V^H V, R = chol(G)^H; pass 0 sets delta_0 = R, pass 1 sets
// delta_0 = R delta_0. Writes R^-1 for Q = V R^-1 and (re)initialises state.
__global__ __launch_bounds__(BMS_WG) void k_small_init(SmallParams p, SmallState s,
                                                       SolverFlags* fl, const double2* Gin,
                                                       double2* Rinv_out, int pass) {
  __shared__ double2 L0[NN], L1[NN], L2[NN];
  const int n = p.n;
  if (pass == 0 && threadIdx.x == 0) {
    fl->stop = 0;
    fl->halted = 0;
    fl->rel_restart = 0;
    fl->diverged = 0;
    fl->rel_stall = 0;
    *s.rel_last = 1e300;
    fl->error = 0;
    fl->iter = 0;
    fl->need_explicit = 0;
    fl->upd_done = -1;
    fl->rel_count = 0;
    *s.counter = 0;
  }
  if (pass == 0)
    for (int i = threadIdx.x; i < BMS_MAX_SHIFTS; i += BMS_WG) {
      fl->active[i] = i < p.ns;
      fl->conv[i] = 0;
      fl->res[i] = 1.0;
      fl->win_j[0][i] = fl->win_j[1][i] = 0;
      fl->win_flush[0][i] = fl->win_flush[1][i] = 1;
    }
  if (pass == 0 && threadIdx.x == 0) fl->upd_stop = 0;
  sm_load(L0, Gin, n);
  int st = sm_chol_upper(L1, L0, n, p.breakdown_tol);
  if (st) {
    raise_error(fl, st);
    return;
  }
  sm_triinv_upper(L2, L1, n);
  sm_store(Rinv_out, L2, n);
  if (pass == 0) {
    sm_store(s.delta, L1, n);
    __syncthreads();
    sm_load(L0, L1, n);  // delta_0 in L0
  } else {
    sm_load(L2, s.delta, n);
    sm_mm(L0, L1, 0, L2, 0, n);  // delta_0 = R delta_0
    sm_store(s.delta, L0, n);
  }
  // rho_0 = delta_0 in the "previous" slot of iteration 0; alpha_0 = 1 so G_0 = 1
  sm_store(s.rhob + n * n, L0, n);
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    s.Gb[n * n + e] = make_double2(i == j ? 1.0 : 0.0, 0);
    for (int q = 0; q < p.ns; ++q) {
      s.beta_s[(size_t)q * n * n + e] = make_double2(i == j ? 1.0 : 0.0, 0);
      s.alpha_s[(size_t)q * n * n + e] = make_double2(i == j ? 1.0 : 0.0, 0);
    }
  }
  for (int i = threadIdx.x; i < n; i += BMS_WG) {
    double c = 0;
    for (int k = 0; k < n; ++k) c += cabs2(L0[k * n + i]);
    s.norm0[i] = sqrt(c);
  }
}

// Reliable update of the unshifted system: the true FP64 residual R0 =
// B - (A + s0) X^(0) replaces the iterated one, R0 = Q delta with the
// Cholesky-QR factor delta = chol(R0^H R0)^H.
__global__ __launch_bounds__(BMS_WG) void k_small_reliable(SmallParams p, SmallState s,
                                                           SolverFlags* fl, const double2* Gin,
                                                           double2* Rinv_out) {
  __shared__ double2 L0[NN], L1[NN], L2[NN];
  const int n = p.n;
  if (fl->stop) {
    if (threadIdx.x == 0) {
      fl->rel_skip = 1;
      fl->rel_restart = 0;
    }
    return;
  }
  if (threadIdx.x == 0) fl->rel_count += 1;
  sm_load(L0, Gin, n);
  int st = sm_chol_upper(L1, L0, n, p.breakdown_tol);
  if (st) {
    // columns of the true residual too unequal to factor: keep the iterated one
    if (threadIdx.x == 0) {
      fl->rel_skip = 1;
      fl->rel_restart = 0;
    }
    if (st == BMS_ENAN) raise_error(fl, st);
    return;
  }
  // How far the true residual is from the iterated one (column norms of the
  // new and the old delta). A large jump (the iterated residual had run far
  // below the rounding drift, e.g. past Krylov exhaustion) leaves P^(0)
  // inconsistent with the new Q: with one shift the search restarts from
  // P^(0) = Q; with several the multi-shift iteration stops here and the
  // per-shift defect correction takes over.
  // It also watches the true residual itself: growth beyond 2x its smallest
  // value so far, or four reliable updates in a row without a 1% gain, means
  // the FP32 iteration diverges or stalls (e.g. after Krylov exhaustion on a
  // small lattice); the loop then stops softly and the caller falls back to
  // FP64.
  __shared__ double jump, trel;
  if (threadIdx.x == 0) {
    double m = 0, mt = 0;
    for (int i = 0; i < n; ++i) {
      double ct = 0, ci = 0;
      for (int k = 0; k < n; ++k) {
        ct += cabs2(L1[k * n + i]);
        ci += cabs2(s.delta[k * n + i]);
      }
      double r = sqrt(ct) / fmax(sqrt(ci), 1e-300);
      m = r > m ? r : m;
      double t = sqrt(ct) / s.norm0[i];
      mt = t > mt ? t : mt;
    }
    jump = m;
    trel = mt;
  }
  __syncthreads();
  sm_triinv_upper(L2, L1, n);
  sm_store(Rinv_out, L2, n);
  sm_store(s.delta, L1, n);
  if (threadIdx.x == 0) {
    fl->rel_skip = 0;
    const bool big = jump > 10.0;
    fl->rel_restart = big && p.ns == 1;
    if (big && p.ns > 1) fl->stop = 1;
    const double best = *s.rel_last;
    if (trel < 0.99 * best) {
      *s.rel_last = trel;
      fl->rel_stall = 0;
    } else {
      fl->rel_stall += 1;
    }
    if (!(trel <= 2.0 * best) || fl->rel_stall >= 4) {
      fl->diverged = 1;
      fl->stop = 1;
    }
  }
}

// Completion of one iteration's small step: count this block's arrival and
// whether its shift met tol; the last block to arrive stops the solve when
// all did, logs the update's traffic and work and advances the iteration
// counter. The
// update moves 3 block vectors for the Q step, 4 for each shift it applies
// (P and X read and written) and, once, the ring buffers of the longest
// window applied that are not in registers (Q_{k0+1} .. Q_{k-1}).
__device__ void finish_shift(const SmallParams& p, const SmallState& s, SolverFlags* fl,
                             int done) {
  if (threadIdx.x == 0) {
    __threadfence();
    int v = atomicAdd(s.counter, 1 + (done << 16)) + 1 + (done << 16);
    if ((v & 0xffff) == p.ns) {
      __threadfence();
      if ((v >> 16) == p.ns || fl->error) fl->stop = 1;
      const int ws = (fl->iter + 1) & 1;
      int units = 3, qx = 0, prods = 0;
      for (int i = 0; i < p.ns; ++i) {
        const int j = fl->win_j[ws][i];
        if (j > 0 && (fl->win_flush[ws][i] || fl->stop)) {
          units += 4;
          prods += 2 * j;
          qx = j - 2 > qx ? j - 2 : qx;
        }
      }
      units += qx;
      // block vectors moved, and the n x n right products of the applied
      // windows above bit 16 (the Q step's two are added by the host)
      if (s.upd_log && fl->iter < p.max_iter) s.upd_log[fl->iter] = units | (prods << 16);
      fl->need_explicit = 0;
      fl->iter = fl->iter + 1;
      atomicExch(s.counter, 0);
    }
  }
}

// C = C0 + A B (C0 = NULL: C = A B) for a stack of rows / n matrices A (rows x
// n, global memory) and one n x n matrix B (LDS); C also goes to Ct in the
// block precision.
template <typename T>
__device__ void win_mm(double2* C, const double2* C0, const double2* A, const double2* B,
                       int rows, int n, cplx<T>* Ct) {
  for (int e = threadIdx.x; e < rows * n; e += BMS_WG) {
    int r = e / n, j = e - (e / n) * n;
    double2 acc = C0 ? C0[e] : make_double2(0, 0);
#pragma unroll 4
    for (int k = 0; k < n; ++k) acc = cfma(A[r * n + k], B[k * n + j], acc);
    C[e] = acc;
    Ct[e] = from_d<cplx<T>>(acc);
  }
}

// One iteration into shift q's update window (layout in SmallState::wst).
// The window read is slot `cur` (what the previous small step wrote), the
// one written slot cur ^ 1; a window that the last update applied (its flush
// flag) starts again. With j0 iterations gathered, the new step's Mx, Mp give
//   X family: [Cx, Ex_i] += [Cp, Ep_i] Mx, then Ex_{j0-1} = Mx (Q_k enters X)
//   P family: [Cp, Ep_i]  = [Cp, Ep_i] Mp, then Ep_{j0-1} = Mp
// (a fresh window: Cx = Mx, Cp = Mp). The update applies the window when it
// holds `len` iterations (1 for sigma_0, whose P feeds the operator every
// iteration) or the shift converged.
template <typename T>
__device__ void win_step(const SmallParams& p, const SmallState& s, SolverFlags* fl,
                         cplx<T>* Wm, const double2* Mx, const double2* Mp, int q, int cur,
                         bool conv_now) {
  const int n = p.n, nn = n * n;
  const int len = q == 0 ? 1 : p.win;
  const int ws = cur ^ 1;
  const int j0 = (fl->win_flush[cur][q] || fl->win_j[cur][q] == 0) ? 0 : fl->win_j[cur][q];
  const size_t fam = (size_t)BMS_MAX_WIN * nn;
  const double2* ox = s.wst + (size_t)(cur * p.ns + q) * 2 * fam;
  const double2* op = ox + fam;
  double2* nx = s.wst + (size_t)(ws * p.ns + q) * 2 * fam;
  double2* np = nx + fam;
  cplx<T>* tx = Wm + (size_t)q * 2 * fam;
  cplx<T>* tp = tx + fam;
  if (j0 > 0) {
    win_mm<T>(nx, ox, op, Mx, j0 * n, n, tx);
    win_mm<T>(np, nullptr, op, Mp, j0 * n, n, tp);
  }
  for (int e = threadIdx.x; e < nn; e += BMS_WG) {
    nx[(size_t)j0 * nn + e] = Mx[e];
    tx[(size_t)j0 * nn + e] = from_d<cplx<T>>(Mx[e]);
    np[(size_t)j0 * nn + e] = Mp[e];
    tp[(size_t)j0 * nn + e] = from_d<cplx<T>>(Mp[e]);
  }
  if (threadIdx.x == 0) {
    fl->win_j[ws][q] = j0 + 1;
    fl->win_flush[ws][q] = (j0 + 1 >= len) || conv_now;
  }
  __syncthreads();
}

// Everything that needs rho_k (in R, LDS): rho_k^-1, delta_k, the shift's
// residual coefficients delta^(s)_k = rho_k alpha_k^-1 alpha^(s)_k, its update
// matrix Mp and its convergence. Gk = G_k = alpha_k^-1 (LDS copy).
template <typename T>
__device__ void rho_part(const SmallParams& p, const SmallState& s, SolverFlags* fl, cplx<T>* Mp,
                         cplx<T>* Wm, const double2* R, const double2* Gk, double2* T0,
                         double2* T1, double2* D, int q, int cur) {
  __shared__ double colmax;
  const int n = p.n, nn = n * n;
  if (q == 0) {
    sm_triinv_upper(T0, R, n);
    sm_store(s.rhoinv, T0, n);
    sm_store(s.rhob + cur * nn, R, n);
    sm_load(T1, s.delta, n);
    sm_mm(D, R, 0, T1, 0, n);  // delta_k = rho_k delta_{k-1}
    sm_store(s.delta, D, n);
    for (int e = threadIdx.x; e < nn; e += BMS_WG) {
      int i = e / n, j = e - (e / n) * n;
      Mp[e] = from_d<cplx<T>>(cconj(R[j * n + i]));  // rho_k^dag
    }
  } else {
    sm_mm(T0, R, 0, Gk, 0, n);  // rho_k alpha_k^-1
    sm_load(T1, s.alpha_s + (size_t)q * nn, n);
    sm_mm(D, T0, 0, T1, 0, n);  // delta^(s)_k
    sm_load(T1, s.beta_s + (size_t)q * nn, n);
    sm_mm(T0, T1, 0, R, 1, n);  // beta^(s)_k rho_k^dag
    sm_store_t(Mp + (size_t)q * nn, T0, n);
  }
  // relative residual estimate: max_i |delta^(s) e_i| / |b_i| (a thread per
  // column, then the maximum)
  __shared__ double colr[NMAX];
  for (int i = threadIdx.x; i < n; i += BMS_WG) {
    double c = 0;
#pragma unroll 4
    for (int k = 0; k < n; ++k) c += cabs2(D[k * n + i]);
    double r = sqrt(c) / s.norm0[i];
    if (!(r == r)) r = 1e300;
    colr[i] = r;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int i = 0; i < n; ++i) m = colr[i] > m ? colr[i] : m;
    colmax = m;
  }
  __syncthreads();
  double r = colmax;
  if (threadIdx.x == 0) {
    fl->res[q] = r;
    if (q > 0) fl->conv[q] = r < p.freeze_tol;
    if (r >= 1e300) {
      atomicCAS(&fl->error, 0, BMS_ENAN);
      fl->halted = 1;
    }
  }
  // the step into the shift's update window: Mx = alpha^(s)_k, Mp (FP64, T0)
  if (q == 0)
    for (int e = threadIdx.x; e < nn; e += BMS_WG) {
      int i = e / n, j = e - (e / n) * n;
      T0[e] = cconj(R[j * n + i]);
    }
  sm_load(T1, s.alpha_s + (size_t)q * nn, n);
  win_step<T>(p, s, fl, Wm, T1, T0, q, cur, q > 0 && r < p.freeze_tol);
  finish_shift(p, s, fl, r < p.tol);
}

// One iteration's n x n work, after G4 = [P^H W, Q^H W, W^H W, Q^H Q]:
//   alpha_k = (P^H W)^-1; beta^(s)_k, alpha^(s)_k (Algorithm 1, shift recurrences);
//   V^H V from the expansion, rho_k = chol(V^H V)^H; then rho_part.
// If that Cholesky loses its pivot, need_explicit is raised and the explicit
// Gram of V plus k_small_rho_explicit finish the iteration instead.
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_small_iter(SmallParams p, SmallState s,
                                                       SolverFlags* fl, cplx<T>* Mx,
                                                       cplx<T>* Mp, cplx<T>* Wm) {
  __shared__ double2 Gk[NN], A[NN], R[NN], T0[NN], T1[NN], T2[NN], T3[NN];
  const int n = p.n, nn = n * n;
  const int q = blockIdx.x;
  if (fl->stop || fl->iter >= p.max_iter) {
    if (q == 0 && threadIdx.x == 0) {
      fl->stop = 1;
      fl->halted = 1;
    }
    return;
  }
  const int cur = fl->iter & 1, prev = cur ^ 1;
  if (q > 0 && (fl->conv[q] || !fl->active[q])) {
    // frozen: its last window was applied when it converged
    if (threadIdx.x == 0) {
      fl->active[q] = 0;
      fl->win_j[prev][q] = 0;
      fl->win_flush[prev][q] = 1;
    }
    finish_shift(p, s, fl, 1);
    return;
  }
  sm_load(Gk, s.G4, n);
  int st = sm_chol_upper(T0, Gk, n, 0.0);
  if (st) {
    if (q == 0) raise_error(fl, st);
    return;
  }
  sm_triinv_upper(T1, T0, n);
  sm_mm(A, T1, 0, T1, 1, n);  // alpha_k = R^-1 R^-H = G_k^-1
  if (q == 0) {
    sm_store(s.alpha, A, n);
    sm_store(s.Gb + cur * nn, Gk, n);
    sm_load(T1, s.delta, n);
    sm_mm(T0, A, 0, T1, 0, n);  // alpha^(0)_k = alpha_k delta_{k-1}
    sm_store(s.alpha_s, T0, n);
    sm_store_t(Mx, T0, n);
  } else {
    const double dsig = p.sigma[q] - p.sigma[0];
    sm_load(T1, s.rhob + prev * nn, n);
    sm_mm(T2, A, 0, T1, 0, n);  // alpha_k rho_{k-1}
    sm_load(T1, s.Gb + prev * nn, n);
    sm_mm(T0, T2, 0, T1, 0, n);  // t = alpha_k rho_{k-1} alpha_{k-1}^-1
    const double2* bold = s.beta_s + (size_t)q * nn;
    for (int e = threadIdx.x; e < nn; e += BMS_WG) {
      int i = e / n, j = e - (e / n) * n;
      T1[e] = csub(make_double2(i == j ? 1.0 : 0.0, 0), bold[e]);
    }
    __syncthreads();
    sm_mm(T2, T0, 0, T1, 0, n);  // t (1 - beta_{k-1})
    sm_load(T1, s.rhob + prev * nn, n);
    sm_mm(T3, T2, 0, T1, 1, n);  // ... rho_{k-1}^dag
    for (int e = threadIdx.x; e < nn; e += BMS_WG) {
      int i = e / n, j = e - (e / n) * n;
      double2 v = cadd(T3[e], cscale(A[e], dsig));
      if (i == j) v.x += 1.0;
      T3[e] = v;
    }
    __syncthreads();
    st = sm_inv_general(T2, T3, n);  // beta^(s)_k
    if (st) {
      raise_error(fl, BMS_ENAN);
      return;
    }
    sm_mm(T3, T2, 0, T0, 0, n);  // beta t
    sm_load(T1, s.alpha_s + (size_t)q * nn, n);
    sm_mm(T0, T3, 0, T1, 0, n);  // alpha^(s)_k = beta t alpha^(s)_{k-1}
    sm_store(s.beta_s + (size_t)q * nn, T2, n);
    sm_store(s.alpha_s + (size_t)q * nn, T0, n);
    sm_store_t(Mx + (size_t)q * nn, T0, n);
    __syncthreads();
  }
  // V^H V = QQ - QW A - A^H QW^H + A^H WW A
  sm_load(T1, s.G4 + nn, n);       // Q^H W
  sm_mm(T0, T1, 0, A, 0, n);       // QW A
  sm_load(T2, s.G4 + 2 * nn, n);   // W^H W
  sm_mm(T3, T2, 0, A, 0, n);       // WW A
  sm_mm(T2, A, 1, T3, 0, n);       // A^H WW A
  const double2* QQ = s.G4 + 3 * nn;
  for (int e = threadIdx.x; e < nn; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    // (QW A)^H = A^H QW^H
    T3[e] = cadd(csub(csub(QQ[e], T0[e]), cconj(T0[j * n + i])), T2[e]);
  }
  __syncthreads();
  // The expansion cancels when V is small next to Q (|V|^2 / |Q|^2 ~ rounding
  // relative to the result); then the explicit Gram of V is used instead.
  __shared__ int cancel;
  if (threadIdx.x == 0) {
    double tv = 0, tq = 0;
    for (int i = 0; i < n; ++i) {
      tv += T3[i * n + i].x;
      tq += QQ[i * n + i].x;
    }
    cancel = !(tv >= 1e-4 * tq);
  }
  __syncthreads();
  st = cancel ? BMS_EBREAKDOWN : sm_chol_upper(R, T3, n, p.breakdown_tol);
  if (st) {
    if (st == BMS_ENAN) {
      if (q == 0) raise_error(fl, st);
    } else if (q == 0 && threadIdx.x == 0) {
      fl->need_explicit = 1;  // the explicit Gram finishes this iteration
    }
    return;
  }
  rho_part<T>(p, s, fl, Mp, Wm, R, Gk, T0, T1, T2, q, cur);
}

// Fallback when the expansion lost accuracy: rho_k from the explicit V^H V.
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_small_rho_explicit(SmallParams p, SmallState s,
                                                               SolverFlags* fl, cplx<T>* Mp,
                                                               cplx<T>* Wm) {
  __shared__ double2 Gk[NN], R[NN], T0[NN], T1[NN], T2[NN];
  const int n = p.n;
  const int q = blockIdx.x;
  if (fl->stop || !fl->need_explicit) return;
  if (q > 0 && !fl->active[q]) return;  // already counted by k_small_iter
  const int cur = fl->iter & 1;
  sm_load(T0, s.Gqr, n);
  int st = sm_chol_upper(R, T0, n, p.breakdown_tol);
  if (st) {
    if (q == 0) raise_error(fl, st);
    return;
  }
  sm_load(Gk, s.G4, n);
  rho_part<T>(p, s, fl, Mp, Wm, R, Gk, T0, T1, T2, q, cur);
}

}  // namespace

hipError_t launch_small_init(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             const double2* Gb_in, double2* Rinv_out) {
  k_small_init<<<1, BMS_WG, 0, st>>>(p, s, fl, Gb_in, Rinv_out, 0);
  return hipGetLastError();
}

hipError_t launch_small_init_pass2(hipStream_t st, const SmallParams& p, SmallState s,
                                   SolverFlags* fl, const double2* Gb_in, double2* Rinv_out) {
  k_small_init<<<1, BMS_WG, 0, st>>>(p, s, fl, Gb_in, Rinv_out, 1);
  return hipGetLastError();
}

hipError_t launch_small_reliable(hipStream_t st, const SmallParams& p, SmallState s,
                                 SolverFlags* fl, const double2* Gin, double2* Rinv_out) {
  k_small_reliable<<<1, BMS_WG, 0, st>>>(p, s, fl, Gin, Rinv_out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_iter(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                             cplx<T>* Mx, cplx<T>* Mp, cplx<T>* Wm) {
  k_small_iter<T><<<p.ns, BMS_WG, 0, st>>>(p, s, fl, Mx, Mp, Wm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_rho_explicit(hipStream_t st, const SmallParams& p, SmallState s,
                                     SolverFlags* fl, cplx<T>* Mp, cplx<T>* Wm) {
  k_small_rho_explicit<T><<<p.ns, BMS_WG, 0, st>>>(p, s, fl, Mp, Wm);
  return hipGetLastError();
}

#define INST_SMALL(T, C)                                                                    \
  template hipError_t launch_small_iter<T>(hipStream_t, const SmallParams&, SmallState,     \
                                           SolverFlags*, C*, C*, C*);                       \
  template hipError_t launch_small_rho_explicit<T>(hipStream_t, const SmallParams&,         \
                                                   SmallState, SolverFlags*, C*, C*);
INST_SMALL(double, double2)
INST_SMALL(float, float2)
