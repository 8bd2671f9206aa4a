// The n_pf x n_pf FP64 algebra of Algorithm 1 on the device: Cholesky-QR
// factors, alpha_k = (P^H (A+s0) P)^-1, and the two coupled two-term
// recurrences of the shifted systems (Algorithm 1, lines 10-11):
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
__device__ void sm_mm(double2* C, const double2* A, int ta, const double2* B, int tb, int n) {
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    double2 s = make_double2(0, 0);
    for (int k = 0; k < n; ++k) {
      double2 a = ta ? cconj(A[k * n + i]) : A[i * n + k];
      double2 b = tb ? cconj(B[j * n + k]) : B[k * n + j];
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
__device__ int sm_chol_upper(double2* R, const double2* G, int n, double tol) {
  __shared__ int status;
  __shared__ double trace;
  if (threadIdx.x == 0) {
    status = 0;
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += G[i * n + i].x;
    trace = tr;
  }
  for (int e = threadIdx.x; e < n * n; e += BMS_WG) R[e] = make_double2(0, 0);
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = G[j * n + j].x;
      for (int k = 0; k < j; ++k) d -= cabs2(R[k * n + j]);
      if (!(d == d) || !(trace == trace) || !(fabs(trace) < 1e300)) status = BMS_ENAN;
      else if (!(d > tol * trace)) status = BMS_EBREAKDOWN;
      R[j * n + j] = make_double2(status ? 1.0 : sqrt(d), 0);
    }
    __syncthreads();
    if (status) return status;
    double djj = R[j * n + j].x;
    for (int i = j + 1 + threadIdx.x; i < n; i += BMS_WG) {
      double2 s = G[j * n + i];
      for (int k = 0; k < j; ++k) s = csub(s, cmul(cconj(R[k * n + j]), R[k * n + i]));
      R[j * n + i] = cdiv_real(s, djj);
    }
    __syncthreads();
  }
  return 0;
}

// X = R^-1 for upper triangular R (one thread per column)
__device__ void sm_triinv_upper(double2* X, const double2* R, int n) {
  for (int j = threadIdx.x; j < n; j += BMS_WG) {
    for (int i = n - 1; i >= 0; --i) {
      if (i > j) {
        X[i * n + j] = make_double2(0, 0);
        continue;
      }
      double2 s = make_double2(i == j ? 1.0 : 0.0, 0);
      for (int k = i + 1; k <= j; ++k) s = csub(s, cmul(R[i * n + k], X[k * n + j]));
      X[i * n + j] = cdiv_real(s, R[i * n + i].x);
    }
  }
  __syncthreads();
}

// Ainv = A^-1 by Gauss-Jordan elimination with partial pivoting; A is
// destroyed. Returns 0 or BMS_ENAN (singular / non-finite).
__device__ int sm_inv_general(double2* Ainv, double2* A, int n) {
  __shared__ int status;
  __shared__ int piv;
  __shared__ double2 fac[NMAX];
  sm_identity(Ainv, n);
  if (threadIdx.x == 0) status = 0;
  for (int c = 0; c < n; ++c) {
    if (threadIdx.x == 0) {
      int p = c;
      double best = cabs2(A[c * n + c]);
      for (int r = c + 1; r < n; ++r) {
        double v = cabs2(A[r * n + c]);
        if (v > best) {
          best = v;
          p = r;
        }
      }
      if (!(best > 0) || !(best < 1e300)) status = BMS_ENAN;
      piv = p;
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
    double2 inv = crecip(A[c * n + c]);
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += BMS_WG) {
      A[c * n + k] = cmul(A[c * n + k], inv);
      Ainv[c * n + k] = cmul(Ainv[c * n + k], inv);
    }
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += BMS_WG) fac[r] = A[r * n + c];
    __syncthreads();
    for (int e = threadIdx.x; e < n * n; e += BMS_WG) {
      int r = e / n, k = e - (e / n) * n;
      if (r == c) continue;
      double2 f = fac[r];
      A[e] = csub(A[e], cmul(f, A[c * n + k]));
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
    fl->error = 0;
    fl->iter = 0;
    *s.counter = 0;
  }
  if (pass == 0)
    for (int i = threadIdx.x; i < p.ns; i += BMS_WG) {
      fl->active[i] = 1;
      fl->conv[i] = 0;
      fl->res[i] = 1.0;
    }
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

// Per iteration, after G_k = P^H (A + s0) P: alpha_k and every active shift's
// beta^(s)_k, alpha^(s)_k. Block s handles shift s (sorted; s = 0 is s0).
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_small_alpha(SmallParams p, SmallState s,
                                                        SolverFlags* fl, cplx<T>* Mx) {
  __shared__ double2 L0[NN], L1[NN], L2[NN], L3[NN], L4[NN];
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
  if (q > 0 && fl->conv[q]) {
    if (threadIdx.x == 0) fl->active[q] = 0;
    if (q > 0) return;
  }
  if (q > 0 && !fl->active[q]) return;
  sm_load(L0, s.Ggram, n);
  int st = sm_chol_upper(L1, L0, n, 0.0);
  if (st) {
    if (q == 0) raise_error(fl, st == BMS_EBREAKDOWN ? BMS_EBREAKDOWN : BMS_ENAN);
    return;
  }
  sm_triinv_upper(L2, L1, n);
  sm_mm(L3, L2, 0, L2, 1, n);  // alpha = R^-1 R^-H = G^-1
  if (q == 0) {
    sm_store(s.alpha, L3, n);
    sm_store(s.Gb + cur * nn, L0, n);
    sm_load(L1, s.delta, n);
    sm_mm(L2, L3, 0, L1, 0, n);  // alpha^(0)_k = alpha_k delta_{k-1}
    sm_store(s.alpha_s, L2, n);
    sm_store_t(Mx, L2, n);
    return;
  }
  const double dsig = p.sigma[q] - p.sigma[0];
  sm_load(L1, s.rhob + prev * nn, n);
  sm_mm(L2, L3, 0, L1, 0, n);  // alpha_k rho_{k-1}
  sm_load(L1, s.Gb + prev * nn, n);
  sm_mm(L0, L2, 0, L1, 0, n);  // t = alpha_k rho_{k-1} alpha_{k-1}^-1
  const double2* bold = s.beta_s + (size_t)q * nn;
  for (int e = threadIdx.x; e < nn; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    L1[e] = csub(make_double2(i == j ? 1.0 : 0.0, 0), bold[e]);
  }
  __syncthreads();
  sm_mm(L2, L0, 0, L1, 0, n);  // t (1 - beta_{k-1})
  sm_load(L1, s.rhob + prev * nn, n);
  sm_mm(L4, L2, 0, L1, 1, n);  // ... rho_{k-1}^dag
  for (int e = threadIdx.x; e < nn; e += BMS_WG) {
    int i = e / n, j = e - (e / n) * n;
    double2 v = cadd(L4[e], cscale(L3[e], dsig));
    if (i == j) v.x += 1.0;
    L4[e] = v;
  }
  __syncthreads();
  st = sm_inv_general(L2, L4, n);  // beta^(s)_k
  if (st) {
    raise_error(fl, BMS_ENAN);
    return;
  }
  sm_mm(L4, L2, 0, L0, 0, n);  // beta t
  sm_load(L1, s.alpha_s + (size_t)q * nn, n);
  sm_mm(L0, L4, 0, L1, 0, n);  // alpha^(s)_k = beta t alpha^(s)_{k-1}
  sm_store(s.beta_s + (size_t)q * nn, L2, n);
  sm_store(s.alpha_s + (size_t)q * nn, L0, n);
  sm_store_t(Mx + (size_t)q * nn, L0, n);
}

// Per iteration, after G = V^H V with V = Q_{k-1} - W alpha_k: rho_k, rho_k^-1,
// delta_k, the update matrices Mp[s] = beta^(s)_k rho_k^dag, and convergence.
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_small_rho(SmallParams p, SmallState s,
                                                      SolverFlags* fl, cplx<T>* Mp) {
  __shared__ double2 L0[NN], L1[NN], L2[NN], L3[NN];
  __shared__ double colmax;
  const int n = p.n, nn = n * n;
  const int q = blockIdx.x;
  if (fl->stop) return;
  const int cur = fl->iter & 1;
  const bool act = (q == 0) || fl->active[q];
  int done = 1;
  if (act) {
    sm_load(L0, s.Gqr, n);
    int st = sm_chol_upper(L1, L0, n, p.breakdown_tol);
    if (st) {
      if (q == 0) raise_error(fl, st);
      return;
    }
    if (q == 0) {
      sm_triinv_upper(L2, L1, n);
      sm_store(s.rhoinv, L2, n);
      sm_store(s.rhob + cur * nn, L1, n);
      sm_load(L0, s.delta, n);
      sm_mm(L3, L1, 0, L0, 0, n);  // delta_k = rho_k delta_{k-1}
      sm_store(s.delta, L3, n);
      for (int e = threadIdx.x; e < nn; e += BMS_WG) {
        int i = e / n, j = e - (e / n) * n;
        Mp[e] = from_d<cplx<T>>(cconj(L1[j * n + i]));  // rho_k^dag
      }
    } else {
      sm_load(L0, s.Gb + cur * nn, n);
      sm_mm(L2, L1, 0, L0, 0, n);  // rho_k alpha_k^-1
      sm_load(L0, s.alpha_s + (size_t)q * nn, n);
      sm_mm(L3, L2, 0, L0, 0, n);  // delta^(s)_k
      sm_load(L0, s.beta_s + (size_t)q * nn, n);
      sm_mm(L2, L0, 0, L1, 1, n);  // beta^(s)_k rho_k^dag
      sm_store_t(Mp + (size_t)q * nn, L2, n);
    }
    // relative residual estimate: max_i |delta^(s) e_i| / |b_i|
    if (threadIdx.x == 0) {
      double m = 0;
      for (int i = 0; i < n; ++i) {
        double c = 0;
        for (int k = 0; k < n; ++k) c += cabs2(L3[k * n + i]);
        double r = sqrt(c) / s.norm0[i];
        if (!(r == r)) r = 1e300;
        m = r > m ? r : m;
      }
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
    done = r < p.tol;
  }
  // grid completion: count arrivals (low 16 bits) and converged shifts (high)
  if (threadIdx.x == 0) {
    __threadfence();
    int v = atomicAdd(s.counter, 1 + (done << 16)) + 1 + (done << 16);
    if ((v & 0xffff) == p.ns) {
      __threadfence();
      if ((v >> 16) == p.ns || fl->error) fl->stop = 1;
      int na = 1;
      for (int i = 1; i < p.ns; ++i) na += fl->active[i];
      if (s.nact_log && fl->iter < p.max_iter) s.nact_log[fl->iter] = na;
      fl->iter = fl->iter + 1;
      atomicExch(s.counter, 0);
    }
  }
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

template <typename T>
hipError_t launch_small_alpha(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                              cplx<T>* Mx) {
  k_small_alpha<T><<<p.ns, BMS_WG, 0, st>>>(p, s, fl, Mx);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_small_rho(hipStream_t st, const SmallParams& p, SmallState s, SolverFlags* fl,
                            cplx<T>* Mp) {
  k_small_rho<T><<<p.ns, BMS_WG, 0, st>>>(p, s, fl, Mp);
  return hipGetLastError();
}

template hipError_t launch_small_alpha<double>(hipStream_t, const SmallParams&, SmallState,
                                               SolverFlags*, double2*);
template hipError_t launch_small_alpha<float>(hipStream_t, const SmallParams&, SmallState,
                                              SolverFlags*, float2*);
template hipError_t launch_small_rho<double>(hipStream_t, const SmallParams&, SmallState,
                                             SolverFlags*, double2*);
template hipError_t launch_small_rho<float>(hipStream_t, const SmallParams&, SmallState,
                                            SolverFlags*, float2*);
