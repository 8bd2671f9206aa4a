// Tall-skinny block kernels of the solver: Gram matrices X^H Y, the
// Cholesky-QR Gram, the fused per-iteration block update of every shift,
// residual norms and the action reduction.
//
// A block vector is `rows` rows of n complex numbers (row = (site, colour)),
// contiguous, right-hand side fastest. Threads map to (row, column) so that a
// work-group's loads of a run of rows are one contiguous, coalesced span; the
// row mixing of "block times n x n matrix" goes through LDS.
#include "blas.h"

namespace {

// ---- helpers ----------------------------------------------------------------

struct RowRange {
  int r0, r1;
};

__device__ __forceinline__ RowRange block_rows(int rows, int per_block) {
  RowRange r;
  r.r0 = blockIdx.x * per_block;
  r.r1 = min(rows, r.r0 + per_block);
  return r;
}

// Deterministic completion of a grid-wide sum: every block has written its
// P-element partial; the block that finishes last adds them in block order.
__device__ void last_block_sum(double2* __restrict__ partials, double2* __restrict__ out, int P,
                               int* __restrict__ counter) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) is_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  for (int p = threadIdx.x; p < P; p += BMS_WG) {
    double2 s = make_double2(0, 0);
    for (int b = 0; b < (int)gridDim.x; ++b) s = cadd(s, partials[(size_t)b * P + p]);
    out[p] = s;
  }
  if (threadIdx.x == 0) atomicExch(counter, 0);
}

// Accumulate sum_r conj(xs[r][i]) ys[r][j] over the nr rows staged in LDS.
// Pair mapping: P = n*n pairs over pth = min(256, P) threads, nrg = 256/pth
// row groups, up to 4 pairs per thread (n <= 32).
struct PairMap {
  int P, pth, nrg, npp, rg, p0;
};

__device__ __forceinline__ PairMap pair_map(int n) {
  PairMap m;
  m.P = n * n;
  m.pth = m.P < BMS_WG ? m.P : BMS_WG;
  m.nrg = BMS_WG / m.pth;
  m.npp = (m.P + m.pth - 1) / m.pth;
  m.rg = threadIdx.x / m.pth;
  m.p0 = threadIdx.x - m.rg * m.pth;
  return m;
}

__device__ __forceinline__ void pair_accumulate(const PairMap& m, int n, int nr,
                                                const double2* xs, const double2* ys,
                                                double2 acc[4]) {
  if (m.rg >= m.nrg) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (q >= m.npp) break;
    int p = m.p0 + q * m.pth;
    if (p >= m.P) break;
    int i = p / n, j = p - (p / n) * n;
    double2 a = acc[q];
    for (int r = m.rg; r < nr; r += m.nrg) a = cjfma(xs[r * n + i], ys[r * n + j], a);
    acc[q] = a;
  }
}

__device__ __forceinline__ void pair_finish(const PairMap& m, double2 acc[4], double2* red,
                                            double2* __restrict__ partials, double2* __restrict__ G,
                                            int* __restrict__ counter) {
  // red holds nrg*P <= 1024 entries
  if (m.rg < m.nrg) {
    for (int q = 0; q < m.npp; ++q) {
      int p = m.p0 + q * m.pth;
      if (p < m.P) red[m.rg * m.P + p] = acc[q];
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < m.P; p += BMS_WG) {
    double2 s = make_double2(0, 0);
    for (int g = 0; g < m.nrg; ++g) s = cadd(s, red[g * m.P + p]);
    partials[(size_t)blockIdx.x * m.P + p] = s;
  }
  last_block_sum(partials, G, m.P, counter);
}

// ---- kernels ----------------------------------------------------------------

__global__ void k_fill_zero(uint4* p, size_t n16) {
  size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x;
  if (i < n16) p[i] = make_uint4(0, 0, 0, 0);
}

// G = X^H Y (FP64 accumulation)
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_gram(int rows, int n, int per_block,
                                                 const cplx<T>* __restrict__ X,
                                                 const cplx<T>* __restrict__ Y,
                                                 double2* __restrict__ G,
                                                 double2* __restrict__ partials,
                                                 int* __restrict__ counter,
                                                 const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double2 xs[BMS_WG], ys[BMS_WG];
  __shared__ double2 red[4 * BMS_WG];
  RowRange rr = block_rows(rows, per_block);
  int C = BMS_WG / n;
  PairMap m = pair_map(n);
  double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  for (int r0 = rr.r0; r0 < rr.r1; r0 += C) {
    int nr = min(C, rr.r1 - r0);
    int t = threadIdx.x;
    if (t < nr * n) {
      xs[t] = to_d(X[(size_t)r0 * n + t]);
      ys[t] = to_d(Y[(size_t)r0 * n + t]);
    }
    __syncthreads();
    pair_accumulate(m, n, nr, xs, ys, acc);
    __syncthreads();
  }
  pair_finish(m, acc, red, partials, G, counter);
}

// G = V^H V with V = Q - W alpha computed on the fly (alpha FP64, n x n)
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_cholqr_gram(int rows, int n, int per_block,
                                                        const cplx<T>* __restrict__ Q,
                                                        const cplx<T>* __restrict__ W,
                                                        const double2* __restrict__ alpha,
                                                        double2* __restrict__ G,
                                                        double2* __restrict__ partials,
                                                        int* __restrict__ counter,
                                                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double2 ws[BMS_WG], vs[BMS_WG];
  __shared__ double2 red[4 * BMS_WG];
  RowRange rr = block_rows(rows, per_block);
  int C = BMS_WG / n;
  PairMap m = pair_map(n);
  double2 acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
  int t = threadIdx.x;
  int lr = t / n, j = t - (t / n) * n;
  for (int r0 = rr.r0; r0 < rr.r1; r0 += C) {
    int nr = min(C, rr.r1 - r0);
    if (t < nr * n) ws[t] = to_d(W[(size_t)r0 * n + t]);
    __syncthreads();
    if (t < nr * n) {
      double2 v = to_d(Q[(size_t)r0 * n + t]);
      double2 wa = make_double2(0, 0);
      for (int k = 0; k < n; ++k) wa = cfma(ws[lr * n + k], alpha[k * n + j], wa);
      vs[t] = csub(v, wa);
    }
    __syncthreads();
    pair_accumulate(m, n, nr, vs, vs, acc);
    __syncthreads();
  }
  pair_finish(m, acc, red, partials, G, counter);
}

// Y = X M for a rows x n block and an n x n FP64 matrix
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_block_matmul(int rows, int n,
                                                         const cplx<T>* __restrict__ X,
                                                         const double2* __restrict__ M,
                                                         cplx<T>* __restrict__ Y) {
  __shared__ double2 xs[BMS_WG];
  int C = BMS_WG / n;
  int r0 = blockIdx.x * C;
  int nr = min(C, rows - r0);
  int t = threadIdx.x;
  if (t < nr * n) xs[t] = to_d(X[(size_t)r0 * n + t]);
  __syncthreads();
  if (t < nr * n) {
    int lr = t / n, j = t - lr * n;
    double2 a = make_double2(0, 0);
    for (int k = 0; k < n; ++k) a = cfma(xs[lr * n + k], M[k * n + j], a);
    Y[(size_t)r0 * n + t] = from_d<cplx<T>>(a);
  }
}

// Fused block update of one iteration (Algorithm 1, steps 6-9 and 12-13):
//   Q_k   = (Q_{k-1} - W alpha_k) rho_k^-1          (W = (A + s0) P^(0)_{k-1})
//   X^(s) += P^(s) Mx[s]                              (Mx[0] = alpha_k delta_{k-1},
//                                                      Mx[s] = alpha^(s)_k)
//   P^(s) = Q_k + P^(s) Mp[s]                         (Mp[0] = rho_k^dag,
//                                                      Mp[s] = beta^(s)_k rho_k^dag)
// for every active shift, reading Q and W once. Each block owns NCH chunks of
// C = 256/n rows; Q_k of its rows stays in LDS for all shifts.
template <typename T, typename TX>
__global__ __launch_bounds__(BMS_WG) void k_update(UpdateArgs<T, TX> a) {
  using C_ = cplx<T>;
  using CX = cplx<TX>;
  const SolverFlags* fl = a.flags;
  if (fl->halted) return;
  constexpr int NCH = UPDATE_NCH;
  __shared__ double2 ws[BMS_WG];
  __shared__ double2 vs[BMS_WG];
  __shared__ C_ qs[NCH * BMS_WG];
  __shared__ C_ ps[BMS_WG];
  const int n = a.n;
  const int C = BMS_WG / n;
  const int t = threadIdx.x;
  const int lr = t / n, j = t - (t / n) * n;
  const bool live = t < C * n;
  const int rbase = blockIdx.x * C * NCH;
  // Q path in FP64
  for (int ch = 0; ch < NCH; ++ch) {
    int r0 = rbase + ch * C;
    if (r0 >= a.rows) break;
    int nr = min(C, a.rows - r0);
    bool act = live && lr < nr;
    size_t o = (size_t)r0 * n + t;
    if (act) ws[t] = to_d(a.W[o]);
    __syncthreads();
    if (act) {
      double2 wa = make_double2(0, 0);
      for (int k = 0; k < n; ++k) wa = cfma(ws[lr * n + k], a.alpha[k * n + j], wa);
      vs[t] = csub(to_d(a.Q[o]), wa);
    }
    __syncthreads();
    if (act) {
      double2 q = make_double2(0, 0);
      for (int k = 0; k < n; ++k) q = cfma(vs[lr * n + k], a.rhoinv[k * n + j], q);
      C_ qt = from_d<C_>(q);
      a.Q[o] = qt;
      qs[ch * BMS_WG + t] = qt;
    }
    __syncthreads();
  }
  // shifts
  for (int s = 0; s < a.ns; ++s) {
    if (!fl->active[s]) continue;
    C_* P = a.P + (size_t)s * a.rows * n;
    CX* X = a.X + (size_t)a.xidx[s] * a.rows * n;
    const C_* Mx = a.Mx + (size_t)s * n * n;
    const C_* Mp = a.Mp + (size_t)s * n * n;
    for (int ch = 0; ch < NCH; ++ch) {
      int r0 = rbase + ch * C;
      if (r0 >= a.rows) break;
      int nr = min(C, a.rows - r0);
      bool act = live && lr < nr;
      size_t o = (size_t)r0 * n + t;
      if (act) ps[t] = P[o];
      __syncthreads();
      if (act) {
        C_ dx = czero<C_>();
        C_ np = qs[ch * BMS_WG + t];
        for (int k = 0; k < n; ++k) {
          C_ pk = ps[lr * n + k];
          dx = cfma(pk, Mx[k * n + j], dx);
          np = cfma(pk, Mp[k * n + j], np);
        }
        CX xo = X[o];
        X[o] = cmk<CX>(xo.x + (TX)dx.x, xo.y + (TX)dx.y);
        P[o] = np;
      }
      __syncthreads();
    }
  }
}

// res[s*n + i] partial sums of |B[r][i] - Y[r][i]|^2 and |B[r][i]|^2 for a
// batch of vectors Y (FP64); reduced with last_block_sum into out (2n values).
__global__ __launch_bounds__(BMS_WG) void k_resid_norms(int rows, int n, int per_block,
                                                        const double2* __restrict__ B,
                                                        const double2* __restrict__ Y,
                                                        double2* __restrict__ out,
                                                        double2* __restrict__ partials,
                                                        int* __restrict__ counter) {
  __shared__ double2 red[BMS_WG];
  RowRange rr = block_rows(rows, per_block);
  int groups = BMS_WG / n;
  int t = threadIdx.x;
  int g = t / n, j = t - (t / n) * n;
  double2 acc = make_double2(0, 0);  // x: |b - y|^2, y: |b|^2
  if (g < groups) {
    for (int r = rr.r0 + g; r < rr.r1; r += groups) {
      double2 b = B[(size_t)r * n + j];
      double2 d = csub(b, Y[(size_t)r * n + j]);
      acc.x += d.x * d.x + d.y * d.y;
      acc.y += b.x * b.x + b.y * b.y;
    }
  }
  red[t] = acc;
  __syncthreads();
  for (int p = t; p < n; p += BMS_WG) {
    double2 s = make_double2(0, 0);
    for (int q = 0; q < groups; ++q) s = cadd(s, red[q * n + p]);
    partials[(size_t)blockIdx.x * n + p] = s;
  }
  last_block_sum(partials, out, n, counter);
}

// S_i = Re sum_r conj(B[r][i]) (a0 B[r][i] + sum_s alpha[s] X[s][r][i])
__global__ __launch_bounds__(BMS_WG) void k_action(int rows, int n, int per_block, int ns,
                                                   double a0, const double* __restrict__ alpha,
                                                   const double2* __restrict__ B,
                                                   const double2* __restrict__ X,
                                                   double2* __restrict__ out,
                                                   double2* __restrict__ partials,
                                                   int* __restrict__ counter) {
  __shared__ double2 red[BMS_WG];
  RowRange rr = block_rows(rows, per_block);
  int groups = BMS_WG / n;
  int t = threadIdx.x;
  int g = t / n, j = t - (t / n) * n;
  double acc = 0;
  if (g < groups) {
    for (int r = rr.r0 + g; r < rr.r1; r += groups) {
      size_t o = (size_t)r * n + j;
      double2 b = B[o];
      double2 v = cscale(b, a0);
      for (int s = 0; s < ns; ++s) v = cadd(v, cscale(X[(size_t)s * rows * n + o], alpha[s]));
      acc += b.x * v.x + b.y * v.y;
    }
  }
  red[t] = make_double2(acc, 0);
  __syncthreads();
  for (int p = t; p < n; p += BMS_WG) {
    double2 s = make_double2(0, 0);
    for (int q = 0; q < groups; ++q) s = cadd(s, red[q * n + p]);
    partials[(size_t)blockIdx.x * n + p] = s;
  }
  last_block_sum(partials, out, n, counter);
}

}  // namespace

int gram_blocks(int rows, int n) {
  // enough blocks to fill the chip, each with at least a few chunks of rows
  int C = BMS_WG / n;
  int per = 4 * C;
  int nb = (rows + per - 1) / per;
  return nb < 1 ? 1 : (nb > 1024 ? 1024 : nb);
}

static int rows_per_block(int rows, int nb) { return (rows + nb - 1) / nb; }

hipError_t launch_fill_zero(hipStream_t st, void* p, size_t bytes) {
  size_t n16 = bytes / 16;
  if (n16) k_fill_zero<<<(unsigned)((n16 + BMS_WG - 1) / BMS_WG), BMS_WG, 0, st>>>((uint4*)p, n16);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram(hipStream_t st, int rows, int n, const void* X, const void* Y, double2* G,
                       double2* partials, int* counter, int nb, const int* skip) {
  k_gram<T><<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const cplx<T>*)X,
                                   (const cplx<T>*)Y, G, partials, counter, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cholqr_gram(hipStream_t st, int rows, int n, const void* Q, const void* W,
                              const double2* alpha, double2* G, double2* partials, int* counter,
                              int nb, const int* skip) {
  k_cholqr_gram<T><<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const cplx<T>*)Q,
                                          (const cplx<T>*)W, alpha, G, partials, counter, skip);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_block_matmul(hipStream_t st, int rows, int n, const void* X, const double2* M,
                               void* Y) {
  int C = BMS_WG / n;
  k_block_matmul<T><<<(rows + C - 1) / C, BMS_WG, 0, st>>>(rows, n, (const cplx<T>*)X, M,
                                                           (cplx<T>*)Y);
  return hipGetLastError();
}

template <typename T, typename TX>
hipError_t launch_update(hipStream_t st, const UpdateArgs<T, TX>& a) {
  int per = (BMS_WG / a.n) * UPDATE_NCH;
  k_update<T, TX><<<(a.rows + per - 1) / per, BMS_WG, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_resid_norms(hipStream_t st, int rows, int n, const void* B, const void* Y,
                              double2* out, double2* partials, int* counter, int nb) {
  k_resid_norms<<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const double2*)B,
                                       (const double2*)Y, out, partials, counter);
  return hipGetLastError();
}

hipError_t launch_action(hipStream_t st, int rows, int n, int ns, double a0, const double* alpha,
                         const void* B, const void* X, double2* out, double2* partials,
                         int* counter, int nb) {
  k_action<<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), ns, a0, alpha,
                                  (const double2*)B, (const double2*)X, out, partials, counter);
  return hipGetLastError();
}

#define INST(T)                                                                                \
  template hipError_t launch_gram<T>(hipStream_t, int, int, const void*, const void*, double2*, \
                                     double2*, int*, int, const int*);                          \
  template hipError_t launch_cholqr_gram<T>(hipStream_t, int, int, const void*, const void*,    \
                                            const double2*, double2*, double2*, int*, int,      \
                                            const int*);                                        \
  template hipError_t launch_block_matmul<T>(hipStream_t, int, int, const void*, const double2*, \
                                             void*);
INST(float)
INST(double)
template hipError_t launch_update<double, double>(hipStream_t, const UpdateArgs<double, double>&);
template hipError_t launch_update<float, float>(hipStream_t, const UpdateArgs<float, float>&);
