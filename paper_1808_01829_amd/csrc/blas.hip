// Tall-skinny block kernels of the solver: Gram matrices X^H Y, the
// Cholesky-QR Gram, the fused per-iteration block update of every shift,
// residual norms and the action reduction.
//
// A block vector is `rows` rows of n complex numbers (row = (site, colour)),
// contiguous, right-hand side fastest. Threads map to (row, column) so that a
// work-group's loads of a run of rows are one contiguous, coalesced span; the
// row mixing of "block times n x n matrix" goes through LDS.
#include <algorithm>
#include <type_traits>

#include "blas.h"

// return a failed HIP status to the caller
#define HIP_RET(x)                    \
  do {                                \
    hipError_t e_ = (x);              \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

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

// this block's P entries of the Gram into partials[blockIdx.x * P + p]
__device__ __forceinline__ void pair_finish(const PairMap& m, double2 acc[4], double2* red,
                                            double2* __restrict__ partials) {
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
                                                 double2* __restrict__ partials,
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
  pair_finish(m, acc, red, partials);
}

// G = V^H V with V = Q - W alpha computed on the fly (alpha FP64, n x n)
template <typename T>
__global__ __launch_bounds__(BMS_WG) void k_cholqr_gram(int rows, int n, int per_block,
                                                        const cplx<T>* __restrict__ Q,
                                                        const cplx<T>* __restrict__ W,
                                                        const double2* __restrict__ alpha,
                                                        double2* __restrict__ partials,
                                                        const int* __restrict__ run_if) {
  if (run_if && !*run_if) return;
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
  pair_finish(m, acc, red, partials);
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
// batch of vectors Y (FP64), this block's n entries into partials.
__global__ __launch_bounds__(BMS_WG) void k_resid_norms(int rows, int n, int per_block,
                                                        const double2* __restrict__ B,
                                                        const double2* __restrict__ Y,
                                                        double2* __restrict__ partials) {
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
}

// S_i = Re sum_r conj(B[r][i]) (a0 B[r][i] + sum_s alpha[s] X[s][r][i])
__global__ __launch_bounds__(BMS_WG) void k_action(int rows, int n, int per_block, int ns,
                                                   double a0, const double* __restrict__ alpha,
                                                   const double2* __restrict__ B,
                                                   const double2* __restrict__ X,
                                                   double2* __restrict__ partials) {
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
}

// Final sum of a grid reduction, a kernel of its own: out[p] = sum over b < nb
// of partials[b * P + p]. SUM_TPE threads share an entry, each adding a
// contiguous run of the partials in order (SUM_RB loads in flight), and the
// runs are then added in order: the result depends only on nb. (Finishing
// the sum inside the producing kernel would need a device-scope fence and an
// atomic per block, which on this many-XCD part costs tens of microseconds at
// a few hundred blocks.)
constexpr int SUM_TPE = 16;
constexpr int SUM_EPB = BMS_WG / SUM_TPE;  // entries per block
constexpr int SUM_RB = 8;

__global__ __launch_bounds__(BMS_WG) void k_sum_partials(const double2* __restrict__ partials,
                                                         int nb, int P, double2* __restrict__ out,
                                                         const int* __restrict__ skip,
                                                         const int* __restrict__ run_if) {
  if ((skip && *skip) || (run_if && !*run_if)) return;
  __shared__ double2 red[SUM_TPE][SUM_EPB];
  const int le = threadIdx.x % SUM_EPB, part = threadIdx.x / SUM_EPB;
  const int p = blockIdx.x * SUM_EPB + le;
  const int per = (nb + SUM_TPE - 1) / SUM_TPE;
  const int b0 = part * per, b1 = min(nb, b0 + per);
  double2 s = make_double2(0, 0);
  if (p < P) {
    int b = b0;
    for (; b + SUM_RB <= b1; b += SUM_RB) {
      double2 v[SUM_RB];
#pragma unroll
      for (int k = 0; k < SUM_RB; ++k) v[k] = partials[(size_t)(b + k) * P + p];
#pragma unroll
      for (int k = 0; k < SUM_RB; ++k) s = cadd(s, v[k]);
    }
    for (; b < b1; ++b) s = cadd(s, partials[(size_t)b * P + p]);
  }
  red[part][le] = s;
  __syncthreads();
  if (part == 0 && p < P) {
    double2 t = red[0][le];
    for (int q = 1; q < SUM_TPE; ++q) t = cadd(t, red[q][le]);
    out[p] = t;
  }
}

}  // namespace

hipError_t launch_sum_partials(hipStream_t st, const double2* partials, int nb, int P,
                               double2* out, const int* skip, const int* run_if) {
  k_sum_partials<<<(P + SUM_EPB - 1) / SUM_EPB, BMS_WG, 0, st>>>(partials, nb, P, out, skip,
                                                                 run_if);
  return hipGetLastError();
}

int gram_blocks(int rows, int n, int num_cu) {
  // enough blocks to fill the chip, each with at least a few chunks of rows;
  // on a large block the count is a whole number of rounds of three
  // resident blocks per compute unit (no partly filled last round)
  int C = BMS_WG / n;
  int per = 4 * C;
  int nb = (rows + per - 1) / per;
  int cap = num_cu > 0 ? 3 * num_cu : MAX_RED_BLOCKS;
  if (cap > MAX_RED_BLOCKS) cap = MAX_RED_BLOCKS;
  return nb < 1 ? 1 : (nb > cap ? cap : nb);
}

static int rows_per_block(int rows, int nb) { return (rows + nb - 1) / nb; }

namespace {
__global__ __launch_bounds__(BMS_WG) void k_copy_if(uint4* __restrict__ dst,
                                                    const uint4* __restrict__ src, size_t n16,
                                                    const int* __restrict__ run_if) {
  if (!*run_if) return;
  for (size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x; i < n16;
       i += (size_t)gridDim.x * BMS_WG)
    dst[i] = src[i];
}
}  // namespace

hipError_t launch_copy_if(hipStream_t st, void* dst, const void* src, size_t bytes,
                          const int* run_if) {
  size_t n16 = bytes / 16;
  unsigned blocks = (unsigned)std::min<size_t>((n16 + BMS_WG - 1) / BMS_WG, 8192);
  if (n16) k_copy_if<<<blocks, BMS_WG, 0, st>>>((uint4*)dst, (const uint4*)src, n16, run_if);
  return hipGetLastError();
}

hipError_t launch_fill_zero(hipStream_t st, void* p, size_t bytes) {
  size_t n16 = bytes / 16;
  if (n16) k_fill_zero<<<(unsigned)((n16 + BMS_WG - 1) / BMS_WG), BMS_WG, 0, st>>>((uint4*)p, n16);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gram(hipStream_t st, int rows, int n, const void* X, const void* Y, double2* G,
                       double2* partials, int nb, const int* skip) {
  k_gram<T><<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const cplx<T>*)X,
                                   (const cplx<T>*)Y, partials, skip);
  return launch_sum_partials(st, partials, nb, n * n, G, skip, nullptr);
}

template <typename T>
hipError_t launch_cholqr_gram(hipStream_t st, int rows, int n, const void* Q, const void* W,
                              const double2* alpha, double2* G, double2* partials, int nb,
                              const int* run_if) {
  k_cholqr_gram<T><<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const cplx<T>*)Q,
                                          (const cplx<T>*)W, alpha, partials, run_if);
  return launch_sum_partials(st, partials, nb, n * n, G, nullptr, run_if);
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
                              double2* out, double2* partials, int nb) {
  k_resid_norms<<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), (const double2*)B,
                                       (const double2*)Y, partials);
  return launch_sum_partials(st, partials, nb, n, out, nullptr, nullptr);
}

hipError_t launch_action(hipStream_t st, int rows, int n, int ns, double a0, const double* alpha,
                         const void* B, const void* X, double2* out, double2* partials,
                         int nb) {
  k_action<<<nb, BMS_WG, 0, st>>>(rows, n, rows_per_block(rows, nb), ns, a0, alpha,
                                  (const double2*)B, (const double2*)X, partials);
  return launch_sum_partials(st, partials, nb, n, out, nullptr, nullptr);
}

#define INST(T)                                                                                \
  template hipError_t launch_gram<T>(hipStream_t, int, int, const void*, const void*, double2*, \
                                     double2*, int, const int*);                                \
  template hipError_t launch_cholqr_gram<T>(hipStream_t, int, int, const void*, const void*,    \
                                            const double2*, double2*, double2*, int,            \
                                            const int*);                                        \
  template hipError_t launch_block_matmul<T>(hipStream_t, int, int, const void*, const double2*, \
                                             void*);
INST(float)
INST(double)
template hipError_t launch_update<double, double>(hipStream_t, const UpdateArgs<double, double>&);
template hipError_t launch_update<float, float>(hipStream_t, const UpdateArgs<float, float>&);

// ---- one-pass Grams of an iteration -----------------------------------------
// G4 = [P^H W, Q^H W, W^H W, Q^H Q] (FP64, 4 n x n blocks) in one pass over
// the rows, so that V^H V for V = Q - W alpha follows from the expansion
//   V^H V = Q^H Q - (Q^H W) alpha - alpha^H (Q^H W)^H + alpha^H (W^H W) alpha
// without a second pass. Register blocking: a thread owns a TB x TB tile of
// one Gram; W^H W and Q^H Q are Hermitian and only their upper tiles are
// computed (the reduction mirrors them).
namespace {

struct TileId {
  int g, ti, tj;
};

__device__ __forceinline__ TileId decode_tile(int r, int nt) {
  const int full = nt * nt, half = nt * (nt + 1) / 2;
  TileId d;
  if (r < full) d.g = 0;
  else if ((r -= full) < full) d.g = 1;
  else if ((r -= full) < half) d.g = 2;
  else {
    r -= half;
    d.g = 3;
  }
  if (d.g < 2) {
    d.ti = r / nt;
    d.tj = r - d.ti * nt;
  } else {  // r-th upper tile in row-major order
    d.ti = 0;
    while (r >= nt - d.ti) {
      r -= nt - d.ti;
      ++d.ti;
    }
    d.tj = d.ti + r;
  }
  return d;
}

template <typename T, int TB>
__global__ __launch_bounds__(BMS_WG) void k_gram4(int rows, int n, int per_block,
                                                  const cplx<T>* __restrict__ P,
                                                  const cplx<T>* __restrict__ Q,
                                                  const cplx<T>* __restrict__ W,
                                                                                                    double2* __restrict__ partials,
                                                  const int* __restrict__ skip) {
  using C_ = cplx<T>;
  if (skip && *skip) return;
  // LDS: the staged rows during the sweep, then the row-group reduction
  constexpr int RED = TB == 4 ? 2048 : 1024;  // double2 entries
  // staged rows padded to n+1 entries and the three arrays staggered, so that
  // the rows and arrays a wave reads fall in different LDS banks
  constexpr int STAGE_BYTES = 3 * (2 * BMS_WG + 2) * (int)sizeof(C_);
  constexpr int SM_BYTES = RED * 16 > STAGE_BYTES ? RED * 16 : STAGE_BYTES;
  __shared__ __align__(16) unsigned char smem[SM_BYTES];
  const int C = BMS_WG / n;
  const int RS = n > 1 ? n + 1 : 1;
  const int AS = C * RS + 1;
  C_* ps = (C_*)smem;
  C_* qs = ps + AS;
  C_* wsm = qs + AS;
  const int nt = n / TB;
  const int tiles = 2 * nt * nt + nt * (nt + 1);
  const int nrg = BMS_WG / tiles;
  const int t = threadIdx.x;
  const int rg = t / tiles, tl = t - (t / tiles) * tiles;
  const TileId id = decode_tile(tl, nt);
  const C_* xs = (id.g == 0) ? ps : ((id.g == 2) ? wsm : qs);
  const C_* ys = (id.g == 3) ? qs : wsm;
  RowRange rr = block_rows(rows, per_block);
  const int lw = (t / n) * RS + (t - (t / n) * n);  // this thread's staging slot
  double2 acc[TB][TB];
#pragma unroll
  for (int a = 0; a < TB; ++a)
#pragma unroll
    for (int b = 0; b < TB; ++b) acc[a][b] = make_double2(0, 0);
  // register prefetch of the next chunk while the current one is reduced
  C_ np_ = czero<C_>(), nq_ = czero<C_>(), nw_ = czero<C_>();
  if (rr.r0 < rr.r1 && t < min(C, rr.r1 - rr.r0) * n) {
    size_t o = (size_t)rr.r0 * n + t;
    np_ = P[o];
    nq_ = Q[o];
    nw_ = W[o];
  }
  for (int r0 = rr.r0; r0 < rr.r1; r0 += C) {
    int nr = min(C, rr.r1 - r0);
    if (t < nr * n) {
      ps[lw] = np_;
      qs[lw] = nq_;
      wsm[lw] = nw_;
    }
    __syncthreads();
    int r1 = r0 + C;
    if (r1 < rr.r1 && t < min(C, rr.r1 - r1) * n) {
      size_t o = (size_t)r1 * n + t;
      np_ = P[o];
      nq_ = Q[o];
      nw_ = W[o];
    }
    if (rg < nrg) {
      for (int r = rg; r < nr; r += nrg) {
        double2 xv[TB], yv[TB];
#pragma unroll
        for (int a = 0; a < TB; ++a) {
          xv[a] = to_d(xs[r * RS + id.ti * TB + a]);
          yv[a] = to_d(ys[r * RS + id.tj * TB + a]);
        }
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) acc[a][b] = cjfma(xv[a], yv[b], acc[a][b]);
      }
    }
    __syncthreads();
  }
  const int nn = n * n;
  double2* part = partials + (size_t)blockIdx.x * 4 * nn;
  double2* red = (double2*)smem;
  if (TB == 4 && nrg == 1) {
    // one row group: write the tile straight from registers
    if (rg < nrg) {
#pragma unroll
      for (int a = 0; a < TB; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
          int i = id.ti * TB + a, j = id.tj * TB + b;
          part[id.g * nn + i * n + j] = acc[a][b];
          if (id.g >= 2 && id.ti != id.tj) part[id.g * nn + j * n + i] = cconj(acc[a][b]);
        }
    }
  } else {
    if (TB == 4) {
      // few row groups: accumulate them one after another in tiles*16 entries
      for (int g = 0; g < nrg; ++g) {
        if (rg == g) {
#pragma unroll
          for (int a = 0; a < TB; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) {
              int e = tl * TB * TB + a * TB + b;
              red[e] = g == 0 ? acc[a][b] : cadd(red[e], acc[a][b]);
            }
        }
        __syncthreads();
      }
    } else {
      if (rg < nrg) {
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
          for (int b = 0; b < TB; ++b) red[(rg * tiles + tl) * TB * TB + a * TB + b] = acc[a][b];
      }
      __syncthreads();
    }
    for (int e = t; e < tiles * TB * TB; e += BMS_WG) {
      int tile = e / (TB * TB), ab = e - tile * TB * TB;
      double2 sum;
      if (TB == 4) {
        sum = red[e];
      } else {
        sum = make_double2(0, 0);
        for (int q = 0; q < nrg; ++q) sum = cadd(sum, red[(q * tiles + tile) * TB * TB + ab]);
      }
      TileId d = decode_tile(tile, nt);
      int a = ab / TB, b = ab - (ab / TB) * TB;
      int i = d.ti * TB + a, j = d.tj * TB + b;
      part[d.g * nn + i * n + j] = sum;
      if (d.g >= 2 && d.ti != d.tj) part[d.g * nn + j * n + i] = cconj(sum);
    }
  }
}

// ---- the four Grams of one iteration on the matrix cores --------------------
// Real Gram tiles R = sum_rows x^T y (4 rows per step; the lane holding row
// l/16, column l%16 of a 16-column tile serves as either operand), FP64
// accumulation for FP32 and FP64 inputs: v_mfma_f64_16x16x4 on FP64 blocks;
// on FP32 blocks v_mfma_f32_16x16x4 over one round of D steps (4D rows per
// wave), whose FP32 tiles are then added into FP64 totals.
//  n = 16: tile 0 holds the real parts of the 16 complex columns and tile 1 the
//          imaginary parts, so each lane loads one whole complex per block and
//          step; G[i][j] = R00[i][j] + R11[i][j] + i (R01[i][j] - R10[i][j]).
//  n = 8:  one tile of the 16 interleaved reals; G[i][j] = R[2i][2j] +
//          R[2i+1][2j+1] + i (R[2i][2j+1] - R[2i+1][2j]).
// W^H W and Q^H Q are symmetric in real form: only tiles a <= b are summed.
// D steps of 4 rows are in flight per wave (a register ring).
typedef double gdx4 __attribute__((ext_vector_type(4)));
typedef float gfx4 __attribute__((ext_vector_type(4)));

template <typename T, int N>
struct GramRow {
  static constexpr int NT = 2 * N / 16;
  // the NT operand values of this lane for row r of block X; rows outside the
  // range read row 0 and contribute zero (no branch around the load, so the
  // loads of the ring stay in flight together)
  __device__ static __forceinline__ void load(const cplx<T>* X, int r, bool ok, int c,
                                              double (&v)[NT]) {
    const size_t rc = ok ? (size_t)r : 0;
    if constexpr (N == 16) {
      cplx<T> z = X[rc * N + c];
      v[0] = ok ? (double)z.x : 0.0;
      v[1] = ok ? (double)z.y : 0.0;
    } else {
      const T* x = (const T*)X;
      T z = x[rc * 2 * N + c];
      v[0] = ok ? (double)z : 0.0;
    }
  }
  // complex Gram entry (i, j) from the real Gram R (NR x NR, tile-major)
  __device__ static __forceinline__ double2 entry(const double* R, int i, int j) {
    constexpr int NR = 2 * N;
    if constexpr (N == 16)
      return make_double2(R[i * NR + j] + R[(16 + i) * NR + 16 + j],
                          R[i * NR + 16 + j] - R[(16 + i) * NR + j]);
    else
      return make_double2(R[(2 * i) * NR + 2 * j] + R[(2 * i + 1) * NR + 2 * j + 1],
                          R[(2 * i) * NR + 2 * j + 1] - R[(2 * i + 1) * NR + 2 * j]);
  }
};

// What a lane loads per row and step: the complex of its column (n = 16) or
// the real of its interleaved column (n = 8), kept raw until its step runs.
template <typename T, int N>
struct GramRaw {
  using type = typename std::conditional<N == 16, cplx<T>, T>::type;
  __device__ static __forceinline__ type load(const cplx<T>* X, size_t r, int c) {
    if constexpr (N == 16)
      return X[r * N + c];
    else
      return ((const T*)X)[r * 2 * N + c];
  }
  // the step's operand values (A: double, or float for FP32 blocks), zero
  // for a row past the range
  template <typename A>
  __device__ static __forceinline__ void use(const type& z, bool ok,
                                             A (&v)[GramRow<T, N>::NT]) {
    if constexpr (N == 16) {
      v[0] = ok ? (A)z.x : (A)0;
      v[1] = ok ? (A)z.y : (A)0;
    } else {
      v[0] = ok ? (A)z : (A)0;
    }
  }
};

// Every wave streams its own contiguous rows (a quarter of the block's) in
// steps of 4 and forms all four products, 14 tiles a step for n = 16, so the
// waves carry equal work and never wait for each other. D steps of raw loads
// are in flight: a step's values are taken (and zeroed past the range) right
// before its slot is refilled, and every load is unconditional, so the wait
// for a step covers only that step's loads.
template <typename T, int N, int D>
__global__ __launch_bounds__(BMS_WG) void k_gram4_mfma(int rows,
                                                       const cplx<T>* __restrict__ P,
                                                       const cplx<T>* __restrict__ Q,
                                                       const cplx<T>* __restrict__ W,
                                                                                                              double2* __restrict__ partials,
                                                       const int* __restrict__ skip) {
  using GR = GramRow<T, N>;
  using RW = GramRaw<T, N>;
  using raw = typename RW::type;
  constexpr int NR = 2 * N, NT = GR::NT, NN = N * N;
  constexpr int NPAIR = NT * (NT + 1) / 2;  // tiles a <= b of a symmetric product
  __shared__ double red[4][NR * NR];        // one real Gram per wave
  if (skip && *skip) return;
  const int tid = threadIdx.x, lane = tid & 63;
  // the wave index as a scalar: the step loop's bounds and exits are then
  // uniform branches, which keep the load-wait accounting exact
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, c = lane & 15;
  gdx4 apw[NT][NT], aqw[NT][NT], aww[NPAIR], aqq[NPAIR];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) apw[a][b] = aqw[a][b] = gdx4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < NPAIR; ++e) aww[e] = aqq[e] = gdx4{0.0, 0.0, 0.0, 0.0};
  // steps of 4 rows dealt to the waves of the whole grid in turn (step k of
  // wave v is k * nwaves + v), so the waves in flight read one contiguous
  // stretch of each block vector, as a streaming copy does; each wave runs a
  // whole number of D-step rounds (no exit inside a round, whose loads would
  // then differ by path), steps past the end are empty
  const int nsteps = (rows + 3) >> 2;
  const int nwaves = gridDim.x * 4, vw = blockIdx.x * 4 + wave;
  const int mine = vw < nsteps ? (nsteps - vw + nwaves - 1) / nwaves : 0;
  const int nst = (mine + D - 1) / D * D;
  const size_t rstride = 4 * (size_t)nwaves;  // rows between a wave's steps
  const size_t rbase = 4 * (size_t)vw + g;    // this lane's row at step 0
  raw p[D], q[D], w[D];
  auto fetch = [&](int st, raw& pv, raw& qv, raw& wv) {
    const size_t r = rbase + rstride * st;
    const size_t rc = r < (size_t)rows ? r : 0;
    pv = RW::load(P, rc, c);
    qv = RW::load(Q, rc, c);
    wv = RW::load(W, rc, c);
  };
#pragma unroll
  for (int u = 0; u < D; ++u) fetch(u, p[u], q[u], w[u]);
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (sizeof(T) == 8) {
    for (int st0 = 0; st0 < nst; st0 += D) {
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int st = st0 + u;
        const bool ok = rbase + rstride * st < (size_t)rows;
        double pc[NT], qc[NT], wc[NT];
        RW::use(p[u], ok, pc);
        RW::use(q[u], ok, qc);
        RW::use(w[u], ok, wc);
        fetch(st + D, p[u], q[u], w[u]);
        // keep the refill here, D steps ahead of its use
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b) {
            apw[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(pc[a], wc[b], apw[a][b], 0, 0, 0);
            aqw[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(qc[a], wc[b], aqw[a][b], 0, 0, 0);
          }
        int e = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = a; b < NT; ++b, ++e) {
            aww[e] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[a], wc[b], aww[e], 0, 0, 0);
            aqq[e] = __builtin_amdgcn_mfma_f64_16x16x4f64(qc[a], qc[b], aqq[e], 0, 0, 0);
          }
      }
    }
  } else {
    // FP32 products over one round, then into the FP64 totals
    for (int st0 = 0; st0 < nst; st0 += D) {
      gfx4 fpw[NT][NT], fqw[NT][NT], fww[NPAIR], fqq[NPAIR];
#pragma unroll
      for (int a = 0; a < NT; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) fpw[a][b] = fqw[a][b] = gfx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < NPAIR; ++e) fww[e] = fqq[e] = gfx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < D; ++u) {
        const int st = st0 + u;
        const bool ok = rbase + rstride * st < (size_t)rows;
        float pc[NT], qc[NT], wc[NT];
        RW::use(p[u], ok, pc);
        RW::use(q[u], ok, qc);
        RW::use(w[u], ok, wc);
        fetch(st + D, p[u], q[u], w[u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b) {
            fpw[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(pc[a], wc[b], fpw[a][b], 0, 0, 0);
            fqw[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(qc[a], wc[b], fqw[a][b], 0, 0, 0);
          }
        int e = 0;
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = a; b < NT; ++b, ++e) {
            fww[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(wc[a], wc[b], fww[e], 0, 0, 0);
            fqq[e] = __builtin_amdgcn_mfma_f32_16x16x4f32(qc[a], qc[b], fqq[e], 0, 0, 0);
          }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
          for (int b = 0; b < NT; ++b) {
            apw[a][b][k] += (double)fpw[a][b][k];
            aqw[a][b][k] += (double)fqw[a][b][k];
          }
#pragma unroll
        for (int e = 0; e < NPAIR; ++e) {
          aww[e][k] += (double)fww[e][k];
          aqq[e][k] += (double)fqq[e][k];
        }
      }
    }
  }
  // one product at a time: every wave writes its real Gram (accumulator
  // element k of lane (g, c) is tile row g + 4k for the f64 products, 4g + k
  // for the f32 ones, column c), then the block sums the four and forms the
  // complex entries of its partial
  double* R = red[wave];
  auto put = [&](int a, int b, const gdx4& d, bool mirror) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      int i = a * 16 + (sizeof(T) == 8 ? g + 4 * k : 4 * g + k), j = b * 16 + c;
      R[i * NR + j] = d[k];
      if (mirror) R[j * NR + i] = d[k];
    }
  };
  double2* part = partials + (size_t)blockIdx.x * 4 * NN;
  auto reduce = [&](int gi) {
    __syncthreads();
    for (int e = tid; e < NN; e += BMS_WG) {
      int i = e / N, j = e - (e / N) * N;
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int v = 0; v < 4; ++v) s = cadd(s, GR::entry(red[v], i, j));
      part[gi * NN + e] = s;
    }
    __syncthreads();
  };
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) put(a, b, apw[a][b], false);
  reduce(0);
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) put(a, b, aqw[a][b], false);
  reduce(1);
  {
    int e = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = a; b < NT; ++b, ++e) put(a, b, aww[e], a != b);
  }
  reduce(2);
  {
    int e = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = a; b < NT; ++b, ++e) put(a, b, aqq[e], a != b);
  }
  reduce(3);
}

// Same four Grams, the rows shared through LDS: the block stages chunks of
// GCH rows of P, Q and W (coalesced, the next chunk prefetched into registers
// while the current one is reduced) and each wave owns one product:
// wave 0 P^H W, 1 Q^H W, 2 W^H W, 3 Q^H Q, so a wave holds at most four tiles.
// Per chunk a wave reads all its operands from LDS before its MFMAs; the
// symmetric and the general products run separate loops.
constexpr int GCH = 32;

template <typename T, int N>
struct GramStage {
  using C_ = cplx<T>;
  static constexpr int RS = N + 1;                 // staged row stride (complex), padded
  static constexpr int BS = GCH * RS;              // one staged block
  static constexpr int PER_T = GCH * N / BMS_WG;   // complex per thread and block
};

// operands of row rl of a staged block (GramRow's tile mapping)
template <typename T, int N>
__device__ __forceinline__ void gram_operand(const cplx<T>* blk, int rl, int c,
                                             double (&v)[GramRow<T, N>::NT]) {
  using C_ = cplx<T>;
  constexpr int RS = GramStage<T, N>::RS;
  if constexpr (N == 16) {
    C_ z = blk[rl * RS + c];
    v[0] = (double)z.x;
    v[1] = (double)z.y;
  } else {
    v[0] = (double)((const decltype(C_().x)*)(blk + rl * RS))[c];
  }
}

// one chunk of one wave's product: all its steps' operands, then the MFMAs
template <typename T, int N, bool SYM>
__device__ __forceinline__ void gram_chunk(const cplx<T>* xs, const cplx<T>* ys, int g, int c,
                                           gdx4 (&acc)[GramRow<T, N>::NT][GramRow<T, N>::NT]) {
  constexpr int NT = GramRow<T, N>::NT, ST = GCH / 4;
  double x[ST][NT], y[ST][NT];
#pragma unroll
  for (int st = 0; st < ST; ++st) {
    const int rl = 4 * st + g;
    gram_operand<T, N>(xs, rl, c, x[st]);
    if constexpr (!SYM) gram_operand<T, N>(ys, rl, c, y[st]);
  }
#pragma unroll
  for (int st = 0; st < ST; ++st)
#pragma unroll
    for (int a = 0; a < NT; ++a)
#pragma unroll
      for (int b = SYM ? a : 0; b < NT; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[st][a], SYM ? x[st][b] : y[st][b],
                                                         acc[a][b], 0, 0, 0);
}

// The chunk loop with D chunks in flight: register slot u of the ring holds
// chunk i0 + u; at chunk i the slot of chunk i (already in LDS) is refilled
// with chunk i + D, so a chunk's loads have D - 1 chunks of work to land.
// Every fetch and stash runs unconditionally (rows past the range read a
// valid row and are zeroed by a select, the chunk count is padded to a
// multiple of D with such empty chunks): with loads skipped on some paths the
// compiler can no longer tell which slot is still in flight and waits for all
// of them before every fetch, which serialises the ring.
template <typename T, int N, bool SYM, int D>
__device__ __forceinline__ void gram_sweep(const cplx<T>* P, const cplx<T>* Q, const cplx<T>* W,
                                           RowRange rr, cplx<T>* stage, int xb, int yb,
                                           gdx4 (&acc)[GramRow<T, N>::NT][GramRow<T, N>::NT]) {
  using C_ = cplx<T>;
  using GS = GramStage<T, N>;
  constexpr int NTH = BMS_WG;                      // threads of the block
  constexpr int PER_T = GCH * N / NTH;             // complex per thread and staged block
  static_assert(PER_T >= 1 && GCH * N % NTH == 0, "chunk must cover the block");
  const int tid = threadIdx.x, lane = tid & 63;
  const int g = lane >> 4, c = lane & 15;
  if (rr.r1 <= rr.r0) return;
  const C_* src[3] = {P, Q, W};
  const int nchunks = (rr.r1 - rr.r0 + GCH - 1) / GCH;
  const int npad = (nchunks + D - 1) / D * D;
  C_ nx[D][3][PER_T];
  // element e = tid + k*NTH of a chunk's GCH x N complex; rows past the range
  // load row r0 (the loads stay unconditional) and are zeroed at the stash,
  // so no load result is needed before its chunk is staged
  auto fetch = [&](int ci, C_ (&dst)[3][PER_T]) {
    const int r0 = rr.r0 + ci * GCH;
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
      const int e = tid + k * NTH;
      const size_t at = r0 + e / N < rr.r1 ? (size_t)r0 * N + e : (size_t)rr.r0 * N;
#pragma unroll
      for (int b = 0; b < 3; ++b) dst[b][k] = src[b][at];
    }
  };
  auto stash = [&](const C_ (&from)[3][PER_T], int ci) {
    const int r0 = rr.r0 + ci * GCH, buf = ci & 1;
#pragma unroll
    for (int k = 0; k < PER_T; ++k) {
      const int e = tid + k * NTH;
      const bool ok = r0 + e / N < rr.r1;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        C_ v;
        v.x = ok ? from[b][k].x : 0;
        v.y = ok ? from[b][k].y : 0;
        stage[(buf * 3 + b) * GS::BS + (e / N) * GS::RS + (e % N)] = v;
      }
    }
  };
#pragma unroll
  for (int u = 0; u < D; ++u) fetch(u, nx[u]);
  __builtin_amdgcn_sched_barrier(0);
  stash(nx[0], 0);
  __syncthreads();
  for (int i0 = 0; i0 < npad; i0 += D) {
#pragma unroll
    for (int u = 0; u < D; ++u) {
      const int i = i0 + u;
      fetch(i + D, nx[u]);  // chunk i is in LDS: its slot takes chunk i + D
      // keep the loads here: the scheduler would otherwise sink them next to
      // their use (the stash D - 1 chunks later), leaving no time to land
      __builtin_amdgcn_sched_barrier(0);
      gram_chunk<T, N, SYM>(stage + ((i & 1) * 3 + xb) * GS::BS,
                            stage + ((i & 1) * 3 + yb) * GS::BS, g, c, acc);
      stash(nx[(u + 1) % D], i + 1);
      __syncthreads();
    }
  }
}

template <typename T, int N, int D>
__global__ __launch_bounds__(BMS_WG) void k_gram4_lds(int rows, int per_block,
                                                      const cplx<T>* __restrict__ P,
                                                      const cplx<T>* __restrict__ Q,
                                                      const cplx<T>* __restrict__ W,
                                                      double2* __restrict__ partials,
                                                      const int* __restrict__ skip) {
  using C_ = cplx<T>;
  using GR = GramRow<T, N>;
  using GS = GramStage<T, N>;
  constexpr int NR = 2 * N, NT = GR::NT, NN = N * N;
  constexpr int STAGE = 2 * 3 * GS::BS * (int)sizeof(C_);
  constexpr int REDB = 4 * NR * NR * (int)sizeof(double);
  __shared__ __align__(16) unsigned char smem[STAGE > REDB ? STAGE : REDB];
  if (skip && *skip) return;
  C_* stage = (C_*)smem;  // [2][3][GCH][RS]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int prod = wave;  // this wave's product
  const RowRange rr = block_rows(rows, per_block);
  // this wave's product: x block and y block (0 = P, 1 = Q, 2 = W)
  const int xb = prod == 0 ? 0 : (prod == 2 ? 2 : 1);
  const int yb = prod == 3 ? 1 : 2;
  const bool sym = prod >= 2;
  gdx4 acc[NT][NT];
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = gdx4{0.0, 0.0, 0.0, 0.0};
  if (sym)
    gram_sweep<T, N, true, D>(P, Q, W, rr, stage, xb, yb, acc);
  else
    gram_sweep<T, N, false, D>(P, Q, W, rr, stage, xb, yb, acc);
  // each product's real Gram into LDS (tile row g + 4k, column c), then the
  // complex entries of all four products
  double* R = (double*)smem + prod * NR * NR;
#pragma unroll
  for (int a = 0; a < NT; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) {
      if (sym && b < a) continue;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        int i = a * 16 + g + 4 * k, j = b * 16 + c;
        R[i * NR + j] = acc[a][b][k];
        if (sym && a != b) R[j * NR + i] = acc[a][b][k];
      }
    }
  __syncthreads();
  double2* part = partials + (size_t)blockIdx.x * 4 * NN;
  for (int e = tid; e < 4 * NN; e += BMS_WG) {
    int gi = e / NN, ij = e - gi * NN;
    int i = ij / N, j = ij - (ij / N) * N;
    part[e] = GR::entry((const double*)smem + gi * NR * NR, i, j);
  }
}

}  // namespace

// resident blocks of a BMS_WG-thread kernel per compute unit (0 if unknown)
template <typename K>
static int resident_blocks(K kernel) {
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, BMS_WG, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return occ;
}

int gram4_tb(int n) { return (n >= 16 && n % 4 == 0) ? 4 : ((n % 2 == 0) ? 2 : 1); }

bool gram4_fits(int n) {
  int tb = gram4_tb(n), nt = n / tb;
  return 2 * nt * nt + nt * (nt + 1) <= BMS_WG;
}

bool gram4_mfma_supported(int n) { return n == 8 || n == 16; }

template <typename T>
hipError_t launch_gram4(hipStream_t st, int rows, int n, const void* P, const void* Q,
                        const void* W, double2* G4, double2* partials, int nb,
                        const int* skip, int variant, int num_cu) {
  int per = rows_per_block(rows, nb);
  const cplx<T>* p = (const cplx<T>*)P;
  const cplx<T>* q = (const cplx<T>*)Q;
  const cplx<T>* w = (const cplx<T>*)W;
  const int P4 = 4 * n * n;  // the four Grams' entries per partial
  int grid = nb;
  if (variant >= 3 && gram4_mfma_supported(n)) {
    // chunks in flight per block: variant 3 one, 4 two, 5 four
    // one round of resident blocks: the deeper rings need more registers and
    // fit fewer blocks per compute unit than the three the grid is sized for
#define GL(NN, DD)                                                                              \
  do {                                                                                          \
    static const int occ = resident_blocks(k_gram4_lds<T, NN, DD>);                            \
    const int nbl = num_cu > 0 && occ > 0 ? std::min(nb, occ * num_cu) : nb;                    \
    k_gram4_lds<T, NN, DD><<<nbl, BMS_WG, 0, st>>>(rows, rows_per_block(rows, nbl), p, q, w, \
                                                      partials, skip);                          \
    grid = nbl;                                                                                 \
  } while (0)
    const int depth = variant == 3 ? 1 : (variant == 4 ? 2 : 4);
    if (n == 16) {
      if (depth == 1) GL(16, 1); else if (depth == 2) GL(16, 2); else GL(16, 4);
    } else {
      if (depth == 1) GL(8, 1); else if (depth == 2) GL(8, 2); else GL(8, 4);
    }
#undef GL
    HIP_RET(hipGetLastError());
    return launch_sum_partials(st, partials, grid, P4, G4, skip, nullptr);
  }
  if ((variant < 0 || variant == 1 || variant == 2) && gram4_mfma_supported(n)) {
    // steps in flight per wave: variant 1 four, 2 (and the default) eight
#define GR_(NN, DD)                                                                              \
  do {                                                                                           \
    static const int occ = resident_blocks(k_gram4_mfma<T, NN, DD>);                               \
    const int nbl = num_cu > 0 && occ > 0 ? std::min(nb, occ * num_cu) : nb;                     \
    k_gram4_mfma<T, NN, DD><<<nbl, BMS_WG, 0, st>>>(rows, p, q, w,                                \
                                                    partials, skip);                             \
    grid = nbl;                                                                                  \
  } while (0)
    if (n == 16) {
      if (variant == 1) GR_(16, 4); else GR_(16, 8);
    } else {
      if (variant == 1) GR_(8, 4); else GR_(8, 8);
    }
#undef GR_
    HIP_RET(hipGetLastError());
    return launch_sum_partials(st, partials, grid, P4, G4, skip, nullptr);
  }
  if (!gram4_fits(n)) {  // four pairwise passes
    const cplx<T>* xs[4] = {p, q, w, q};
    const cplx<T>* ys[4] = {w, w, w, q};
    for (int g = 0; g < 4; ++g) HIP_RET(launch_gram<T>(st, rows, n, xs[g], ys[g],
                                                       G4 + (size_t)g * n * n, partials, nb, skip));
    return hipSuccess;
  }
  switch (gram4_tb(n)) {
    case 4:
      k_gram4<T, 4><<<nb, BMS_WG, 0, st>>>(rows, n, per, p, q, w, partials, skip);
      break;
    case 2:
      k_gram4<T, 2><<<nb, BMS_WG, 0, st>>>(rows, n, per, p, q, w, partials, skip);
      break;
    default:
      k_gram4<T, 1><<<nb, BMS_WG, 0, st>>>(rows, n, per, p, q, w, partials, skip);
  }
  HIP_RET(hipGetLastError());
  return launch_sum_partials(st, partials, nb, P4, G4, skip, nullptr);
}
template hipError_t launch_gram4<double>(hipStream_t, int, int, const void*, const void*,
                                         const void*, double2*, double2*, int, const int*, int,
                                         int);
template hipError_t launch_gram4<float>(hipStream_t, int, int, const void*, const void*,
                                        const void*, double2*, double2*, int, const int*, int,
                                        int);

// ---- fused update, specialised on the block width ---------------------------
// Same arithmetic as k_update. Thread (row lr, column j) of each of NCH chunks
// of C = 256/N rows; the j-th columns of alpha_k, rho_k^-1 (FP64) and of each
// shift's Mx, Mp are held in registers, so the only LDS traffic is the row
// broadcast of the block being multiplied. All NCH chunks are staged per sync.
namespace {

__device__ __forceinline__ int next_active(const SolverFlags* fl, int s, int ns) {
  for (++s; s < ns; ++s)
    if (fl->active[s]) break;
  return s;
}

// SPLIT = 0: the j-th columns of Mx and Mp both live in registers;
// SPLIT = 1: one at a time (half the registers, twice the LDS reads).
// The next active shift's P^(s) and X^(s) are prefetched into registers
// while the current one is combined.
template <typename T, typename TX, int N, int NCH, int SPLIT>
__global__ __launch_bounds__(BMS_WG) void k_update_n(UpdateArgs<T, TX> a) {
  using C_ = cplx<T>;
  using CX = cplx<TX>;
  const SolverFlags* fl = a.flags;
  if (fl->halted) return;
  constexpr int C = BMS_WG / N;
  const int t = threadIdx.x;
  const int lr = t / N, j = t % N;
  const bool live = t < C * N;
  const int rbase = blockIdx.x * C * NCH;
  const int rows = a.rows;
  const int ns = a.ns;
  bool act[NCH];
  size_t off[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    int r = rbase + ch * C + lr;
    act[ch] = live && r < rows;
    off[ch] = (size_t)(rbase + ch * C) * N + t;
  }
  C_ qn[NCH];
  if constexpr (N == 1) {
    // no row mixing: every product is a scalar multiplication
    double2 al = a.alpha[0], ri = a.rhoinv[0];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      if (!act[ch]) continue;
      double2 v = csub(to_d(a.Q[off[ch]]), cmul(to_d(a.W[off[ch]]), al));
      qn[ch] = from_d<C_>(cmul(v, ri));
      a.Q[off[ch]] = qn[ch];
    }
    for (int s = 0; s < ns; ++s) {
      if (!fl->active[s]) continue;
      C_* P = a.P + (size_t)s * rows;
      CX* X = a.X + (size_t)a.xidx[s] * rows;
      C_ mx = a.Mx[s], mp = a.Mp[s];
      C_ p[NCH];
      CX x[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (!act[ch]) continue;
        p[ch] = P[off[ch]];
        x[ch] = X[off[ch]];
      }
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) {
        if (!act[ch]) continue;
        C_ dx = cmul(p[ch], mx);
        X[off[ch]] = cmk<CX>(x[ch].x + (TX)dx.x, x[ch].y + (TX)dx.y);
        P[off[ch]] = cfma(p[ch], mp, qn[ch]);
      }
    }
    return;
  } else {
    // rows padded to N + 1 entries: the rows a wave reads sit in different banks
    constexpr int RS = N + 1;
    constexpr int CS = C * RS;
    __shared__ double2 buf[NCH * CS];
    __shared__ C_ ps[NCH * CS];
    const int lw = lr * RS + j;  // this thread's LDS slot inside a chunk
    double2 mcol[N];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      if (act[ch]) buf[ch * CS + lw] = to_d(a.W[off[ch]]);
#pragma unroll
    for (int k = 0; k < N; ++k) mcol[k] = a.alpha[k * N + j];
    __syncthreads();
    double2 v[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      if (!act[ch]) continue;
      double2 wa = make_double2(0, 0);
      const double2* wr = buf + ch * CS + lr * RS;
#pragma unroll
      for (int k = 0; k < N; ++k) wa = cfma(wr[k], mcol[k], wa);
      v[ch] = csub(to_d(a.Q[off[ch]]), wa);
    }
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
      if (act[ch]) buf[ch * CS + lw] = v[ch];
#pragma unroll
    for (int k = 0; k < N; ++k) mcol[k] = a.rhoinv[k * N + j];
    __syncthreads();
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
      if (!act[ch]) continue;
      double2 q = make_double2(0, 0);
      const double2* vr = buf + ch * CS + lr * RS;
#pragma unroll
      for (int k = 0; k < N; ++k) q = cfma(vr[k], mcol[k], q);
      qn[ch] = from_d<C_>(q);
      a.Q[off[ch]] = qn[ch];
    }
    // shifts, with the next active shift's rows prefetched
    C_ pn[NCH];
    CX xn[NCH], xv[NCH];
    int s = next_active(fl, -1, ns);
    if (s < ns) {
      const C_* P = a.P + (size_t)s * rows * N;
      const CX* X = a.X + (size_t)a.xidx[s] * rows * N;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (act[ch]) {
          pn[ch] = P[off[ch]];
          xn[ch] = X[off[ch]];
        }
    }
    while (s < ns) {
      const int s2 = next_active(fl, s, ns);
      C_* P = a.P + (size_t)s * rows * N;
      CX* X = a.X + (size_t)a.xidx[s] * rows * N;
      const C_* Mx = a.Mx + (size_t)s * N * N;
      const C_* Mp = a.Mp + (size_t)s * N * N;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
        if (act[ch]) {
          ps[ch * CS + lw] = pn[ch];
          xv[ch] = xn[ch];
        }
      __syncthreads();
      if (s2 < ns) {
        const C_* P2 = a.P + (size_t)s2 * rows * N;
        const CX* X2 = a.X + (size_t)a.xidx[s2] * rows * N;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
          if (act[ch]) {
            pn[ch] = P2[off[ch]];
            xn[ch] = X2[off[ch]];
          }
      }
      if constexpr (SPLIT) {
        C_ m[N];
#pragma unroll
        for (int k = 0; k < N; ++k) m[k] = Mx[k * N + j];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (!act[ch]) continue;
          const C_* pr = ps + ch * CS + lr * RS;
          C_ dx = czero<C_>();
#pragma unroll
          for (int k = 0; k < N; ++k) dx = cfma(pr[k], m[k], dx);
          X[off[ch]] = cmk<CX>(xv[ch].x + (TX)dx.x, xv[ch].y + (TX)dx.y);
        }
#pragma unroll
        for (int k = 0; k < N; ++k) m[k] = Mp[k * N + j];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (!act[ch]) continue;
          const C_* pr = ps + ch * CS + lr * RS;
          C_ np = qn[ch];
#pragma unroll
          for (int k = 0; k < N; ++k) np = cfma(pr[k], m[k], np);
          P[off[ch]] = np;
        }
      } else {
        C_ mx[N], mp[N];
#pragma unroll
        for (int k = 0; k < N; ++k) {
          mx[k] = Mx[k * N + j];
          mp[k] = Mp[k * N + j];
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
          if (!act[ch]) continue;
          const C_* pr = ps + ch * CS + lr * RS;
          C_ dx = czero<C_>();
          C_ np = qn[ch];
#pragma unroll
          for (int k = 0; k < N; ++k) {
            C_ pk = pr[k];
            dx = cfma(pk, mx[k], dx);
            np = cfma(pk, mp[k], np);
          }
          X[off[ch]] = cmk<CX>(xv[ch].x + (TX)dx.x, xv[ch].y + (TX)dx.y);
          P[off[ch]] = np;
        }
      }
      __syncthreads();
      s = s2;
    }
  }
}

template <typename T, typename TX, int N, int NCH, int SPLIT>
hipError_t launch_update_n(hipStream_t st, const UpdateArgs<T, TX>& a) {
  int per = (BMS_WG / N) * NCH;
  k_update_n<T, TX, N, NCH, SPLIT><<<(a.rows + per - 1) / per, BMS_WG, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace

template <typename T, typename TX>
hipError_t launch_update_fast(hipStream_t st, const UpdateArgs<T, TX>& a, int variant) {
  // variant: 0 = NCH 4 both columns, 1 = NCH 2 split, 2 = NCH 4 split, 3 = NCH 2 both
  switch (a.n) {
    case 1: return launch_update_n<T, TX, 1, 4, 0>(st, a);
    case 2: return launch_update_n<T, TX, 2, 4, 0>(st, a);
    case 4: return launch_update_n<T, TX, 4, 4, 0>(st, a);
    case 8:
      switch (variant) {
        case 1: return launch_update_n<T, TX, 8, 2, 1>(st, a);
        case 2: return launch_update_n<T, TX, 8, 4, 1>(st, a);
        case 3: return launch_update_n<T, TX, 8, 2, 0>(st, a);
        default: return launch_update_n<T, TX, 8, 4, 0>(st, a);
      }
    case 16:
      switch (variant) {
        case 1: return launch_update_n<T, TX, 16, 2, 1>(st, a);
        case 2: return launch_update_n<T, TX, 16, 4, 1>(st, a);
        case 3: return launch_update_n<T, TX, 16, 2, 0>(st, a);
        default: return launch_update_n<T, TX, 16, 4, 0>(st, a);
      }
    default: return launch_update<T, TX>(st, a);
  }
}

template hipError_t launch_update_fast<double, double>(hipStream_t,
                                                       const UpdateArgs<double, double>&, int);
template hipError_t launch_update_fast<float, float>(hipStream_t, const UpdateArgs<float, float>&,
                                                     int);

// ---- precision control: reliable updates and defect correction --------------
namespace {

// R[r][i] = (B[r][i] - Y[r][i]) * cs[i]; a column with cs[i] == 0 is replaced
// by B[r][i] * cb[i] (a harmless non-zero column for the block solver)
__global__ __launch_bounds__(BMS_WG) void k_resid_block(int rows, int n, const double2* __restrict__ B,
                                                        const double2* __restrict__ Y,
                                                        const double* __restrict__ cs,
                                                        const double* __restrict__ cb,
                                                        double2* __restrict__ R,
                                                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x;
  if (i >= (size_t)rows * n) return;
  int col = (int)(i % n);
  double c = cs ? cs[col] : 1.0;
  R[i] = (c != 0.0 || !cb) ? cscale(csub(B[i], Y[i]), c) : cscale(B[i], cb[col]);
}

// X[r][i] += E[r][i] * cs[i]
__global__ __launch_bounds__(BMS_WG) void k_axpy_cols(int rows, int n, double2* __restrict__ X,
                                                      const double2* __restrict__ E,
                                                      const double* __restrict__ cs) {
  size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x;
  if (i >= (size_t)rows * n) return;
  X[i] = cadd(X[i], cscale(E[i], cs[i % n]));
}

// out = a0 B + sum_s alpha[s] X[s] (eq. RA applied to a block, from the
// shifted solutions): one pass over B and every X[s], two complex elements
// per thread, the terms added in shift order.
struct CombineArgs {
  size_t blk;  // complex elements per block
  int ns;
  double a0;
  double alpha[BMS_MAX_SHIFTS];
};

__global__ __launch_bounds__(BMS_WG) void k_rational_combine(CombineArgs a,
                                                             const double2* __restrict__ B,
                                                             const double2* __restrict__ X,
                                                             double2* __restrict__ out) {
  const size_t i = 2 * ((size_t)blockIdx.x * BMS_WG + threadIdx.x);
  if (i >= a.blk) return;
  const bool two = i + 1 < a.blk;
  double2 v0 = cscale(B[i], a.a0), v1 = two ? cscale(B[i + 1], a.a0) : make_double2(0, 0);
  for (int s = 0; s < a.ns; ++s) {
    const double2* xs = X + (size_t)s * a.blk;
    v0 = cadd(v0, cscale(xs[i], a.alpha[s]));
    if (two) v1 = cadd(v1, cscale(xs[i + 1], a.alpha[s]));
  }
  out[i] = v0;
  if (two) out[i + 1] = v1;
}

// X64[xmap[s]] += X32[s]; X32[s] = 0 for every shift (FP32 increments into
// the FP64 solutions)
struct FlushArgs {
  int rows, n, ns;
  float2* X32;
  double2* X64;
  int xmap[BMS_MAX_SHIFTS];
};

__global__ __launch_bounds__(BMS_WG) void k_flush(FlushArgs a, const int* __restrict__ skip) {
  if (skip && *skip) return;
  size_t blk = (size_t)a.rows * a.n;
  size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x;
  if (i >= blk) return;
  for (int s = 0; s < a.ns; ++s) {
    float2 v = a.X32[s * blk + i];
    if (v.x != 0.f || v.y != 0.f) {
      double2* x = a.X64 + (size_t)a.xmap[s] * blk + i;
      *x = make_double2(x->x + v.x, x->y + v.y);
      a.X32[s * blk + i] = make_float2(0.f, 0.f);
    }
  }
}

// Y = X M with FP64 input X, FP64 M, output in precision TO
template <typename TO>
__global__ __launch_bounds__(BMS_WG) void k_block_matmul_d(int rows, int n,
                                                           const double2* __restrict__ X,
                                                           const double2* __restrict__ M,
                                                           cplx<TO>* __restrict__ Y,
                                                           const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double2 xs[BMS_WG];
  int C = BMS_WG / n;
  int r0 = blockIdx.x * C;
  int nr = min(C, rows - r0);
  int t = threadIdx.x;
  if (t < nr * n) xs[t] = X[(size_t)r0 * n + t];
  __syncthreads();
  if (t < nr * n) {
    int lr = t / n, j = t - lr * n;
    double2 acc = make_double2(0, 0);
    for (int k = 0; k < n; ++k) acc = cfma(xs[lr * n + k], M[k * n + j], acc);
    Y[(size_t)r0 * n + t] = from_d<cplx<TO>>(acc);
  }
}

}  // namespace

static unsigned grid_for(size_t n) { return (unsigned)((n + BMS_WG - 1) / BMS_WG); }

hipError_t launch_resid_block(hipStream_t st, int rows, int n, const void* B, const void* Y,
                              const double* cs, const double* cb, void* R, const int* skip) {
  k_resid_block<<<grid_for((size_t)rows * n), BMS_WG, 0, st>>>(
      rows, n, (const double2*)B, (const double2*)Y, cs, cb, (double2*)R, skip);
  return hipGetLastError();
}

hipError_t launch_axpy_cols(hipStream_t st, int rows, int n, void* X, const void* E,
                            const double* cs) {
  k_axpy_cols<<<grid_for((size_t)rows * n), BMS_WG, 0, st>>>(rows, n, (double2*)X,
                                                            (const double2*)E, cs);
  return hipGetLastError();
}

hipError_t launch_rational_combine(hipStream_t st, size_t blk, int ns, double a0,
                                   const double* alpha, const void* B, const void* X, void* out) {
  CombineArgs a;
  a.blk = blk;
  a.ns = ns;
  a.a0 = a0;
  for (int s = 0; s < BMS_MAX_SHIFTS; ++s) a.alpha[s] = s < ns ? alpha[s] : 0.0;
  k_rational_combine<<<grid_for((blk + 1) / 2), BMS_WG, 0, st>>>(a, (const double2*)B,
                                                                 (const double2*)X, (double2*)out);
  return hipGetLastError();
}

hipError_t launch_flush(hipStream_t st, int rows, int n, int ns, void* X32, void* X64,
                        const int* xmap, const int* skip) {
  FlushArgs a;
  a.rows = rows;
  a.n = n;
  a.ns = ns;
  a.X32 = (float2*)X32;
  a.X64 = (double2*)X64;
  for (int s = 0; s < BMS_MAX_SHIFTS; ++s) a.xmap[s] = s < ns ? xmap[s] : 0;
  k_flush<<<grid_for((size_t)rows * n), BMS_WG, 0, st>>>(a, skip);
  return hipGetLastError();
}

template <typename TO>
hipError_t launch_block_matmul_d(hipStream_t st, int rows, int n, const void* X, const double2* M,
                                 void* Y, const int* skip) {
  int C = BMS_WG / n;
  k_block_matmul_d<TO><<<(rows + C - 1) / C, BMS_WG, 0, st>>>(rows, n, (const double2*)X, M,
                                                              (cplx<TO>*)Y, skip);
  return hipGetLastError();
}
template hipError_t launch_block_matmul_d<float>(hipStream_t, int, int, const void*,
                                                 const double2*, void*, const int*);
template hipError_t launch_block_matmul_d<double>(hipStream_t, int, int, const void*,
                                                  const double2*, void*, const int*);

// ---- per-column defect correction -----------------------------------------
namespace {
__global__ __launch_bounds__(BMS_WG) void k_gather_col(int rows, int n, int col,
                                                       const double2* __restrict__ src,
                                                       double2* __restrict__ dst) {
  int r = blockIdx.x * BMS_WG + threadIdx.x;
  if (r < rows) dst[r] = src[(size_t)r * n + col];
}
__global__ __launch_bounds__(BMS_WG) void k_scatter_axpy_col(int rows, int n, int col,
                                                             double2* __restrict__ X,
                                                             const double2* __restrict__ e,
                                                             double scale) {
  int r = blockIdx.x * BMS_WG + threadIdx.x;
  if (r < rows) {
    size_t o = (size_t)r * n + col;
    X[o] = cadd(X[o], cscale(e[r], scale));
  }
}
}  // namespace

hipError_t launch_gather_col(hipStream_t st, int rows, int n, int col, const void* src, void* dst) {
  k_gather_col<<<grid_for(rows), BMS_WG, 0, st>>>(rows, n, col, (const double2*)src,
                                                 (double2*)dst);
  return hipGetLastError();
}

hipError_t launch_scatter_axpy_col(hipStream_t st, int rows, int n, int col, void* X,
                                   const void* e, double scale) {
  k_scatter_axpy_col<<<grid_for(rows), BMS_WG, 0, st>>>(rows, n, col, (double2*)X,
                                                       (const double2*)e, scale);
  return hipGetLastError();
}
