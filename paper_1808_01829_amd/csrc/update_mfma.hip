// FP64 fused block update on the matrix cores (v_mfma_f64_16x16x4).
//
// Same arithmetic as the vector update kernels, per iteration k of
// Algorithm 1 (block CG with Cholesky-QR, Sec. III):
//   Q_{k+1} = (Q_k - W alpha_k) rho_k^-1   computed as  Q_k rho^-1 + W (-alpha rho^-1)
//   X^(s)  += P^(s) Mx^(s)                 (Mx = alpha^(s)_k)
//   P^(s)   = Q_{k+1} + P^(s) Mp^(s)       (Mp = beta^(s)_k rho_k^dag)
// for every shift still active.
//
// A complex row of n entries is 2n interleaved reals; a right product with a
// complex n x n matrix M is the real product with the 2n x 2n matrix
//   [ Re M  Im M ]
//   [-Im M  Re M ]   (rows in (re, im) pairs, columns permuted: all real parts
// first, then all imaginary parts). Each wave owns 16-row tiles. The MFMA
// operand layouts (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k, D[i][j]
// in lane j + 16(i%4), element i/4; the D layout was measured on gfx950) give:
//   A operand: lane (g = lane/16, c = lane%16) holds row c, reals g*KS .. g*KS+KS-1
//              (the contraction order is free, so each lane reads one contiguous run);
//   D: lane (g, c) holds rows g, g+4, g+8, g+12 at real output column nt*16 + c, which for
//      n = 16 is (Re, Im) of complex column c in the two n-tiles: one 16-byte
//      complex per row, so X and P are read and written as whole complex numbers.
// The coefficient matrices are expanded into that B layout in LDS once per
// work-group and shift (double-buffered, one barrier per shift).
#include "blas.h"

namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));

constexpr int MF_WAVES = BMS_WG / 64;

template <int N>
struct MfShape {
  static constexpr int NR = 2 * N;      // reals per row
  static constexpr int KS = NR / 4;     // k-steps of 4
  static constexpr int NT = NR / 16;    // 16-column output tiles
  static constexpr int BSZ = NR * NR;   // doubles of one expanded matrix
};

// entry (kk, flat) of the expanded matrix -> its LDS slot in B-operand order
template <int N>
__device__ __forceinline__ int bslot(int kk, int flat) {
  using S = MfShape<N>;
  int gg = kk / S::KS, ks = kk - gg * S::KS;
  int nt = flat >> 4, cc = flat & 15;
  return ((ks * 64) + gg * 16 + cc) * S::NT + nt;
}

// expand complex m = M[k][j] into the four reals it contributes
template <int N>
__device__ __forceinline__ void bput(double* B, int k, int j, double2 m) {
  B[bslot<N>(2 * k, j)] = m.x;
  B[bslot<N>(2 * k, N + j)] = m.y;
  B[bslot<N>(2 * k + 1, j)] = -m.y;
  B[bslot<N>(2 * k + 1, N + j)] = m.x;
}

template <int N>
__device__ __forceinline__ void bload(const double* B, int lane, double (&b)[MfShape<N>::KS][MfShape<N>::NT]) {
  using S = MfShape<N>;
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt) b[ks][nt] = B[(ks * 64 + lane) * S::NT + nt];
}

// A-operand reals of one tile row: row r, reals g*KS .. g*KS+KS-1
template <int N>
__device__ __forceinline__ void aload(const double2* base, int r, int rows, int g,
                                      double (&a)[MfShape<N>::KS]) {
  using S = MfShape<N>;
  if (r < rows) {
    const double2* p = base + (size_t)r * N + g * (S::KS / 2);
#pragma unroll
    for (int h = 0; h < S::KS / 2; ++h) {
      double2 v = p[h];
      a[2 * h] = v.x;
      a[2 * h + 1] = v.y;
    }
  } else {
#pragma unroll
    for (int h = 0; h < S::KS; ++h) a[h] = 0.0;
  }
}

// D-layout access: lane (g, c), element p is row g+4p of the tile, output
// real column flat = nt*16 + c: part flat / N (0 = re, 1 = im) of complex column flat % N.
template <int N>
__device__ __forceinline__ void dload(const double2* base, int r0, int rows, int g, int c,
                                      dx4 (&d)[MfShape<N>::NT]) {
  if constexpr (N == 16) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r = r0 + g + 4 * p;
      double2 v = r < rows ? base[(size_t)r * N + c] : make_double2(0.0, 0.0);
      d[0][p] = v.x;
      d[1][p] = v.y;
    }
  } else {
    const double* b = (const double*)base;
    const int re = 2 * (c % N) + c / N;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r = r0 + g + 4 * p;
      d[0][p] = r < rows ? b[(size_t)r * 2 * N + re] : 0.0;
    }
  }
}

template <int N>
__device__ __forceinline__ void dstore(double2* base, int r0, int rows, int g, int c,
                                       const dx4 (&d)[MfShape<N>::NT]) {
  if constexpr (N == 16) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r = r0 + g + 4 * p;
      if (r < rows) base[(size_t)r * N + c] = make_double2(d[0][p], d[1][p]);
    }
  } else {
    double* b = (double*)base;
    const int re = 2 * (c % N) + c / N;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      int r = r0 + g + 4 * p;
      if (r < rows) b[(size_t)r * 2 * N + re] = d[0][p];
    }
  }
}

template <int N>
__device__ __forceinline__ void mfma_acc(dx4 (&d)[MfShape<N>::NT], const double (&a)[MfShape<N>::KS],
                                         const double (&b)[MfShape<N>::KS][MfShape<N>::NT]) {
  using S = MfShape<N>;
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt)
      d[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks][nt], d[nt], 0, 0, 0);
}

// T: 16-row tiles per wave (processed one after the other inside each shift,
// so the coefficient operands are read from LDS once per wave and shift).
template <int N, int T>
__global__ __launch_bounds__(BMS_WG) void k_update_mfma(UpdateArgs<double, double> a) {
  using S = MfShape<N>;
  __shared__ double bl[2][2][S::BSZ];
  const SolverFlags* fl = a.flags;
  if (fl->halted) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int rows = a.rows, ns = a.ns;
  const int tile0 = (blockIdx.x * MF_WAVES + wave) * T;
  const double2* Mx = (const double2*)a.Mx;
  const double2* Mp = (const double2*)a.Mp;

  // coefficients of the Q step: B0 = rho^-1, B1 = -alpha rho^-1
  {
    double2* cs = (double2*)&bl[1][0][0];  // complex staging: alpha, rho^-1
    for (int e = tid; e < N * N; e += BMS_WG) {
      cs[e] = a.alpha[e];
      cs[N * N + e] = a.rhoinv[e];
    }
    __syncthreads();
    for (int e = tid; e < N * N; e += BMS_WG) {
      int i = e / N, j = e - (e / N) * N;
      double2 t = make_double2(0.0, 0.0);
      for (int k = 0; k < N; ++k) t = cfma(cs[i * N + k], cs[N * N + k * N + j], t);
      bput<N>(bl[0][0], i, j, cs[N * N + e]);
      bput<N>(bl[0][1], i, j, make_double2(-t.x, -t.y));
    }
    __syncthreads();
  }
  dx4 qn[T][S::NT];
  {
    double b0[S::KS][S::NT], b1[S::KS][S::NT];
    bload<N>(bl[0][0], lane, b0);
    bload<N>(bl[0][1], lane, b1);
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int r0 = (tile0 + t) * 16;
      double av[S::KS];
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt) qn[t][nt] = dx4{0.0, 0.0, 0.0, 0.0};
      if (r0 < rows) {
        aload<N>(a.Q, r0 + c, rows, g, av);
        mfma_acc<N>(qn[t], av, b0);
        aload<N>(a.W, r0 + c, rows, g, av);
        mfma_acc<N>(qn[t], av, b1);
      }
    }
  }
  // every lane of the wave has read its Q tiles before any is overwritten
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int r0 = (tile0 + t) * 16;
    if (r0 < rows) dstore<N>(a.Q, r0, rows, g, c, qn[t]);
  }
  __syncthreads();  // bl[0] is rewritten below

  int buf = 0;
  for (int s = 0; s < ns; ++s) {
    if (!fl->active[s]) continue;
    double* bx = bl[buf][0];
    double* bp = bl[buf][1];
    const double2* mx = Mx + (size_t)s * N * N;
    const double2* mp = Mp + (size_t)s * N * N;
    for (int e = tid; e < N * N; e += BMS_WG) {
      int i = e / N, j = e - (e / N) * N;
      bput<N>(bx, i, j, mx[e]);
      bput<N>(bp, i, j, mp[e]);
    }
    __syncthreads();
    double cx[S::KS][S::NT], cp[S::KS][S::NT];
    bload<N>(bx, lane, cx);
    bload<N>(bp, lane, cp);
    double2* P = a.P + (size_t)s * rows * N;
    double2* X = a.X + (size_t)a.xidx[s] * rows * N;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int r0 = (tile0 + t) * 16;
      if (r0 >= rows) break;
      double pa[S::KS];
      dx4 xa[S::NT], pn[S::NT];
      aload<N>(P, r0 + c, rows, g, pa);
      dload<N>(X, r0, rows, g, c, xa);
      mfma_acc<N>(xa, pa, cx);
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt) pn[nt] = qn[t][nt];
      mfma_acc<N>(pn, pa, cp);
      dstore<N>(X, r0, rows, g, c, xa);
      dstore<N>(P, r0, rows, g, c, pn);
    }
    buf ^= 1;
  }
}

template <int N, int T>
hipError_t launch_mf(hipStream_t st, const UpdateArgs<double, double>& a) {
  int tiles = (a.rows + 15) / 16;
  int waves = (tiles + T - 1) / T;
  int blocks = (waves + MF_WAVES - 1) / MF_WAVES;
  k_update_mfma<N, T><<<blocks, BMS_WG, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace

bool update_mfma_supported(int n) { return n == 8 || n == 16; }

hipError_t launch_update_mfma(hipStream_t st, const UpdateArgs<double, double>& a) {
  switch (a.n) {
    case 16: return launch_mf<16, 2>(st, a);
    case 8: return launch_mf<8, 2>(st, a);
    default: return hipErrorInvalidValue;
  }
}
