// Fused block update on the matrix cores (v_mfma_f64_16x16x4 in FP64,
// v_mfma_f32_16x16x4 for the shift updates of the mixed solver).
//
// Same arithmetic as the vector update kernels, per iteration k of
// Algorithm 1 (block CG with Cholesky-QR, Sec. III):
//   Q_{k+1} = (Q_k - W alpha_k) rho_k^-1   computed as  Q_k rho^-1 + W (-alpha rho^-1)
//   X^(s)  += P^(s) Mx^(s)                 (Mx = alpha^(s)_k)
//   P^(s)   = Q_{k+1} + P^(s) Mp^(s)       (Mp = beta^(s)_k rho_k^dag)
// for every shift still active. The Q step always runs in FP64 (FP32 blocks
// are widened on load), the shift updates in the block precision.
//
// A complex row of n entries is 2n interleaved reals; a right product with a
// complex n x n matrix M is the real product with the 2n x 2n matrix
//   [ Re M  Im M ]
//   [-Im M  Re M ]   (rows in (re, im) pairs, columns permuted: all real parts
// first, then all imaginary parts). Each wave owns 16-row tiles. The MFMA
// operand layouts (A[i][k] in lane i + 16k, B[k][j] in lane j + 16k; the
// accumulator D[i][j] in lane j + 16(i%4), element i/4 for f64 and in lane
// j + 16(i/4), element i%4 for f32 -- both measured on gfx950) give:
//   A operand: lane (g = lane/16, c = lane%16) holds row c, reals g*KS .. g*KS+KS-1
//              (the contraction order is free, so each lane reads one contiguous run);
//   D: lane (g, c) holds four rows of the tile at real output column nt*16 + c,
//      which for n = 16 is (Re, Im) of complex column c in the two n-tiles: one
//      complex per row, so X and P are read and written as whole complex numbers.
// The Q step's two coefficient matrices are expanded into that B layout in
// LDS once per work-group. The shift coefficients are kept in LDS as complex
// n x n matrices (double-buffered, one barrier per shift), and each lane
// forms its B operands from them one k-step at a time.
#include "blas.h"

namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

constexpr int MF_WAVES = BMS_WG / 64;

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glob_void;

// Copy `bytes` rounded up to whole KiB (both regions hold that much) from
// global memory into LDS by direct-to-LDS loads (global_load_lds_dwordx4, lane
// l of a wave writing 16 bytes at the wave's destination + 16 l): wave w
// copies the KiB chunks w, w + 4, ... Nothing passes through registers, so
// every load of a shift's coefficients is in flight at once instead of one
// round trip per matrix.
__device__ __forceinline__ void lds_copy(const void* src, void* dst, int bytes, int wave,
                                         int lane) {
  for (int off = wave * 1024; off < bytes; off += MF_WAVES * 1024)
    __builtin_amdgcn_global_load_lds((glob_void*)((const char*)src + off + lane * 16),
                                     (lds_void*)((char*)dst + off), 16, 0, 0);
}

template <typename F>
struct Mf;
template <>
struct Mf<double> {
  using V = dx4;
  __device__ static __forceinline__ V mfma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // tile row of accumulator element p in lane group g
  __device__ static __forceinline__ int row(int g, int p) { return g + 4 * p; }
};
template <>
struct Mf<float> {
  using V = fx4;
  __device__ static __forceinline__ V mfma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int g, int p) { return 4 * g + p; }
};

template <int N>
struct MfShape {
  static constexpr int NR = 2 * N;      // reals per row
  static constexpr int KS = NR / 4;     // k-steps of 4
  static constexpr int NT = NR / 16;    // 16-column output tiles
  static constexpr int BSZ = NR * NR;   // reals of one expanded matrix
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
template <int N, typename F>
__device__ __forceinline__ void bput(F* B, int k, int j, double2 m) {
  B[bslot<N>(2 * k, j)] = (F)m.x;
  B[bslot<N>(2 * k, N + j)] = (F)m.y;
  B[bslot<N>(2 * k + 1, j)] = (F)-m.y;
  B[bslot<N>(2 * k + 1, N + j)] = (F)m.x;
}

template <int N, typename F>
__device__ __forceinline__ void bload(const F* B, int lane, F (&b)[MfShape<N>::KS][MfShape<N>::NT]) {
  using S = MfShape<N>;
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt) b[ks][nt] = B[(ks * 64 + lane) * S::NT + nt];
}

// The shift coefficients are kept in LDS as the complex n x n matrix, (re,
// im) pairs, half of the expanded form; each lane forms its B-operand
// reals from it: B[2k][j] = Re M[k][j], B[2k][n+j] = Im, B[2k+1][j] = -Im,
// B[2k+1][n+j] = Re, at kk = g*KS + ks, flat = nt*16 + c.
// d += a * B(M), the B operands read from LDS one k-step at a time (few
// registers live: the kernel keeps four waves per SIMD)
template <int N, typename F>
__device__ __forceinline__ void mfma_acc_c(typename Mf<F>::V (&d)[MfShape<N>::NT],
                                           const F (&a)[MfShape<N>::KS], const F* M, int g,
                                           int c) {
  using S = MfShape<N>;
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt) {
      const int kk = g * S::KS + ks, flat = nt * 16 + c;
      const int k = kk >> 1, rim = kk & 1, j = flat % N, cim = flat / N;
      const F v = M[2 * (k * N + j) + (rim ^ cim)];
      d[nt] = Mf<F>::mfma(a[ks], rim && !cim ? -v : v, d[nt]);
    }
}

// n = 16: the complex right product by Gauss's three real products. With
// the A operand of a lane holding complex columns 4g .. 4g+3 of its row (the
// same contiguous run as above), k-step ks contracts over complex column
// kc = 4g + ks, and the three accumulators gather
//   d0 = sum Re a Re M,  d1 = sum Im a Im M,  d2 = sum (Re a + Im a)(Re M + Im M),
// from which Re(a M) = d0 - d1 and Im(a M) = d2 - d0 - d1 (mfma3_re/_im).
// Output column c of every accumulator is complex column c, so the two
// results land in the layout of the n-tiles above (tile 0 real parts, tile 1
// imaginary parts). 12 matrix-core steps per product and 16-row tile, against
// 16 for the 32 x 32 real form. M: complex 16 x 16 in LDS, (re, im) pairs.
template <typename F>
__device__ __forceinline__ void mfma3(typename Mf<F>::V (&d)[3], const F (&a)[MfShape<16>::KS],
                                      const F* M, int g, int c) {
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    const int e = 2 * ((4 * g + ks) * 16 + c);
    const F mr = M[e], mi = M[e + 1];
    const F ar = a[2 * ks], ai = a[2 * ks + 1];
    d[0] = Mf<F>::mfma(ar, mr, d[0]);
    d[1] = Mf<F>::mfma(ai, mi, d[1]);
    d[2] = Mf<F>::mfma(ar + ai, mr + mi, d[2]);
  }
}
template <typename V>
__device__ __forceinline__ V mfma3_re(const V (&d)[3]) {
  return d[0] - d[1];
}
template <typename V>
__device__ __forceinline__ V mfma3_im(const V (&d)[3]) {
  return d[2] - d[0] - d[1];
}

// A-operand reals of one tile row (row r, reals g*KS .. g*KS+KS-1) in the
// arithmetic type F. Rows past the end read row 0 and are zeroed, with no
// branch around the loads (so the loads of several tiles stay in flight).
template <int N, typename F, typename C>
__device__ __forceinline__ void aload(const C* base, int r, int rows, int g,
                                      F (&a)[MfShape<N>::KS]) {
  using S = MfShape<N>;
  const bool ok = r < rows;
  const C* p = base + (size_t)(ok ? r : 0) * N + g * (S::KS / 2);
#pragma unroll
  for (int h = 0; h < S::KS / 2; ++h) {
    C v = p[h];
    a[2 * h] = ok ? (F)v.x : (F)0;
    a[2 * h + 1] = ok ? (F)v.y : (F)0;
  }
}

// D-layout access: lane (g, c), element p is tile row Mf<F>::row(g, p), output
// real column flat = nt*16 + c: part flat / N (0 = re, 1 = im) of complex column flat % N.
template <int N, typename F, typename C>
__device__ __forceinline__ void dload(const C* base, int r0, int rows, int g, int c,
                                      typename Mf<F>::V (&d)[MfShape<N>::NT]) {
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int r = r0 + Mf<F>::row(g, p);
    const bool ok = r < rows;
    const size_t rr = ok ? (size_t)r : 0;
    if constexpr (N == 16) {
      C v = base[rr * N + c];
      d[0][p] = ok ? (F)v.x : (F)0;
      d[1][p] = ok ? (F)v.y : (F)0;
    } else {
      auto v = ((const decltype(C().x)*)base)[rr * 2 * N + 2 * (c % N) + c / N];
      d[0][p] = ok ? (F)v : (F)0;
    }
  }
}

template <int N, typename F, typename C>
__device__ __forceinline__ void dstore(C* base, int r0, int rows, int g, int c,
                                       const typename Mf<F>::V (&d)[MfShape<N>::NT]) {
  using R = decltype(C().x);
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int r = r0 + Mf<F>::row(g, p);
    if (r >= rows) continue;
    if constexpr (N == 16) {
      C v;
      v.x = (R)d[0][p];
      v.y = (R)d[1][p];
      base[(size_t)r * N + c] = v;
    } else {
      ((R*)base)[(size_t)r * 2 * N + 2 * (c % N) + c / N] = (R)d[0][p];
    }
  }
}

template <int N, typename F>
__device__ __forceinline__ void mfma_acc(typename Mf<F>::V (&d)[MfShape<N>::NT],
                                         const F (&a)[MfShape<N>::KS],
                                         const F (&b)[MfShape<N>::KS][MfShape<N>::NT]) {
  using S = MfShape<N>;
#pragma unroll
  for (int ks = 0; ks < S::KS; ++ks)
#pragma unroll
    for (int nt = 0; nt < S::NT; ++nt) d[nt] = Mf<F>::mfma(a[ks], b[ks][nt], d[nt]);
}

// Longest window of the deferred shift update whose coefficients (2 x window
// complex n x n matrices of one shift) the kernel stages in LDS: 32 KiB at
// n = 16 in either precision.
template <typename F>
struct MfWin {
  static constexpr int MW = sizeof(F) == 8 ? 4 : 8;
};

// F: block and shift-update arithmetic type (double, or float in the mixed
// solver). NTILE: 16-row tiles per wave (processed one after the other inside
// each shift).
//
// The Q step reads Q_k from ring buffer k % win and writes Q_{k+1} to
// buffer (k+1) % win (in place for win = 1). Then every shift whose update
// window the small step closed (or, when the solve stops here, every open
// one) is applied, with j iterations in its window:
//   X += P Cx + sum_{i < j-1} Q_{k-j+2+i} Ex_i
//   P  = Q_{k+1} + P Cp + sum_{i < j-1} Q_{k-j+2+i} Ep_i     (in place)
// (sigma_0: j = 1 every iteration, the plain X += P Mx, P = Q + P Mp). A
// shift moves 4 block vectors per window instead of 4 per iteration; the
// ring buffers it also reads are the same for every shift, so after the
// first shift of a tile they come from L2.
// One tile per wave: four waves per SIMD in FP32, three in FP64 (the register
// count the compiler picks by itself leaves fewer; in FP64 four waves need
// spills, whose scratch traffic reached HBM). For n = 16 every complex
// product (Q step and shift windows) takes the three-product form.
template <typename F, int N, int NTILE>
__global__ __launch_bounds__(BMS_WG)
__attribute__((amdgpu_waves_per_eu(NTILE == 1 ? (sizeof(F) == 4 ? 4 : 3) : 1)))
void k_update_mfma(UpdateArgs<F, F> a) {
  using S = MfShape<N>;
  using CF = cplx<F>;
  using VF = typename Mf<F>::V;
  constexpr int MW = MfWin<F>::MW;
  // LDS: the Q-step operands (FP64) and the complex staging, then (FP32) the
  // per-wave layout change of Q, then one shift's window coefficients (F)
  constexpr int QBYTES = 2 * S::BSZ * 8 + 2 * N * N * 16;
  constexpr int TBYTES = MF_WAVES * NTILE * 16 * S::NR * 8;
  constexpr int SBYTES = 2 * MW * 2 * N * N * (int)sizeof(F);
  constexpr int LBYTES = QBYTES > SBYTES ? (QBYTES > TBYTES ? QBYTES : TBYTES)
                                         : (SBYTES > TBYTES ? SBYTES : TBYTES);
  __shared__ __align__(16) unsigned char lds[LBYTES];
  double* qb0 = (double*)lds;
  double* qb1 = qb0 + S::BSZ;
  double2* cs = (double2*)(qb1 + S::BSZ);  // alpha, rho^-1
  F* sb = (F*)lds;                         // [2][MW][N*N] complex: X family, then P family
  SolverFlags* fl = a.flags;
  if (fl->halted) return;
  const int tid = threadIdx.x;
  const int iter = fl->iter;  // k + 1: the small step of iteration k has counted it
  const int stop = fl->stop;
  const int slot = iter & 1;
  // the next small step and the drain read these (nothing else in this
  // kernel reads them)
  if (blockIdx.x == 0 && tid == 0) {
    fl->upd_done = iter;
    fl->upd_stop = stop;
  }
  const int lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int rows = a.rows, ns = a.ns, win = a.win;
  const size_t blk = (size_t)rows * N;
  const int k = iter - 1;
  const CF* Qin = a.Qring + (size_t)(k % win) * blk;
  CF* Qout = a.Qring + (size_t)((k + 1) % win) * blk;
  const int tile0 = (blockIdx.x * MF_WAVES + wave) * NTILE;
  unsigned long long mask =
      __ballot(lane < ns && fl->win_j[slot][lane] > 0 && (fl->win_flush[slot][lane] || stop));

  // coefficients of the Q step: B0 = rho^-1, B1 = -alpha rho^-1
  for (int e = tid; e < N * N; e += BMS_WG) {
    cs[e] = a.alpha[e];
    cs[N * N + e] = a.rhoinv[e];
  }
  __syncthreads();
  for (int e = tid; e < N * N; e += BMS_WG) {
    int i = e / N, j = e - (e / N) * N;
    double2 t = make_double2(0.0, 0.0);
    for (int kk = 0; kk < N; ++kk) t = cfma(cs[i * N + kk], cs[N * N + kk * N + j], t);
    if constexpr (N == 16) {
      // complex matrices for the three-product form (qb0: rho^-1, then -alpha rho^-1)
      qb0[2 * e] = cs[N * N + e].x;
      qb0[2 * e + 1] = cs[N * N + e].y;
      qb0[2 * N * N + 2 * e] = -t.x;
      qb0[2 * N * N + 2 * e + 1] = -t.y;
    } else {
      bput<N>(qb0, i, j, cs[N * N + e]);
      bput<N>(qb1, i, j, make_double2(-t.x, -t.y));
    }
  }
  __syncthreads();
  dx4 qd[NTILE][S::NT];
  if constexpr (N == 16) {
    double av[NTILE][S::KS], wv[NTILE][S::KS];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      const int r0 = (tile0 + t) * 16;
      aload<N>(Qin, r0 + c, rows, g, av[t]);
      aload<N>(a.W, r0 + c, rows, g, wv[t]);
    }
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      dx4 d3[3] = {dx4{0.0, 0.0, 0.0, 0.0}, dx4{0.0, 0.0, 0.0, 0.0}, dx4{0.0, 0.0, 0.0, 0.0}};
      mfma3<double>(d3, av[t], qb0, g, c);
      mfma3<double>(d3, wv[t], qb0 + 2 * N * N, g, c);
      qd[t][0] = mfma3_re(d3);
      qd[t][1] = mfma3_im(d3);
    }
  } else {
    double b0[S::KS][S::NT], b1[S::KS][S::NT];
    double av[NTILE][S::KS], wv[NTILE][S::KS];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      const int r0 = (tile0 + t) * 16;
      aload<N>(Qin, r0 + c, rows, g, av[t]);
      aload<N>(a.W, r0 + c, rows, g, wv[t]);
    }
    bload<N>(qb0, lane, b0);
    bload<N>(qb1, lane, b1);
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt) qd[t][nt] = dx4{0.0, 0.0, 0.0, 0.0};
      mfma_acc<N>(qd[t], av[t], b0);
      mfma_acc<N>(qd[t], wv[t], b1);
    }
  }
  // every lane of the wave has read its Q tiles before any is overwritten
  // (win = 1: Q_{k+1} replaces Q_k in place)
#pragma unroll
  for (int t = 0; t < NTILE; ++t) dstore<N, double>(Qout, (tile0 + t) * 16, rows, g, c, qd[t]);
  __syncthreads();  // the Q-step LDS is reused below
  // Q_{k+1} in the shift-update layout and precision: the same registers in
  // FP64; in FP32 rounded and moved to the f32 row mapping through LDS
  VF qn[NTILE][S::NT];
  if constexpr (sizeof(F) == 8) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt) qn[t][nt] = qd[t][nt];
  } else {
    double* tq = (double*)lds + wave * (NTILE * 16 * S::NR);
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt)
#pragma unroll
        for (int p = 0; p < 4; ++p)
          tq[(t * 16 + Mf<double>::row(g, p)) * S::NR + nt * 16 + c] = qd[t][nt][p];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NTILE; ++t)
#pragma unroll
      for (int nt = 0; nt < S::NT; ++nt)
#pragma unroll
        for (int p = 0; p < 4; ++p)
          qn[t][nt][p] = (F)tq[(t * 16 + Mf<F>::row(g, p)) * S::NR + nt * 16 + c];
    __syncthreads();  // the shift coefficients overwrite this LDS
  }

  // the P and X tiles of a shift (the next shift's P, and for n = 8 its X,
  // are loaded while the current one finishes; for n = 16 X is loaded after
  // the products, which keeps the three-accumulator form at three waves per
  // SIMD with 16 bytes of spills outside the product loop)
  F pa[NTILE][S::KS];
  VF xa[NTILE][S::NT];
  auto fetch = [&](int s, int t) {
    const int r0 = (tile0 + t) * 16;
    aload<N>(a.P + (size_t)s * blk, r0 + c, rows, g, pa[t]);
    if constexpr (N != 16) dload<N, F>(a.X + (size_t)a.xidx[s] * blk, r0, rows, g, c, xa[t]);
  };
  int s = mask ? __ffsll((long long)mask) - 1 : -1;
  if (s >= 0) {
#pragma unroll
    for (int t = 0; t < NTILE; ++t) fetch(s, t);
  }
  constexpr size_t FAM = (size_t)BMS_MAX_WIN * N * N;  // one family in Wm
  while (s >= 0) {
    mask &= mask - 1;
    const int s2 = mask ? __ffsll((long long)mask) - 1 : -1;
    const int j = __builtin_amdgcn_readfirstlane(fl->win_j[slot][s]);
    // the window's 2j coefficient matrices into LDS (complex n x n, the X
    // family, then the P family MW matrices further)
    const CF* wm = a.Wm + (size_t)s * 2 * FAM;
    lds_copy(wm, sb, j * N * N * (int)sizeof(CF), wave, lane);
    lds_copy(wm + FAM, sb + 2 * MW * N * N, j * N * N * (int)sizeof(CF), wave, lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const F* bx = sb;
    const F* bp = sb + 2 * MW * N * N;
    CF* X = a.X + (size_t)a.xidx[s] * blk;
    CF* P = a.P + (size_t)s * blk;
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
      const int r0 = (tile0 + t) * 16;
      constexpr int NACC = N == 16 ? 3 : S::NT;  // accumulators of one product family
      VF pn[NACC], dx[NACC];
#pragma unroll
      for (int nt = 0; nt < NACC; ++nt) {
        pn[nt] = (N == 16 || nt >= S::NT) ? VF{0, 0, 0, 0} : qn[t][nt];
        dx[nt] = VF{0, 0, 0, 0};
      }
      // ring buffers Q_{k-j+2} .. Q_k, two in flight
      F qa[2][S::KS];
      if (j >= 2) aload<N>(a.Qring + (size_t)((k - j + 2) % win) * blk, r0 + c, rows, g, qa[0]);
      // the increment is formed on its own and added to X once, so X (large
      // next to one window's increment) is rounded once
      auto prod = [&](const F(&av)[S::KS], int m) {
        if constexpr (N == 16) {
          mfma3<F>(dx, av, bx + (size_t)m * 2 * N * N, g, c);
          mfma3<F>(pn, av, bp + (size_t)m * 2 * N * N, g, c);
        } else {
          mfma_acc_c<N>(dx, av, bx + (size_t)m * 2 * N * N, g, c);
          mfma_acc_c<N>(pn, av, bp + (size_t)m * 2 * N * N, g, c);
        }
      };
      prod(pa[t], 0);
#pragma unroll
      for (int i = 0; i < MW - 1; ++i) {
        if (i < j - 1) {
          if (i + 1 < j - 1)
            aload<N>(a.Qring + (size_t)((k - j + 3 + i) % win) * blk, r0 + c, rows, g,
                     qa[(i + 1) & 1]);
          prod(qa[i & 1], i + 1);
        }
      }
      if constexpr (N == 16) {
        dload<N, F>(X, r0, rows, g, c, xa[t]);
        xa[t][0] += mfma3_re(dx);
        xa[t][1] += mfma3_im(dx);
        const VF pst[S::NT] = {qn[t][0] + mfma3_re(pn), qn[t][1] + mfma3_im(pn)};
        dstore<N, F>(X, r0, rows, g, c, xa[t]);
        dstore<N, F>(P, r0, rows, g, c, pst);
      } else {
#pragma unroll
        for (int nt = 0; nt < S::NT; ++nt) xa[t][nt] += dx[nt];
        dstore<N, F>(X, r0, rows, g, c, xa[t]);
        dstore<N, F>(P, r0, rows, g, c, pn);
      }
      if (s2 >= 0) fetch(s2, t);
    }
    s = s2;
    __syncthreads();  // every wave is done with this shift's coefficients
  }
}

// After the last iteration: every update window still open (the solve ended
// without its update applying it) is applied to X,
//   X += P Cx + sum_{i < j-1} Q_{k-j+2+i} Ex_i
// with the FP64 window state of the last update that ran (k = its iteration).
// One thread per complex entry of a row block.
template <typename F>
__global__ __launch_bounds__(BMS_WG) void k_update_drain(UpdateArgs<F, F> a) {
  using CF = cplx<F>;
  const SolverFlags* fl = a.flags;
  const int u = fl->upd_done;
  if (u < 0 || fl->upd_stop) return;
  const int slot = u & 1, k = u - 1, win = a.win;
  const int n = a.n, ns = a.ns;
  const size_t blk = (size_t)a.rows * n, nn = (size_t)n * n;
  const size_t fam = (size_t)BMS_MAX_WIN * nn;
  const size_t e = (size_t)blockIdx.x * BMS_WG + threadIdx.x;
  if (e >= blk) return;
  const size_t row = e / n;
  const int col = (int)(e - row * n);
  for (int s = 0; s < ns; ++s) {
    const int j = fl->win_j[slot][s];
    if (j == 0 || fl->win_flush[slot][s]) continue;
    const double2* xf = a.wst + (size_t)(slot * ns + s) * 2 * fam;
    const CF* P = a.P + (size_t)s * blk + row * n;
    double2 acc = make_double2(0, 0);
    for (int kk = 0; kk < n; ++kk) acc = cfma(to_d(P[kk]), xf[(size_t)kk * n + col], acc);
    for (int i = 0; i < j - 1; ++i) {
      const CF* Q = a.Qring + (size_t)((k - j + 2 + i) % win) * blk + row * n;
      const double2* ex = xf + (size_t)(i + 1) * nn;
      for (int kk = 0; kk < n; ++kk) acc = cfma(to_d(Q[kk]), ex[(size_t)kk * n + col], acc);
    }
    CF* X = a.X + (size_t)a.xidx[s] * blk + e;
    *X = cadd(*X, from_d<CF>(acc));
  }
}

template <typename F, int N, int NTILE>
hipError_t launch_mf(hipStream_t st, const UpdateArgs<F, F>& a) {
  int tiles = (a.rows + 15) / 16;
  int waves = (tiles + NTILE - 1) / NTILE;
  int blocks = (waves + MF_WAVES - 1) / MF_WAVES;
  k_update_mfma<F, N, NTILE><<<blocks, BMS_WG, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace

bool update_mfma_supported(int n) { return n == 8 || n == 16; }

template <typename F>
int update_mfma_max_win() {
  return MfWin<F>::MW;
}

// two_tiles: two 16-row tiles per wave instead of one
template <typename F>
hipError_t launch_update_mfma(hipStream_t st, const UpdateArgs<F, F>& a, bool two_tiles) {
  switch (a.n) {
    case 16: return two_tiles ? launch_mf<F, 16, 2>(st, a) : launch_mf<F, 16, 1>(st, a);
    case 8: return two_tiles ? launch_mf<F, 8, 2>(st, a) : launch_mf<F, 8, 1>(st, a);
    default: return hipErrorInvalidValue;
  }
}

template <typename F>
hipError_t launch_update_drain(hipStream_t st, const UpdateArgs<F, F>& a) {
  const size_t blk = (size_t)a.rows * a.n;
  k_update_drain<F><<<(unsigned)((blk + BMS_WG - 1) / BMS_WG), BMS_WG, 0, st>>>(a);
  return hipGetLastError();
}

template hipError_t launch_update_mfma<double>(hipStream_t, const UpdateArgs<double, double>&,
                                               bool);
template hipError_t launch_update_mfma<float>(hipStream_t, const UpdateArgs<float, float>&, bool);
template hipError_t launch_update_drain<double>(hipStream_t, const UpdateArgs<double, double>&);
template hipError_t launch_update_drain<float>(hipStream_t, const UpdateArgs<float, float>&);
template int update_mfma_max_win<double>();
template int update_mfma_max_win<float>();
