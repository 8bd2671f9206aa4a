// Gauge import and the multi-RHS staggered half hop (the block Dirac operator
// of Sec. III-IV: one application serves all n pseudofermion columns).
#include <cstring>

#include "internal.h"

namespace {

struct Bc {
  int b[4];
};

// U[mu][idx][a][b] complex128 -> per output parity p and cb site s the 8 links
//   k = mu     :  +1/2 eta_mu(x) bf U_mu(x)              (hop to x+mu)
//   k = 4 + mu :  -1/2 eta_mu(x) bb U_mu(x-mu)^dag       (hop to x-mu)
// bf / bb = bc[mu] if that hop crosses the boundary. FP64 and FP32 copies.
// With r64 set, also the two-row copies (entries 0..5 of each link, FP64 and
// FP32), bit k of sign[p][s] set when link k's scale c (+-1/2) is negative,
// and in *dev the largest difference, over the links and the parts of their
// entries, between a third row and the one the first two give for an SU(3)
// matrix, row2(c V) = conj(row0 x row1) / c (+inf if not finite). A
// non-negative double orders like its bit pattern, so an integer atomic
// maximum of the bits keeps it.
__device__ __forceinline__ void store_link(const double2 (&v)[9], double f, uint32_t s, int k,
                                           size_t pbase, size_t rbase, int sbl, double2* l64,
                                           float2* l32, double2* r64, float2* r32,
                                           unsigned long long* dev, uint32_t& mask) {
  for (int e = 0; e < 9; ++e) {
    const size_t o = pbase + link_off(s, k, e, sbl);
    l64[o] = v[e];
    l32[o] = make_float2((float)v[e].x, (float)v[e].y);
  }
  if (!r64) return;
  for (int e = 0; e < 6; ++e) {
    const size_t o = rbase + link_off(s, k, e, sbl, 48, 6);
    r64[o] = v[e];
    r32[o] = make_float2((float)v[e].x, (float)v[e].y);
  }
  if (f < 0) mask |= 1u << k;
  const double inv = 1.0 / f;
  double d = 0;
  for (int b = 0; b < 3; ++b) {
    const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
    const double2 x = csub(cmul(v[b1], v[3 + b2]), cmul(v[b2], v[3 + b1]));
    const double2 r = cscale(cconj(x), inv);
    const double dx = fabs(r.x - v[6 + b].x), dy = fabs(r.y - v[6 + b].y);
    d = dx > d ? dx : d;
    d = dy > d ? dy : d;
    if (!(dx == dx) || !(dy == dy)) d = __builtin_huge_val();
  }
  if (d > 0) atomicMax(dev, (unsigned long long)__double_as_longlong(d));
}

__global__ __launch_bounds__(BMS_WG) void k_gauge_import(
    const double2* __restrict__ U, double2* __restrict__ l64, float2* __restrict__ l32,
    double2* __restrict__ r64, float2* __restrict__ r32, uint32_t* __restrict__ sign,
    unsigned long long* __restrict__ dev, Geom g, Bc bc, int sbl, int nblk, int vol) {
  uint32_t tid = blockIdx.x * BMS_WG + threadIdx.x;
  if (tid >= 2u * (uint32_t)g.vh) return;
  int par = tid >= (uint32_t)g.vh;
  uint32_t s = tid - (par ? g.vh : 0);
  SiteCoord c = site_coords(s, g, par);
  int co[4] = {c.x, c.y, c.z, c.t};
  const size_t pbase = (size_t)par * nblk * 72 << sbl;
  const size_t rbase = (size_t)par * nblk * 48 << sbl;
  auto lex = [&](const int* q) { return q[0] + g.L[0] * (q[1] + g.L[1] * (q[2] + g.L[2] * q[3])); };
  int idx = lex(co);
  uint32_t mask = 0;
  for (int mu = 0; mu < 4; ++mu) {
    int esum = 0;
    for (int nu = 0; nu < mu; ++nu) esum += co[nu];
    double eta = (esum & 1) ? -0.5 : 0.5;
    double2 v[9];
    // forward
    const double ff = eta * ((co[mu] == g.L[mu] - 1) ? bc.b[mu] : 1);
    const double2* uf = U + ((size_t)mu * vol + idx) * 9;
    for (int e = 0; e < 9; ++e) v[e] = cscale(uf[e], ff);
    store_link(v, ff, s, mu, pbase, rbase, sbl, l64, l32, r64, r32, dev, mask);
    // backward: daggered link of the neighbour x - mu
    int nb[4] = {co[0], co[1], co[2], co[3]};
    nb[mu] = co[mu] == 0 ? g.L[mu] - 1 : co[mu] - 1;
    const double fb = -eta * ((co[mu] == 0) ? bc.b[mu] : 1);
    const double2* ub = U + ((size_t)mu * vol + lex(nb)) * 9;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v[3 * a + b] = cscale(cconj(ub[3 * b + a]), fb);
    store_link(v, fb, s, 4 + mu, pbase, rbase, sbl, l64, l32, r64, r32, dev, mask);
  }
  if (sign) sign[(size_t)par * g.vh + s] = mask;
}

// Signed distance of hop k: one step forward (0..3) and back (4..7), for the
// improved operator three steps forward (8..11) and back (12..15).
__device__ __forceinline__ int hop_dist(int k) {
  return k < 4 ? 1 : (k < 8 ? -1 : (k < 12 ? 3 : -3));
}

// The improved operator (all extents >= 4): per output parity p and cb site
// s the 16 links of its half hop,
//   k = mu      :  +1/2 eta_mu(x) bf  V_mu(x)                (to x + mu)
//   k = 4 + mu  :  -1/2 eta_mu(x) bb  V_mu(x - mu)^dag       (to x - mu)
//   k = 8 + mu  :  +1/2 eta_mu(x) b3f W_mu(x)                (to x + 3 mu)
//   k = 12 + mu :  -1/2 eta_mu(x) b3b W_mu(x - 3 mu)^dag     (to x - 3 mu)
// b3f = bc[mu] when x + 3 mu wraps (x_mu >= L_mu - 3), b3b when x - 3 mu
// wraps (x_mu < 3): with L_mu >= 4 a three-hop wraps at most once.
__global__ __launch_bounds__(BMS_WG) void k_gauge_import_improved(
    const double2* __restrict__ V, const double2* __restrict__ W, double2* __restrict__ l64,
    float2* __restrict__ l32, Geom g, Bc bc, int sbl, int nblk, int vol) {
  uint32_t tid = blockIdx.x * BMS_WG + threadIdx.x;
  if (tid >= 2u * (uint32_t)g.vh) return;
  const int par = tid >= (uint32_t)g.vh;
  const uint32_t s = tid - (par ? g.vh : 0);
  const int per = 9 * 16;
  SiteCoord c = site_coords(s, g, par);
  int co[4] = {c.x, c.y, c.z, c.t};
  const size_t pbase = (size_t)par * nblk * per << sbl;
  auto lex = [&](const int* q) { return q[0] + g.L[0] * (q[1] + g.L[1] * (q[2] + g.L[2] * q[3])); };
  const int idx = lex(co);
  for (int mu = 0; mu < 4; ++mu) {
    int esum = 0;
    for (int nu = 0; nu < mu; ++nu) esum += co[nu];
    const double eta = (esum & 1) ? -0.5 : 0.5;
    for (int h = 0; h < 2; ++h) {  // h = 0: one-hop V, h = 1: three-hop W
      const int dist = h ? 3 : 1;
      const double2* F = h ? W : V;
      const double ff = eta * ((co[mu] + dist >= g.L[mu]) ? bc.b[mu] : 1);
      const double2* uf = F + ((size_t)mu * vol + idx) * 9;
      for (int e = 0; e < 9; ++e) {
        double2 v = cscale(uf[e], ff);
        size_t o = pbase + link_off(s, 8 * h + mu, e, sbl, per);
        l64[o] = v;
        l32[o] = make_float2((float)v.x, (float)v.y);
      }
      int nb[4] = {co[0], co[1], co[2], co[3]};
      nb[mu] = co[mu] - dist < 0 ? co[mu] - dist + g.L[mu] : co[mu] - dist;
      const double fb = -eta * ((co[mu] - dist < 0) ? bc.b[mu] : 1);
      const double2* ub = F + ((size_t)mu * vol + lex(nb)) * 9;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double2 v = cscale(cconj(ub[3 * b + a]), fb);
          size_t o = pbase + link_off(s, 8 * h + 4 + mu, 3 * a + b, sbl, per);
          l64[o] = v;
          l32[o] = make_float2((float)v.x, (float)v.y);
        }
    }
  }
}

// A link element, loaded with the non-temporal hint when NT (the links are
// read once per half hop; the hint keeps them from displacing the input
// block's neighbour columns in L2).
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ double2 link_ld(const double2* p) {
  if (!NT) return *p;
  const d2v v = __builtin_nontemporal_load((const d2v*)p);
  return make_double2(v.x, v.y);
}
template <bool NT>
__device__ __forceinline__ float2 link_ld(const float2* p) {
  if (!NT) return *p;
  const f2v v = __builtin_nontemporal_load((const f2v*)p);
  return make_float2(v.x, v.y);
}

// Third row of a link kept as two rows: row2 = conj(row0 x row1) / c with the
// link's scale c = +-1/2 (neg: bit k of the site's sign mask).
template <typename C>
__device__ __forceinline__ void link_row2(C (&l)[9], bool neg) {
  using T = decltype(C().x);
  const T f = neg ? (T)-2 : (T)2;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int b1 = (b + 1) % 3, b2 = (b + 2) % 3;
    l[6 + b] = cscale(cconj(csub(cmul(l[b1], l[3 + b2]), cmul(l[b2], l[3 + b1]))), f);
  }
}

// Tiled traversal. A tile is hx x ty x tz x tt checkerboard sites (whole
// x-rows); the tiles of one (y, z) pencil are walked along t. Work-groups go
// to the 8 XCDs in turn (work-group b to XCD b % 8); XCD x takes pencils x,
// x + 8, ... and runs its work-groups tile after tile, so a tile's
// t-neighbour slices were just read by the previous tile on the same XCD and
// only the y and z faces come from beyond that XCD's L2.
struct HopTiles {
  int on;            // 0: natural order (the kernels then ignore the plan)
  int ty, tz, tt;    // tile extent in y, z, t
  int npy;           // pencils along y (Ly / ty)
  int tpp;           // tiles per pencil (Lt / tt)
  int bpt;           // work-groups per tile
  int spb;           // sites per work-group
};

// first checkerboard site of block b of the tiled order (block b belongs to
// XCD b % 8; blocks of m.spb sites)
__device__ __forceinline__ uint32_t hop_block_site(const HopTiles& m, const Geom& g, uint32_t b) {
  const uint32_t x = b & 7, j = b >> 3;
  const uint32_t per_pencil = (uint32_t)(m.bpt * m.tpp);
  const uint32_t pencil = x + 8u * (j / per_pencil);
  const uint32_t jt = j % per_pencil;
  const uint32_t tile_t = jt / (uint32_t)m.bpt, bit = jt % (uint32_t)m.bpt;
  const uint32_t py = pencil % (uint32_t)m.npy, pz = pencil / (uint32_t)m.npy;
  // local index of the first site inside the tile (x-rows of hx sites, then y, z, t)
  const uint32_t li = bit * (uint32_t)m.spb;
  const uint32_t r = li / (uint32_t)g.hx;  // whole rows: spb is a multiple of hx
  const uint32_t yl = r % (uint32_t)m.ty, r2 = r / (uint32_t)m.ty;
  const uint32_t zl = r2 % (uint32_t)m.tz, tl = r2 / (uint32_t)m.tz;
  const uint32_t y = py * m.ty + yl, z = pz * m.tz + zl, t = tile_t * m.tt + tl;
  return (uint32_t)g.hx * (y + (uint32_t)g.L[1] * (z + (uint32_t)g.L[2] * t));
}

// first checkerboard site of this work-group's sites
__device__ __forceinline__ uint32_t hop_first_site(const HopTiles& m, const Geom& g) {
  return hop_block_site(m, g, blockIdx.x);
}

// out(s) = b * sum_k L_k(s) in(nbr_k(s)) + a * aux(s) on n columns.
// One thread per (site, column group g): the n/R threads of a site share its
// links (the block operator reads each link once per n columns) and each link
// element is reused across the thread's R columns g, g + n/R, g + 2n/R, ...
// In FP64 the columns are interleaved this way, so that every load and store
// instruction touches one contiguous run per site (the site's threads read
// neighbouring columns) and a wave touches as few cache lines as the bytes
// allow. In FP32 a thread's R columns are consecutive instead (g*R .. g*R+R-1),
// which the compiler loads as 16-byte vectors.
// EPL: link entries stored, 9, or 6 for SU(3) links kept as two rows (the
// third rebuilt from them and the site's sign mask `sgn`).
template <typename T, int R, bool NT, int NL, int EPL>
__global__ __launch_bounds__(BMS_WG) void k_hop(const cplx<T>* __restrict__ links,
                                                const cplx<T>* __restrict__ in,
                                                cplx<T>* __restrict__ out,
                                                const cplx<T>* __restrict__ aux, T a, T b, Geom g,
                                                int n, FastDiv dgrp, int par, int sbl,
                                                const int* __restrict__ skip, HopTiles tiles,
                                                const uint32_t* __restrict__ sgn) {
  using C = cplx<T>;
  if (skip && *skip) return;
  const uint32_t ngrp = dgrp.d;  // n / R column groups per site
  uint32_t tid = blockIdx.x * BMS_WG + threadIdx.x;
  if (tid >= (uint32_t)g.vh * ngrp) return;
  uint32_t s, grp;
  if (tiles.on) {
    // BMS_WG / ngrp consecutive sites (whole x-rows) of a tile
    const uint32_t ls = fdiv(threadIdx.x, dgrp);
    s = hop_first_site(tiles, g) + ls;
    grp = threadIdx.x - ls * ngrp;
  } else {
    s = fdiv(tid, dgrp);
    grp = tid - s * ngrp;
  }
  constexpr bool kInterleave = sizeof(T) == 8;
  const int cstep = kInterleave ? (int)ngrp : 1;  // column stride of a thread
  const int j0 = (int)grp * (kInterleave ? 1 : R);  // its first column
  SiteCoord c = site_coords(s, g, par);
  C acc[3][R];
#pragma unroll
  for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[a3][r] = czero<C>();
  const size_t st = (size_t)1 << sbl;
  const uint32_t msk = EPL == 6 ? sgn[s] : 0u;
#pragma unroll 2
  for (int k = 0; k < NL; ++k) {
    int mu = k & 3;
    int nb = neighbour_cb((int)s, c, g, mu, hop_dist(k));
    const C* src = in + (size_t)nb * 3 * n + j0;
    const C* L = links + link_off(s, k, 0, sbl, EPL * NL, EPL);
    C l[9], v[3][R];
#pragma unroll
    for (int e = 0; e < EPL; ++e) l[e] = link_ld<NT>(L + e * st);
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int r = 0; r < R; ++r) v[cb][r] = src[cb * n + r * cstep];
    // all of the hop's loads in flight before the first use (as in k_hop_q)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (EPL == 6) link_row2(l, (msk >> k) & 1);
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[a3][r] = cfma(l[3 * a3 + cb], v[cb][r], acc[a3][r]);
  }
  size_t o = (size_t)s * 3 * n + j0;
#pragma unroll
  for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      size_t oo = o + a3 * n + r * cstep;
      out[oo] = aux ? cadd(cscale(aux[oo], a), cscale(acc[a3][r], b)) : cscale(acc[a3][r], b);
    }
}

// Broadcast a value from lane Q of each group of four lanes to the whole group
// (DPP quad permute [Q, Q, Q, Q]).
template <int Q>
__device__ __forceinline__ float quad_bcast(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), Q * 0x55,
                                                              0xF, 0xF, false));
}
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
  long long u = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)u, Q * 0x55, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), Q * 0x55, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The same half hop with four threads per site (n = 4R columns) that share
// the site's links: for each hop, thread q of the site loads link elements q,
// q+4 (and thread 0 element 8), a third of the link load instructions, and
// element e reaches the other three threads of the quad by a DPP broadcast
// from lane e % 4. Columns as in k_hop (interleaved in FP64, consecutive in
// FP32).
// With links kept as two rows (EPL = 6) thread q loads entries q and 4 + q%2,
// and every thread rebuilds the third row.
template <typename T, int R, bool NT, int NL, int EPL>
__global__ __launch_bounds__(BMS_WG) void k_hop_q(const cplx<T>* __restrict__ links,
                                                  const cplx<T>* __restrict__ in,
                                                  cplx<T>* __restrict__ out,
                                                  const cplx<T>* __restrict__ aux, T a, T b,
                                                  Geom g, int n, int par, int sbl,
                                                  const int* __restrict__ skip, HopTiles tiles,
                                                  const uint32_t* __restrict__ sgn) {
  using C = cplx<T>;
  if (skip && *skip) return;
  // whole quads leave together (4 * Vh threads), so every DPP source lane is active
  if (blockIdx.x * BMS_WG + threadIdx.x >= (uint32_t)g.vh * 4) return;
  const uint32_t s = tiles.on ? hop_first_site(tiles, g) + (threadIdx.x >> 2)
                              : (blockIdx.x * BMS_WG + threadIdx.x) >> 2;
  const int q = (int)(threadIdx.x & 3);
  constexpr bool kInterleave = sizeof(T) == 8;
  const int cstep = kInterleave ? 4 : 1;
  const int j0 = kInterleave ? q : q * R;
  // second and third entries this thread fetches: 9 entries, q + 4 and
  // (thread 0) 8, others repeat q + 4; 6 entries, 4 + q%2
  const int e1 = EPL == 6 ? 4 + (q & 1) : q + 4;
  const int e2 = q == 0 ? 8 : q + 4;
  const uint32_t msk = EPL == 6 ? sgn[s] : 0u;
  SiteCoord c = site_coords(s, g, par);
  C acc[3][R];
#pragma unroll
  for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
    for (int r = 0; r < R; ++r) acc[a3][r] = czero<C>();
  const size_t st = (size_t)1 << sbl;
  // hop k's link entries of this thread, and hop k's contribution to acc
  auto link_load = [&](int k, C& t0, C& t1, C& t2) {
    const C* L = links + link_off(s, k, 0, sbl, EPL * NL, EPL);
    t0 = link_ld<NT>(L + q * st);
    t1 = link_ld<NT>(L + e1 * st);
    t2 = EPL == 9 ? link_ld<NT>(L + e2 * st) : t1;
  };
  auto accumulate = [&](int k, const C (&v)[3][R], C t0, C t1, C t2) {
    C l[9];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const C own = e < 4 ? t0 : (e < 8 ? t1 : t2);
      switch (e & 3) {
        case 0: l[e].x = quad_bcast<0>(own.x); l[e].y = quad_bcast<0>(own.y); break;
        case 1: l[e].x = quad_bcast<1>(own.x); l[e].y = quad_bcast<1>(own.y); break;
        case 2: l[e].x = quad_bcast<2>(own.x); l[e].y = quad_bcast<2>(own.y); break;
        default: l[e].x = quad_bcast<3>(own.x); l[e].y = quad_bcast<3>(own.y);
      }
    }
    if constexpr (EPL == 6) link_row2(l, (msk >> k) & 1);
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[a3][r] = cfma(l[3 * a3 + cb], v[cb][r], acc[a3][r]);
  };
  auto col_load = [&](int nb, C (&v)[3][R]) {
    const C* src = in + (size_t)nb * 3 * n + j0;
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int r = 0; r < R; ++r) v[cb][r] = src[cb * n + r * cstep];
  };
  // The two x hops first. Along an x-row the -x neighbour of a site is the
  // +x neighbour of the site before it (with the row's wrap, of the row's
  // last site), so where the wave holds that site (four lanes down, the same
  // q) the -x columns come from its +x columns by cross-lane moves instead of
  // a second read from L2; the other lanes (first site of the wave, rows that
  // do not fill the wave) load them.
  {
    const int lane = (int)(threadIdx.x & 63);
    const bool full = blockIdx.x * BMS_WG + (threadIdx.x & ~63u) + 64 <= (uint32_t)g.vh * 4;
    const int from = (lane - 4) & 63;
    const int nb0 = neighbour_cb((int)s, c, g, 0, 1), nb4 = neighbour_cb((int)s, c, g, 0, -1);
    C t0, t1, t2, v[3][R];
    link_load(0, t0, t1, t2);
    col_load(nb0, v);
    __builtin_amdgcn_sched_barrier(0);
    C u0, u1, u2, w[3][R];
    link_load(4, u0, u1, u2);
    const int there = __shfl(nb0, from);
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        w[cb][r].x = __shfl(v[cb][r].x, from);
        w[cb][r].y = __shfl(v[cb][r].y, from);
      }
    if (!((lane >= 4 || full) && there == nb4)) col_load(nb4, w);
    accumulate(0, v, t0, t1, t2);
    accumulate(4, w, u0, u1, u2);
  }
  // The other hops: every load of a hop (three link elements, 3R input
  // columns) is issued before any of them is used; the scheduling barrier
  // keeps the scheduler from spreading them next to their uses, which leaves
  // about two in flight.
#pragma unroll 2
  for (int kk = 0; kk < NL - 2; ++kk) {
    const int k = kk + (kk < 3 ? 1 : 2);
    const int nb = neighbour_cb((int)s, c, g, k & 3, hop_dist(k));
    C t0, t1, t2, v[3][R];
    link_load(k, t0, t1, t2);
    col_load(nb, v);
    __builtin_amdgcn_sched_barrier(0);
    accumulate(k, v, t0, t1, t2);
  }
  const size_t o = (size_t)s * 3 * n + j0;
#pragma unroll
  for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
    for (int r = 0; r < R; ++r) {
      size_t oo = o + a3 * n + r * cstep;
      out[oo] = aux ? cadd(cscale(aux[oo], a), cscale(acc[a3][r], b)) : cscale(acc[a3][r], b);
    }
}


typedef __attribute__((address_space(3))) void hop_lds_void;
typedef __attribute__((address_space(1))) void hop_glob_void;
typedef float f4v __attribute__((ext_vector_type(4)));

// s_waitcnt immediate that waits until at most n vector memory operations
// are outstanding (n < 64) and leaves the other counters alone
constexpr int vm_wait(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Direct-to-LDS loads of a wave: lane l's 16 (4) bytes go to dst + 16 l
// (dst + 4 l); CP is the cache policy (2: non-temporal).
template <int CP = 0>
__device__ __forceinline__ void dma16(const void* src, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds((const hop_glob_void*)src, (hop_lds_void*)dst, 16, 0, CP);
}
template <int CP = 0>
__device__ __forceinline__ void dma4(const void* src, unsigned char* dst) {
  __builtin_amdgcn_global_load_lds((const hop_glob_void*)src, (hop_lds_void*)dst, 4, 0, CP);
}
__device__ __forceinline__ uint32_t lds_addr(const unsigned char* p) {
  return (uint32_t)(uintptr_t)(const hop_lds_void*)p;
}

// Bytes of one ring slot of k_hop_s: the neighbour columns of 16 sites for
// one hop (48 complex per site), then the link entries the wave's lanes load.
template <typename T, int EPL>
constexpr int hop_s_slot() {
  return 16 * 48 * (int)sizeof(cplx<T>) + (EPL == 9 ? 3 : 2) * (sizeof(T) == 8 ? 1024 : 512);
}
// LDS of one k_hop_s wave: D slots and the group's aux columns
template <typename T, int EPL>
constexpr int hop_s_wave_lds(int d) {
  return d * hop_s_slot<T, EPL>() + 16 * 48 * (int)sizeof(cplx<T>);
}

// The half hop at n = 16 with the next hops' loads in flight. A thread quad
// per site as in k_hop_q (FP64: columns q + 4r; FP32: columns 4q .. 4q+3).
// Every wave runs its own list of 16-site groups, hop after hop, through a
// ring of D slots in LDS: while it computes one hop from its slot, the
// neighbour columns and link entries of the next D-1 hops are on their way by
// direct-to-LDS loads (a wave's 64 lanes fill one contiguous run, so a lane
// reads back exactly what it loaded). Loads complete in issue order, so
// waiting until at most (D-1) hops of loads are outstanding completes the
// slot (any other load issued in between only lengthens the wait). Nothing
// is loaded into registers: the compiler cannot order its own waits for a
// register load against direct-to-LDS loads and would wait for all of them.
// So the epilogue's aux columns come with the group's last hop into an area
// of their own, and with two-row links the lanes q = 2, 3 of a site, whose
// second link entry only repeats that of q = 0, 1, fetch the site's sign
// mask instead. A wave touches only its own LDS: no barriers. The grid is
// persistent (a multiple of 8 work-groups): group j of XCD x (the
// work-groups b with b % 8 = x) is block 8j + x of the traversal (tiled:
// hop_block_site with 16-site blocks; natural: sites 16 (8j + x) ..), and
// the XCD's waves take its groups in turn, so they sweep the same part of
// the lattice together.
template <typename T, bool NT, int NL, int EPL, int D>
__global__ __launch_bounds__(BMS_WG) void k_hop_s(const cplx<T>* __restrict__ links,
                                                  const cplx<T>* __restrict__ in,
                                                  cplx<T>* __restrict__ out,
                                                  const cplx<T>* __restrict__ aux, T a, T b,
                                                  Geom g, int par, int sbl,
                                                  const int* __restrict__ skip, HopTiles tiles,
                                                  const uint32_t* __restrict__ sgn, int gpx) {
  using C = cplx<T>;
  constexpr int N = 16, R = 4;
  constexpr bool kF64 = sizeof(T) == 8;
  constexpr int IN = 16 * 48 * (int)sizeof(C);  // neighbour columns of one hop
  constexpr int SLOT = hop_s_slot<T, EPL>();
  constexpr int NLK = EPL == 9 ? 3 : 2;                    // link entries per lane
  constexpr int OPS = IN / 1024 + (kF64 ? NLK : 2 * NLK);  // loads per hop and wave
  constexpr int CP = NT ? 2 : 0;
  static_assert(NL % D == 0 && (D - 1) * OPS < 64, "ring depth");
  extern __shared__ __align__(16) unsigned char hs_lds[];
  if (skip && *skip) return;
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int q = lane & 3, ls = lane >> 2;
  unsigned char* ring = hs_lds + wave * hop_s_wave_lds<T, EPL>(D);
  unsigned char* auxa = ring + D * SLOT;
  const uint32_t xcd = blockIdx.x & 7;
  const uint32_t u = (blockIdx.x >> 3) * (BMS_WG / 64) + (uint32_t)wave;
  const uint32_t U = (gridDim.x >> 3) * (BMS_WG / 64);
  const int ng = u < (uint32_t)gpx ? (int)(((uint32_t)gpx - 1 - u) / U) + 1 : 0;
  const int nt = ng * NL;  // hops this wave runs
  const size_t st = (size_t)1 << sbl;
  const int e1 = EPL == 6 ? 4 + (q & 1) : q + 4;
  const int e2 = q == 0 ? 8 : q + 4;
  auto group_site = [&](int i) {
    const uint32_t bk = 8u * (u + (uint32_t)i * U) + xcd;
    return (tiles.on ? hop_block_site(tiles, g, bk) : 16u * bk) + (uint32_t)ls;
  };
  // the prefetch side: the site of the group whose hops are being requested
  uint32_t ps = 0;
  SiteCoord pc{};
  // 16 bytes of column data per lane and load: FP64 column q + 4r, FP32
  // bytes 16r .. 16r+15 of columns 4q .. 4q+3 (r < 4 in FP64, < 2 in FP32)
  auto col_ptr = [&](const C* row, int cb, int r) {
    return kF64 ? (const void*)(row + cb * N + q + 4 * r)
                : (const void*)((const char*)(row + cb * N + 4 * q) + 16 * r);
  };
  auto prefetch = [&](int i, int k, int slot) {
    if (k == 0) {
      ps = group_site(i);
      pc = site_coords(ps, g, par);
    }
    const int nb = neighbour_cb((int)ps, pc, g, k & 3, hop_dist(k));
    const C* src = in + (size_t)nb * 3 * N;
    unsigned char* dst = ring + slot * SLOT;
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int r = 0; r < IN / 3 / 1024; ++r)
        dma16(col_ptr(src, cb, r), dst + (cb * (IN / 3 / 1024) + r) * 1024);
    const C* L = links + link_off(ps, k, 0, sbl, EPL * NL, EPL);
    // two-row links: lanes q = 2, 3 fetch the sign masks (FP64: the aligned
    // 16 bytes holding the site's)
    const bool mlane = EPL == 6 && q >= 2;
    const void* le[3] = {L + q * st,
                         mlane ? (const void*)(sgn + (kF64 ? (ps & ~3u) : ps))
                               : (const void*)(L + e1 * st),
                         EPL == 9 ? L + e2 * st : L};
#pragma unroll
    for (int e = 0; e < NLK; ++e) {
      if constexpr (kF64) {
        dma16<CP>(le[e], dst + IN + e * 1024);
      } else {
        dma4<CP>(le[e], dst + IN + e * 512);
        dma4<CP>(e == 1 && mlane ? le[e] : (const void*)((const float*)le[e] + 1),
                 dst + IN + e * 512 + 256);
      }
    }
    if (aux && k == NL - 1) {
      const C* ar = aux + (size_t)ps * 3 * N;
#pragma unroll
      for (int cb = 0; cb < 3; ++cb)
#pragma unroll
        for (int r = 0; r < IN / 3 / 1024; ++r)
          dma16(col_ptr(ar, cb, r), auxa + (cb * (IN / 3 / 1024) + r) * 1024);
    }
  };
  // LDS reads the compiler does not see: one it sees after a direct-to-LDS
  // load makes it wait for every load in flight (it cannot tell the slots
  // apart), which would drain the ring at every hop. Each block completes
  // its reads before it ends, and its outputs are early-clobber (a read must
  // not land in the address register the later reads of the block use).
  // 12 (FP64) or 6 (FP32) 16-byte columns per lane from `cols`:
  auto read_cols = [&](const unsigned char* cols, C (&v)[3][R]) {
    const uint32_t la = lds_addr(cols + 16 * lane);
    if constexpr (kF64) {
      d2v w[12];
      asm volatile(
          "ds_read_b128 %0, %12\n ds_read_b128 %1, %12 offset:1024\n"
          "ds_read_b128 %2, %12 offset:2048\n ds_read_b128 %3, %12 offset:3072\n"
          "ds_read_b128 %4, %12 offset:4096\n ds_read_b128 %5, %12 offset:5120\n"
          "ds_read_b128 %6, %12 offset:6144\n ds_read_b128 %7, %12 offset:7168\n"
          "ds_read_b128 %8, %12 offset:8192\n ds_read_b128 %9, %12 offset:9216\n"
          "ds_read_b128 %10, %12 offset:10240\n ds_read_b128 %11, %12 offset:11264\n"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5]),
            "=&v"(w[6]), "=&v"(w[7]), "=&v"(w[8]), "=&v"(w[9]), "=&v"(w[10]), "=&v"(w[11])
          : "v"(la));
#pragma unroll
      for (int cb = 0; cb < 3; ++cb)
#pragma unroll
        for (int r = 0; r < R; ++r) v[cb][r] = make_double2(w[cb * R + r].x, w[cb * R + r].y);
    } else {
      f4v w[6];
      asm volatile(
          "ds_read_b128 %0, %6\n ds_read_b128 %1, %6 offset:1024\n"
          "ds_read_b128 %2, %6 offset:2048\n ds_read_b128 %3, %6 offset:3072\n"
          "ds_read_b128 %4, %6 offset:4096\n ds_read_b128 %5, %6 offset:5120\n"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5])
          : "v"(la));
#pragma unroll
      for (int cb = 0; cb < 3; ++cb) {
        v[cb][0] = make_float2(w[2 * cb].x, w[2 * cb].y);
        v[cb][1] = make_float2(w[2 * cb].z, w[2 * cb].w);
        v[cb][2] = make_float2(w[2 * cb + 1].x, w[2 * cb + 1].y);
        v[cb][3] = make_float2(w[2 * cb + 1].z, w[2 * cb + 1].w);
      }
    }
  };
  uint32_t cs = 0, cmsk = 0;
  C acc[3][R];
  auto compute = [&](int i, int k, int slot) {
    const int t = i * NL + k;
    if (t + D - 1 < nt)
      __builtin_amdgcn_s_waitcnt(vm_wait((D - 1) * OPS));
    else
      __builtin_amdgcn_s_waitcnt(vm_wait(0));
    const unsigned char* sp = ring + slot * SLOT;
    C v[3][R], lt[3];
    read_cols(sp, v);
    lt[2] = lt[0];  // (a third entry only with nine-entry links)
    if constexpr (kF64) {
      d2v w[3];
      const uint32_t lb = lds_addr(sp + IN + 16 * lane);
      if constexpr (NLK == 3) {
        asm volatile(
            "ds_read_b128 %0, %3\n ds_read_b128 %1, %3 offset:1024\n"
            "ds_read_b128 %2, %3 offset:2048\n s_waitcnt lgkmcnt(0)"
            : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2])
            : "v"(lb));
      } else {
        asm volatile("ds_read_b128 %0, %2\n ds_read_b128 %1, %2 offset:1024\n s_waitcnt lgkmcnt(0)"
                     : "=&v"(w[0]), "=&v"(w[1])
                     : "v"(lb));
      }
#pragma unroll
      for (int e = 0; e < NLK; ++e) lt[e] = make_double2(w[e].x, w[e].y);
    } else {
      float w[6];
      const uint32_t lb = lds_addr(sp + IN + 4 * lane);
      if constexpr (NLK == 3) {
        asm volatile(
            "ds_read_b32 %0, %6\n ds_read_b32 %1, %6 offset:256\n"
            "ds_read_b32 %2, %6 offset:512\n ds_read_b32 %3, %6 offset:768\n"
            "ds_read_b32 %4, %6 offset:1024\n ds_read_b32 %5, %6 offset:1280\n"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3]), "=&v"(w[4]), "=&v"(w[5])
            : "v"(lb));
      } else {
        asm volatile(
            "ds_read_b32 %0, %4\n ds_read_b32 %1, %4 offset:256\n"
            "ds_read_b32 %2, %4 offset:512\n ds_read_b32 %3, %4 offset:768\n"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(w[0]), "=&v"(w[1]), "=&v"(w[2]), "=&v"(w[3])
            : "v"(lb));
      }
#pragma unroll
      for (int e = 0; e < NLK; ++e) lt[e] = make_float2(w[2 * e], w[2 * e + 1]);
    }
    if (k == 0) {
      cs = group_site(i);
      if constexpr (EPL == 6) {
        // lane q = 2 of the site holds its mask (FP64: word cs % 4 of the 16 bytes)
        uint32_t m;
        if constexpr (kF64) {
          const uint64_t lo = __builtin_bit_cast(uint64_t, lt[1].x);
          const uint64_t hi = __builtin_bit_cast(uint64_t, lt[1].y);
          const uint64_t h = (cs & 2) ? hi : lo;
          m = (uint32_t)((cs & 1) ? (h >> 32) : h);
        } else {
          m = __builtin_bit_cast(uint32_t, lt[1].x);
        }
        cmsk = (uint32_t)__builtin_amdgcn_mov_dpp((int)m, 2 * 0x55, 0xF, 0xF, false);
      }
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[a3][r] = czero<C>();
    }
    C l[9];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const C own = e < 4 ? lt[0] : (e < 8 ? lt[1] : lt[2]);
      switch (e & 3) {
        case 0: l[e].x = quad_bcast<0>(own.x); l[e].y = quad_bcast<0>(own.y); break;
        case 1: l[e].x = quad_bcast<1>(own.x); l[e].y = quad_bcast<1>(own.y); break;
        case 2: l[e].x = quad_bcast<2>(own.x); l[e].y = quad_bcast<2>(own.y); break;
        default: l[e].x = quad_bcast<3>(own.x); l[e].y = quad_bcast<3>(own.y);
      }
    }
    if constexpr (EPL == 6) link_row2(l, (cmsk >> k) & 1);
#pragma unroll
    for (int cb = 0; cb < 3; ++cb)
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[a3][r] = cfma(l[3 * a3 + cb], v[cb][r], acc[a3][r]);
    if (k == NL - 1) {
      C ax[3][R];
      if (aux) read_cols(auxa, ax);
      const size_t o = (size_t)cs * 3 * N + (kF64 ? q : 4 * q);
#pragma unroll
      for (int a3 = 0; a3 < 3; ++a3)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const size_t oo = o + a3 * N + r * (kF64 ? 4 : 1);
          out[oo] = aux ? cadd(cscale(ax[a3][r], a), cscale(acc[a3][r], b)) : cscale(acc[a3][r], b);
        }
    }
  };
  if (ng == 0) return;
#pragma unroll
  for (int d = 0; d < D; ++d) prefetch(0, d, d);
  for (int i = 0; i < ng; ++i) {
    // D hops per iteration, unrolled: the ring slot of each is a constant
#pragma unroll 1
    for (int k0 = 0; k0 < NL; k0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int k = k0 + d;
        compute(i, k, d);
        // the slot's values are in registers (the reads completed) before it refills
        __builtin_amdgcn_sched_barrier(0);
        if (k + D < NL)
          prefetch(i, k + D, d);
        else if (i + 1 < ng)
          prefetch(i + 1, k + D - NL, d);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

}  // namespace

hipError_t launch_gauge_import(const bms_ctx* c, const void* U, void* l64, void* l32,
                               void* r64, void* r32, void* sign, void* dev) {
  Bc bc;
  for (int i = 0; i < 4; ++i) bc.b[i] = c->bc[i];
  uint32_t nthr = 2u * c->vh;
  k_gauge_import<<<(nthr + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>(
      (const double2*)U, (double2*)l64, (float2*)l32, (double2*)r64, (float2*)r32,
      (uint32_t*)sign, (unsigned long long*)dev, c->geom, bc, c->sbl, c->nblk, (int)c->vol);
  return hipGetLastError();
}

hipError_t launch_gauge_import_improved(const bms_ctx* c, const void* V, const void* W, void* l64,
                                        void* l32) {
  Bc bc;
  for (int i = 0; i < 4; ++i) bc.b[i] = c->bc[i];
  uint32_t nthr = 2u * c->vh;
  k_gauge_import_improved<<<(nthr + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>(
      (const double2*)V, (const double2*)W, (double2*)l64, (float2*)l32, c->geom, bc, c->sbl,
      c->nblk, (int)c->vol);
  return hipGetLastError();
}

// The tile plan for spb sites per work-group (off when the lattice does not
// divide into whole-row tiles whose (y, z) pencils split evenly over 8 XCDs).
static HopTiles hop_tiles(const bms_ctx* c, int spb, int ty, int tz, int tt) {
  HopTiles m;
  memset(&m, 0, sizeof m);
  const Geom& g = c->geom;
  if (spb % g.hx || ty % (spb / g.hx) || g.L[1] % ty || g.L[2] % tz || g.L[3] % tt) return m;
  const long tile = (long)g.hx * ty * tz * tt;
  const int np = (g.L[1] / ty) * (g.L[2] / tz);
  if (tile % spb || np % 8) return m;
  m.on = 1;
  m.ty = ty;
  m.tz = tz;
  m.tt = tt;
  m.npy = g.L[1] / ty;
  m.tpp = g.L[3] / tt;
  m.bpt = (int)(tile / spb);
  m.spb = spb;
  return m;
}

bool hop_tiling_valid(const bms_ctx* c, int n, int ty, int tz, int tt) {
  const bool quad = n == 4 || n == 8 || n == 16 || n == 32;
  const int R = (n % 4 == 0) ? 4 : ((n % 2 == 0) ? 2 : 1);
  const int spb = quad ? BMS_WG / 4 : (BMS_WG % (n / R) == 0 ? BMS_WG / (n / R) : 0);
  return spb > 0 && hop_tiles(c, spb, ty, tz, tt).on != 0;
}

// LDS a hop work-group reserves (and leaves unused) so that at most `cap`
// are resident per compute unit; 0 when that would exceed one work-group's
// limit (the cap is then not applied).
size_t hop_cap_lds(const bms_ctx* c, int cap) {
  if (cap <= 0 || c->lds_per_cu <= 0) return 0;
  const size_t lds = (size_t)c->lds_per_cu / (cap + 1) + 1;
  return c->lds_per_block > 0 && lds > (size_t)c->lds_per_block ? 0 : lds;
}

// The traversal of one half hop for this context, block width and precision.
HopPlan hop_plan(const bms_ctx* c, int n, bool fp64) {
  HopPlan p;
  const HopCfg& hc = c->hop_cfg[fp64 ? 0 : 1];
  const int hv = c->hop_variant;
  p.quad = (n == 4 || n == 8 || n == 16 || n == 32) && (hv == 1 || hv == 3 || hv < 0);
  // tile extents: the configured ones, else 8 x 8 x 4; tiled for variants 2
  // and 3, or by the configuration (ty > 0; ty = 0 keeps the natural order),
  // or by default in FP64 at n >= 16
  const bool tiled_default = fp64 && n >= 16;
  p.tiled = hv == 2 || hv == 3 || (hv < 0 && (hc.ty > 0 || (hc.ty < 0 && tiled_default)));
  p.ty = hc.ty > 0 ? hc.ty : 8;
  p.tz = hc.ty > 0 ? hc.tz : 8;
  p.tt = hc.ty > 0 ? hc.tt : 4;
  // At most `cap` resident work-groups per compute unit (by reserving LDS the
  // kernel does not use): fewer sites in flight keep the neighbours' re-reads
  // inside each XCD's L2 (at 32^4 FP64 n = 16 513 -> 455 us natural order).
  p.cap = hc.cap >= 0 ? hc.cap : (n >= 16 ? 2 : (n == 8 ? 3 : 0));
  p.nt = hc.nt > 0;
  // Variant 4 (n = 16, whole groups of 16 sites over 8 XCDs): the streamed
  // kernel, tiled unless the configuration asks for the natural order; the
  // configuration's cap is its ring depth (2 or 4 slots per wave; the
  // default 2 in FP64, 4 in FP32).
  if (hv == 4 && n == 16 && c->vh % 128 == 0) {
    // LDS of a work-group (four waves) at ring depth d; a depth that does not
    // fit falls back to 2, and if that does not fit either the quad kernel runs
    const bool two = c->links_two_rows && c->nlinks == 8;
    const auto bytes = [&](int d) {
      return (BMS_WG / 64) *
             (fp64 ? (two ? hop_s_wave_lds<double, 6>(d) : hop_s_wave_lds<double, 9>(d))
                   : (two ? hop_s_wave_lds<float, 6>(d) : hop_s_wave_lds<float, 9>(d)));
    };
    int d = hc.cap >= 4 ? 4 : (hc.cap >= 2 ? 2 : (fp64 ? 2 : 4));
    if (d == 4 && bytes(4) > c->lds_per_block) d = 2;
    if (bytes(d) <= c->lds_per_block) {
      p.stream = true;
      p.quad = false;
      p.tiled = hc.ty != 0;
      p.depth = d;
      p.cap = 0;
    }
  }
  return p;
}

template <typename T>
hipError_t launch_hop(const bms_ctx* c, int par, int n, const void* in, void* out, const void* aux,
                      double a, double b, const int* skip) {
  // SU(3) links as two rows when the field passed the import's check
  const bool two = c->links_two_rows && c->nlinks == 8;
  const DevBuf& lb = two ? (sizeof(T) == 8 ? c->links64r : c->links32r)
                         : (sizeof(T) == 8 ? c->links64 : c->links32);
  size_t pstride = (size_t)c->nblk * (two ? 6 : 9) * c->nlinks << c->sbl;
  const cplx<T>* links = (const cplx<T>*)lb.p + (size_t)par * pstride;
  const uint32_t* sgn = two ? (const uint32_t*)c->lsign.p + (size_t)par * c->vh : nullptr;
  // Variants: 0 one thread per (site, column group), 1 four threads per site
  // sharing the links (n = 4, 8, 16, 32), 2 and 3 the same in the tiled
  // traversal; the default is 1, tiled in FP64 at n >= 16. The traversal's
  // tile extents, resident cap and link-load hint come from the context's
  // hop configuration (bms_set_hop_config, bms_autotune).
  const HopPlan hp = hop_plan(c, n, sizeof(T) == 8);
  if (hp.stream) {
    // a ring of `depth` slots per wave and the group's aux columns; a
    // persistent grid of whole groups of 8 work-groups, as many per compute
    // unit as the LDS holds
    const int d = hp.depth;
    const size_t lds = (size_t)(BMS_WG / 64) *
                       (two ? hop_s_wave_lds<T, 6>(d) : hop_s_wave_lds<T, 9>(d));
    int wpc = c->lds_per_cu > 0 ? c->lds_per_cu / (int)lds : 1;
    wpc = wpc < 1 ? 1 : (wpc > 8 ? 8 : wpc);
    int nblk = (c->num_cu > 0 ? c->num_cu : 8) * wpc;
    nblk = nblk < 8 ? 8 : nblk - nblk % 8;
    const HopTiles tiles = hp.tiled ? hop_tiles(c, 16, hp.ty, hp.tz, hp.tt) : HopTiles{};
    const int gpx = c->vh / 128;
#define HOPS(NT, NL, EPL, DD)                                                              \
  k_hop_s<T, NT, NL, EPL, DD><<<nblk, BMS_WG, lds, c->stream>>>(                           \
      links, (const cplx<T>*)in, (cplx<T>*)out, (const cplx<T>*)aux, (T)a, (T)b, c->geom,  \
      par, c->sbl, skip, tiles, sgn, gpx)
#define HOPSD(NT, NL, EPL) \
  if (d == 2)              \
    HOPS(NT, NL, EPL, 2);  \
  else                     \
    HOPS(NT, NL, EPL, 4)
#define HOPSN(NT)             \
  if (c->nlinks == 16) {      \
    HOPSD(NT, 16, 9);         \
  } else if (two) {           \
    HOPSD(NT, 8, 6);          \
  } else {                    \
    HOPSD(NT, 8, 9);          \
  }
    if (hp.nt) {
      HOPSN(true)
    } else {
      HOPSN(false)
    }
#undef HOPSN
#undef HOPSD
#undef HOPS
    return hipGetLastError();
  }
  const size_t lds = hop_cap_lds(c, hp.cap);
  if (hp.quad) {
    dim3 qgrid((4u * (uint32_t)c->vh + BMS_WG - 1) / BMS_WG);
    HopTiles tiles = hp.tiled ? hop_tiles(c, BMS_WG / 4, hp.ty, hp.tz, hp.tt) : HopTiles{};
#define HOPQ(RR, NT, NL, EPL)                                                              \
  k_hop_q<T, RR, NT, NL, EPL><<<qgrid, BMS_WG, lds, c->stream>>>(                          \
      links, (const cplx<T>*)in, (cplx<T>*)out, (const cplx<T>*)aux, (T)a, (T)b, c->geom,  \
      n, par, c->sbl, skip, tiles, sgn)
#define HOPQN(RR)                                   \
  if (c->nlinks == 16) {                            \
    if (hp.nt)                                      \
      HOPQ(RR, true, 16, 9);                        \
    else                                            \
      HOPQ(RR, false, 16, 9);                       \
  } else if (two) {                                 \
    if (hp.nt)                                      \
      HOPQ(RR, true, 8, 6);                         \
    else                                            \
      HOPQ(RR, false, 8, 6);                        \
  } else if (hp.nt)                                 \
    HOPQ(RR, true, 8, 9);                           \
  else                                              \
    HOPQ(RR, false, 8, 9)
    switch (n) {
      case 4: HOPQN(1); break;
      case 8: HOPQN(2); break;
      case 16: HOPQN(4); break;
      default: HOPQN(8);
    }
#undef HOPQN
#undef HOPQ
    return hipGetLastError();
  }
  const int R = (n % 4 == 0) ? 4 : ((n % 2 == 0) ? 2 : 1);
  uint32_t ngrp = (uint32_t)(n / R);
  uint32_t nthr = (uint32_t)c->vh * ngrp;
  dim3 grid((nthr + BMS_WG - 1) / BMS_WG);
  FastDiv dg = make_fastdiv(ngrp);
  HopTiles tiles = hp.tiled && BMS_WG % ngrp == 0
                       ? hop_tiles(c, BMS_WG / (int)ngrp, hp.ty, hp.tz, hp.tt)
                       : HopTiles{};
#define HOP_LAUNCH(RR, NT, NL, EPL)                                                        \
  k_hop<T, RR, NT, NL, EPL><<<grid, BMS_WG, lds, c->stream>>>(                             \
      links, (const cplx<T>*)in, (cplx<T>*)out, (const cplx<T>*)aux, (T)a, (T)b, c->geom,  \
      n, dg, par, c->sbl, skip, tiles, sgn)
#define HOPN(RR)                                    \
  if (c->nlinks == 16) {                            \
    if (hp.nt)                                      \
      HOP_LAUNCH(RR, true, 16, 9);                  \
    else                                            \
      HOP_LAUNCH(RR, false, 16, 9);                 \
  } else if (two) {                                 \
    if (hp.nt)                                      \
      HOP_LAUNCH(RR, true, 8, 6);                   \
    else                                            \
      HOP_LAUNCH(RR, false, 8, 6);                  \
  } else if (hp.nt)                                 \
    HOP_LAUNCH(RR, true, 8, 9);                     \
  else                                              \
    HOP_LAUNCH(RR, false, 8, 9)
  if (R == 4)
    HOPN(4);
  else if (R == 2)
    HOPN(2);
  else
    HOPN(1);
#undef HOPN
#undef HOP_LAUNCH
  return hipGetLastError();
}

template hipError_t launch_hop<float>(const bms_ctx*, int, int, const void*, void*, const void*,
                                      double, double, const int*);
template hipError_t launch_hop<double>(const bms_ctx*, int, int, const void*, void*, const void*,
                                       double, double, const int*);
