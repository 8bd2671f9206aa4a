// Shared device/host helpers of the bms HIP library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define BMS_WG 256  // work-group size of the streaming kernels (4 wave64)

// ---- complex arithmetic on float2 / double2 ---------------------------------

template <typename T>
struct cplx_t;
template <>
struct cplx_t<float> {
  using type = float2;
};
template <>
struct cplx_t<double> {
  using type = double2;
};
template <typename T>
using cplx = typename cplx_t<T>::type;

template <typename C>
__host__ __device__ __forceinline__ C cmk(decltype(C().x) re, decltype(C().x) im) {
  C r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename C>
__host__ __device__ __forceinline__ C czero() {
  return cmk<C>(0, 0);
}
template <typename C>
__host__ __device__ __forceinline__ C cadd(C a, C b) {
  return cmk<C>(a.x + b.x, a.y + b.y);
}
template <typename C>
__host__ __device__ __forceinline__ C csub(C a, C b) {
  return cmk<C>(a.x - b.x, a.y - b.y);
}
template <typename C>
__host__ __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__host__ __device__ __forceinline__ C cconj(C a) {
  return cmk<C>(a.x, -a.y);
}
template <typename C, typename S>
__host__ __device__ __forceinline__ C cscale(C a, S s) {
  return cmk<C>(a.x * s, a.y * s);
}
// acc + a*b
template <typename C>
__host__ __device__ __forceinline__ C cfma(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// acc + conj(a)*b
template <typename C>
__host__ __device__ __forceinline__ C cjfma(C a, C b, C acc) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}

__device__ __forceinline__ double2 to_d(float2 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ double2 to_d(double2 a) { return a; }
template <typename C>
__device__ __forceinline__ C from_d(double2 a);
template <>
__device__ __forceinline__ float2 from_d<float2>(double2 a) {
  return make_float2((float)a.x, (float)a.y);
}
template <>
__device__ __forceinline__ double2 from_d<double2>(double2 a) {
  return a;
}

// ---- division by a runtime constant (n < 2^31) ---------------------------
// Granlund-Montgomery: q = (umulhi(n, m) + n) >> l with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1.
struct FastDiv {
  uint32_t d, m, l;
};

static inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  f.l = l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  return f;
}

__host__ __device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) {
#ifdef __HIP_DEVICE_COMPILE__
  uint32_t hi = __umulhi(n, f.m);
#else
  uint32_t hi = (uint32_t)(((uint64_t)n * f.m) >> 32);
#endif
  return (hi + n) >> f.l;
}

// ---- lattice geometry for on-the-fly neighbour indices ------------------
// Checkerboard index s of a site of parity par: idx0 = 2s = x0 + Lx*(y + ...)
// with x0 even; the site is x = x0 + ((y+z+t+par)&1).
struct Geom {
  int L[4];      // extents x,y,z,t
  int hx;        // Lx/2
  int stride[4]; // cb-index stride of a unit step in y,z,t (stride[0] unused)
  int vh;        // V/2
  FastDiv d_hx, d_ly, d_lz;
};

struct SiteCoord {
  int x, y, z, t, xh;  // xh = x0/2 (cb offset inside the x-row)
};

__device__ __forceinline__ SiteCoord site_coords(uint32_t s, const Geom& g, int par) {
  SiteCoord c;
  uint32_t r = fdiv(s, g.d_hx);
  c.xh = (int)(s - r * (uint32_t)g.hx);
  uint32_t r2 = fdiv(r, g.d_ly);
  c.y = (int)(r - r2 * (uint32_t)g.L[1]);
  uint32_t r3 = fdiv(r2, g.d_lz);
  c.z = (int)(r2 - r3 * (uint32_t)g.L[2]);
  c.t = (int)r3;
  c.x = 2 * c.xh + ((c.y + c.z + c.t + par) & 1);
  return c;
}

// cb index of the neighbour in direction mu (0..3) at distance dir (+-1, or
// +-3 for the three-hop links of the improved operator; |dir| <= L_mu)
__device__ __forceinline__ int neighbour_cb(int s, const SiteCoord& c, const Geom& g, int mu, int dir) {
  if (mu == 0) {
    int xn = c.x + dir;
    xn = xn < 0 ? xn + g.L[0] : (xn >= g.L[0] ? xn - g.L[0] : xn);
    return s - c.xh + (xn >> 1);
  }
  int v = mu == 1 ? c.y : (mu == 2 ? c.z : c.t);
  int vn = v + dir;
  vn = vn < 0 ? vn + g.L[mu] : (vn >= g.L[mu] ? vn - g.L[mu] : vn);
  return s + (vn - v) * g.stride[mu];
}

// Links of one output parity, blocked structure-of-arrays:
// link k (0..3 forward mu=k, 4..7 backward mu=k-4; for the improved operator
// also 8..11 three-hop forward, 12..15 three-hop backward) element e (0..8,
// row-major) of checkerboard site s lives at
// ((s>>sbl)*per + k*epl + e) << sbl | (s & (SB-1)), per = epl * links per
// site, with epl = 9 entries per link, or 6 for links kept as two rows.
__device__ __forceinline__ size_t link_off(uint32_t s, int k, int e, int sbl, int per = 72,
                                           int epl = 9) {
  return ((((size_t)(s >> sbl)) * per + k * epl + e) << sbl) | (s & ((1u << sbl) - 1));
}
