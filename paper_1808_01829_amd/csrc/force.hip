// Pseudofermion force (eq. force): the link derivative of
//   S = sum_i sum_j alpha_j phi_i^dag (A + s_j)^-1 phi_i
// from the solutions x_ij = (A + s_j)^-1 phi_i. With y = D_oe x,
//   dS = -2 sum_ij alpha_j Re[y_ij^dag dD_oe x_ij] = sum_links Re Tr[dU M]
//   M_mu(w) = -eta_mu(w) b sum_ij alpha_j x_ij(w+mu) y_ij(w)^dag   (w odd)
//   M_mu(w) = +eta_mu(w) b sum_ij alpha_j y_ij(w+mu) x_ij(w)^dag   (w even)
// Every link joins an even and an odd site, so each is written exactly once.
#include <string.h>

#include <vector>

#include "internal.h"

namespace {

struct ForceArgs {
  Geom g;
  int bc[4];
  int n, ns, sbl, lie;
  const double2* X;      // [ns][vh][3][n] even sites
  const double2* Y;      // [ns][vh][3][n] odd sites, Y = D_oe X
  const double2* links;  // FP64 internal links, both parities
  size_t pstride;        // complex elements per parity of `links`
  double2* G;            // raw gradient [mu][idx][3][3]
  double* F;             // Lie-algebra force [mu][idx][8]
  double alpha[BMS_MAX_SHIFTS];
};

// Sum of a complex value over the LPL lanes of this lane's group (LPL a power
// of two dividing the wave): every lane of the group ends with the total.
__device__ __forceinline__ double2 group_sum(double2 v, int lpl) {
  for (int off = 1; off < lpl; off <<= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  return v;
}

// One group of lpl lanes per link (the 4 links of a site are neighbouring
// groups): lane l of the group takes columns l, l + lpl, ... of every shift,
// so the group's loads of one colour row are one contiguous run, and the 3 x 3
// partial sums are added across the group at the end.
__global__ __launch_bounds__(BMS_WG) void k_force(ForceArgs a, int lpl) {
  const Geom& g = a.g;
  const uint32_t vol = 2u * g.vh;
  const uint32_t tid = blockIdx.x * BMS_WG + threadIdx.x;
  // whole groups leave together (lpl divides BMS_WG and 4 * vol * lpl threads
  // are launched in whole work-groups), so every lane of a shuffle is active
  const uint32_t link = tid / (uint32_t)lpl;
  const int lane = (int)(tid - link * (uint32_t)lpl);
  const bool live = link < 4u * vol;
  const int mu = (int)(link & 3);
  const uint32_t idx = live ? link >> 2 : 0;
  uint32_t cb = idx >> 1;
  uint32_t r = fdiv(cb, g.d_hx);
  int x = (int)(idx - r * (uint32_t)g.L[0]);
  uint32_t r2 = fdiv(r, g.d_ly);
  int y = (int)(r - r2 * (uint32_t)g.L[1]);
  uint32_t r3 = fdiv(r2, g.d_lz);
  int z = (int)(r2 - r3 * (uint32_t)g.L[2]);
  int t = (int)r3;
  int co[4] = {x, y, z, t};
  int par = (x + y + z + t) & 1;
  SiteCoord sc;
  sc.x = x;
  sc.y = y;
  sc.z = z;
  sc.t = t;
  sc.xh = x >> 1;
  int nb = neighbour_cb((int)cb, sc, g, mu, 1);
  int esum = 0;
  for (int nu = 0; nu < mu; ++nu) esum += co[nu];
  double eb = (esum & 1) ? -1.0 : 1.0;
  if (co[mu] == g.L[mu] - 1) eb *= a.bc[mu];
  // w odd: M = -eb sum alpha X(nb) Y(w)^dag ; w even: M = +eb sum alpha Y(nb) X(w)^dag
  const double2* colv = par ? a.X : a.Y;
  const double2* rowv = par ? a.Y : a.X;
  double sgn = par ? -eb : eb;
  const int n = a.n;
  size_t blk = (size_t)g.vh * 3 * n;
  double2 m[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = make_double2(0, 0);
  if (live) {
    for (int s = 0; s < a.ns; ++s) {
      const double2* cs = colv + s * blk + (size_t)nb * 3 * n;
      const double2* rs = rowv + s * blk + (size_t)cb * 3 * n;
      double al = a.alpha[s] * sgn;
      for (int i = lane; i < n; i += lpl) {
        double2 c0 = cscale(cs[i], al), c1 = cscale(cs[n + i], al), c2 = cscale(cs[2 * n + i], al);
        double2 r0 = rs[i], r1 = rs[n + i], r2v = rs[2 * n + i];
        // m[a][b] += c[a] conj(r[b])
        m[0] = cjfma(r0, c0, m[0]);
        m[1] = cjfma(r1, c0, m[1]);
        m[2] = cjfma(r2v, c0, m[2]);
        m[3] = cjfma(r0, c1, m[3]);
        m[4] = cjfma(r1, c1, m[4]);
        m[5] = cjfma(r2v, c1, m[5]);
        m[6] = cjfma(r0, c2, m[6]);
        m[7] = cjfma(r1, c2, m[7]);
        m[8] = cjfma(r2v, c2, m[8]);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = group_sum(m[e], lpl);
  if (!live) return;
  size_t lo = ((size_t)mu * vol + idx);
  if (!a.lie) {
    // the group's lanes share the nine entries of the output
    double2* G = a.G + lo * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e)
      if (e % lpl == lane) G[e] = cconj(m[3 * (e % 3) + e / 3]);
    return;
  }
  if (lane != 0) return;
  // U_mu(w) from the forward link of parity par: L = (1/2) eta b U
  const double2* L = a.links + (size_t)par * a.pstride;
  double2 u[9];
  double f = 2.0 * ((esum & 1) ? -1.0 : 1.0) * ((co[mu] == g.L[mu] - 1) ? a.bc[mu] : 1);
  for (int e = 0; e < 9; ++e) u[e] = cscale(L[link_off(cb, mu, e, a.sbl)], f);
  // W = U M; F^a = Im Tr[T^a W], T^a = lambda_a / 2
  double2 w[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
      for (int k = 0; k < 3; ++k) s = cfma(u[3 * i + k], m[3 * k + j], s);
      w[3 * i + j] = s;
    }
  // Tr[T W] = sum_ij T_ij W_ji
  double* F = a.F + lo * 8;
  F[0] = 0.5 * (w[3].y + w[1].y);                   // lambda_1: (0,1),(1,0)
  F[1] = 0.5 * (-(w[3].x) + w[1].x);                // lambda_2: -i at (0,1), +i at (1,0)
  F[2] = 0.5 * (w[0].y - w[4].y);                   // lambda_3
  F[3] = 0.5 * (w[6].y + w[2].y);                   // lambda_4: (0,2),(2,0)
  F[4] = 0.5 * (-(w[6].x) + w[2].x);                // lambda_5
  F[5] = 0.5 * (w[7].y + w[5].y);                   // lambda_6: (1,2),(2,1)
  F[6] = 0.5 * (-(w[7].x) + w[5].x);                // lambda_7
  F[7] = 0.5 / sqrt(3.0) * (w[0].y + w[4].y - 2.0 * w[8].y);  // lambda_8
}

}  // namespace

extern "C" int bms_force(bms_ctx* c, int n, int ns, const double* alpha, const void* X, void* out,
                         int flags) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 1 || ns > BMS_MAX_SHIFTS) return set_err(c, BMS_EINVAL, "bad n_shifts");
  if (!alpha || !X || !out) return set_err(c, BMS_EINVAL, "null pointer");
  if (flags != BMS_FORCE_RAW && flags != BMS_FORCE_LIE) return set_err(c, BMS_EINVAL, "bad flags");
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  int rc;
  if ((rc = stream_begin(c))) return rc;
  size_t blk = (size_t)c->vh * 3 * n;
  void* Y;
  if ((rc = scratch_buf(c, S_Y, blk * ns * sizeof(double2), &Y))) return rc;
  for (int s = 0; s < ns; ++s)
    HIP_TRY(c, launch_hop<double>(c, 1, n, (const double2*)X + s * blk, (double2*)Y + s * blk,
                                  nullptr, 0.0, 1.0, nullptr));
  ForceArgs a;
  memset(&a, 0, sizeof a);
  a.g = c->geom;
  for (int i = 0; i < 4; ++i) a.bc[i] = c->bc[i];
  a.n = n;
  a.ns = ns;
  a.sbl = c->sbl;
  a.lie = flags == BMS_FORCE_LIE;
  a.X = (const double2*)X;
  a.Y = (const double2*)Y;
  a.links = (const double2*)c->links64.p;
  a.pstride = (size_t)c->nblk * 72 << c->sbl;
  a.G = (double2*)out;
  a.F = (double*)out;
  for (int s = 0; s < ns; ++s) a.alpha[s] = alpha[s];
  // lanes per link: the block width rounded up to a power of two, at most 16
  int lpl = 1;
  while (lpl < n && lpl < 16) lpl <<= 1;
  uint32_t nthr = 4u * (uint32_t)c->vol * (uint32_t)lpl;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (c->timing) {
    HIP_TRY(c, hipEventCreate(&ev[0]));
    HIP_TRY(c, hipEventCreate(&ev[1]));
    HIP_TRY(c, hipEventRecord(ev[0], c->stream));
  }
  k_force<<<(nthr + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>(a, lpl);
  HIP_TRY(c, hipGetLastError());
  if (c->timing) {
    // algorithmic bytes: X and Y of every shift once, the 4V FP64 links, the output
    HIP_TRY(c, hipEventRecord(ev[1], c->stream));
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    const double vol = (double)c->vol;
    c->kt_ms[BMS_KERNEL_FORCE] += ms;
    c->kt_launches[BMS_KERNEL_FORCE] += 1;
    c->kt_bytes[BMS_KERNEL_FORCE] += 2.0 * ns * blk * sizeof(double2) + 4 * vol * 9 * 16 +
                                     (a.lie ? 4 * vol * 8 * 8 : 4 * vol * 9 * 16);
    hipEventDestroy(ev[0]);
    hipEventDestroy(ev[1]);
  }
  return stream_end(c);
}
