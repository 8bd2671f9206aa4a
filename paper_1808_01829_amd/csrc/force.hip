// Pseudofermion force (eq. force): the link derivative of
//   S = sum_i sum_j alpha_j phi_i^dag (A + s_j)^-1 phi_i
// from the solutions x_ij = (A + s_j)^-1 phi_i. With y = D_oe x,
//   dS = -2 sum_ij alpha_j Re[y_ij^dag dD_oe x_ij] = sum_links Re Tr[dU M]
//   M_mu(w) = -eta_mu(w) b sum_ij alpha_j x_ij(w+mu) y_ij(w)^dag   (w odd)
//   M_mu(w) = +eta_mu(w) b sum_ij alpha_j y_ij(w+mu) x_ij(w)^dag   (w even)
// Every link joins an even and an odd site, so each is written exactly once.
#include <string.h>

#include <cmath>

#include <vector>

#include "internal.h"

namespace {

struct ForceArgs {
  Geom g;
  int bc[4];
  int n, ns, sbl, lie, add;
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
      if (e % lpl == lane) {
        const double2 v = cconj(m[3 * (e % 3) + e / 3]);
        G[e] = a.add ? cadd(G[e], v) : v;
      }
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
  double fv[8];
  fv[0] = 0.5 * (w[3].y + w[1].y);                   // lambda_1: (0,1),(1,0)
  fv[1] = 0.5 * (-(w[3].x) + w[1].x);                // lambda_2: -i at (0,1), +i at (1,0)
  fv[2] = 0.5 * (w[0].y - w[4].y);                   // lambda_3
  fv[3] = 0.5 * (w[6].y + w[2].y);                   // lambda_4: (0,2),(2,0)
  fv[4] = 0.5 * (-(w[6].x) + w[2].x);                // lambda_5
  fv[5] = 0.5 * (w[7].y + w[5].y);                   // lambda_6: (1,2),(2,1)
  fv[6] = 0.5 * (-(w[7].x) + w[5].x);                // lambda_7
  fv[7] = 0.5 / sqrt(3.0) * (w[0].y + w[4].y - 2.0 * w[8].y);  // lambda_8
  double* F = a.F + lo * 8;
  for (int k = 0; k < 8; ++k) F[k] = a.add ? F[k] + fv[k] : fv[k];
}

// Quad sum by DPP: every lane of each group of four ends with the group's sum.
__device__ __forceinline__ double dpp_xor1(double v) {
  long long u = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)u, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0xB1, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double dpp_xor2(double v) {
  long long u = __builtin_bit_cast(long long, v);
  int lo = __builtin_amdgcn_mov_dpp((int)u, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), 0x4E, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 quad_sum(double2 v) {
  v.x += dpp_xor1(v.x);
  v.y += dpp_xor1(v.y);
  v.x += dpp_xor2(v.x);
  v.y += dpp_xor2(v.y);
  return v;
}

// Fused force, one odd site z per 16 lanes. Every link joins an odd and an
// even site, so the links of z's forward hops (z, mu) and of its backward
// hops (z - mu, mu) cover each link of the lattice once. Lane q = lane % 4
// of the site owns direction mu = q, both links (as the half hop D_oe stores
// them: 1/2 eta b U_mu(z) and -1/2 eta b' U_mu(z-mu)^dag); lane
// g = (lane / 4) % 4 takes the flat columns c = g, g + 4, ... of the
// K = n * N_s columns (c = shift * n + column). Per column the four q-lanes
// form their share of y(z) = (D_oe x)(z) from x(z + mu) and x(z - mu), add
// the shares by DPP (a quad), and accumulate
//   M_a += alpha x(z + mu) y(z)^dag     (link (z, mu),      z odd)
//   M_b += alpha y(z) x(z - mu)^dag     (link (z - mu, mu), z - mu even),
// so y never leaves the registers and each x load serves both. At the end the
// four g-lanes add their partial 3 x 3 sums and write each link once.
//
// LDS_LINKS: the links wait in LDS (18 KB per work-group) instead of 72
// registers, read back every column; the registers freed hold the x loads of
// the next PF columns, issued before the current column is computed.
constexpr int kForceSites = BMS_WG / 16;  // odd sites per work-group
constexpr int kLinkPitch = 8 * 9 + 1;     // complex per site in LDS (one pad)

struct FCol {
  double2 va[3], vb[3];
  double al;
};

template <int PF, bool LDS_LINKS, int WAVES>
__global__ __launch_bounds__(BMS_WG, WAVES) void k_force_fused(ForceArgs a) {
  const Geom& g = a.g;
  const int lane = threadIdx.x & 63;
  const int q = lane & 3, gl = (lane >> 2) & 3;
  const int sl = threadIdx.x >> 4;  // site within the work-group
  const uint32_t z0 = blockIdx.x * kForceSites + sl;
  const bool live = z0 < (uint32_t)g.vh;
  // dead sites of the last block compute on the last site and write nothing,
  // so every lane of a quad and of a g-group takes part in the shuffles
  const uint32_t z = live ? z0 : (uint32_t)g.vh - 1;
  const int mu = q;
  SiteCoord sc = site_coords(z, g, 1);
  const int co[4] = {sc.x, sc.y, sc.z, sc.t};
  const int ef = neighbour_cb((int)z, sc, g, mu, 1);
  const int eb = neighbour_cb((int)z, sc, g, mu, -1);
  int esum = 0;
  for (int nu = 0; nu < mu; ++nu) esum += co[nu];
  const double eta = (esum & 1) ? -1.0 : 1.0;
  const double bf = co[mu] == g.L[mu] - 1 ? (double)a.bc[mu] : 1.0;
  const double be = co[mu] == 0 ? (double)a.bc[mu] : 1.0;
  const double2* L = a.links + a.pstride;  // parity 1 (odd output sites)
  __shared__ double2 lds[LDS_LINKS ? kForceSites * kLinkPitch : 1];
  double2 la[9], lb[9];
  if (LDS_LINKS) {
    // the four g-lanes of (site, q) stage the site's links mu and 4 + mu
    for (int e = gl; e < 9; e += 4) {
      lds[sl * kLinkPitch + mu * 9 + e] = L[link_off(z, mu, e, a.sbl)];
      lds[sl * kLinkPitch + (4 + mu) * 9 + e] = L[link_off(z, 4 + mu, e, a.sbl)];
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      la[e] = L[link_off(z, mu, e, a.sbl)];
      lb[e] = L[link_off(z, 4 + mu, e, a.sbl)];
    }
  }
  double2 ma[9], mb[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    ma[e] = make_double2(0, 0);
    mb[e] = make_double2(0, 0);
  }
  const int n = a.n;
  const int K = n * a.ns;
  const size_t blk = (size_t)g.vh * 3 * n;
  const double2* xf = a.X + (size_t)ef * 3 * n;
  const double2* xbk = a.X + (size_t)eb * 3 * n;
  // load cursor: flat column c = j * n + i = 4 t + g. Every lane runs the
  // same steps; columns past K load column 0 and add nothing.
  const int T = (K + 3) >> 2;
  int j = gl / n, i = gl - (gl / n) * n, c = gl;
  auto load = [&](FCol& f) {
    const bool valid = c < K;
    const size_t o = valid ? (size_t)j * blk + i : 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      f.va[b] = xf[o + (size_t)b * n];
      f.vb[b] = xbk[o + (size_t)b * n];
    }
    f.al = valid ? a.alpha[valid ? j : 0] : 0.0;
    c += 4;
    i += 4;
    while (i >= n) {
      i -= n;
      ++j;
    }
  };
  int lofs = sl * kLinkPitch + mu * 9;
  auto compute = [&](const FCol& f) {
    if (LDS_LINKS) {
      // a fresh address every column keeps the LDS reads inside the loop
      asm volatile("" : "+v"(lofs));
    }
    double2 y[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      double2 t = make_double2(0, 0);
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const double2 lfa = LDS_LINKS ? lds[lofs + 3 * r + b] : la[3 * r + b];
        const double2 lfb = LDS_LINKS ? lds[lofs + 36 + 3 * r + b] : lb[3 * r + b];
        t = cfma(lfa, f.va[b], t);
        t = cfma(lfb, f.vb[b], t);
      }
      y[r] = cscale(quad_sum(t), f.al);
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        ma[3 * r + b] = cjfma(y[b], f.va[r], ma[3 * r + b]);  // x_f[r] conj(y[b])
        mb[3 * r + b] = cjfma(f.vb[b], y[r], mb[3 * r + b]);  // y[r] conj(x_b[b])
      }
  };
  FCol buf[PF];
#pragma unroll
  for (int u = 0; u < PF; ++u) load(buf[u]);
  for (int t = 0; t < T; t += PF) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const FCol cur = buf[u];
      load(buf[u]);  // PF columns ahead
      compute(cur);
    }
  }
  // add the four column groups (lanes 4 and 8 apart)
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    ma[e].x += __shfl_xor(ma[e].x, 4);
    ma[e].y += __shfl_xor(ma[e].y, 4);
    mb[e].x += __shfl_xor(mb[e].x, 4);
    mb[e].y += __shfl_xor(mb[e].y, 4);
    ma[e].x += __shfl_xor(ma[e].x, 8);
    ma[e].y += __shfl_xor(ma[e].y, 8);
    mb[e].x += __shfl_xor(mb[e].x, 8);
    mb[e].y += __shfl_xor(mb[e].y, 8);
  }
  if (!live) return;
  // M_mu(z) = -eta b_f sum alpha x(z+mu) y(z)^dag ; M_mu(z-mu) = +eta b_e sum alpha y(z) x(z-mu)^dag
  const double sa = -eta * bf, sb = eta * be;
  const uint32_t vol = 2u * (uint32_t)g.vh;
  const uint32_t idx_a = (uint32_t)(sc.x + g.L[0] * (sc.y + g.L[1] * (sc.z + g.L[2] * sc.t)));
  int cb_[4] = {sc.x, sc.y, sc.z, sc.t};
  cb_[mu] = co[mu] == 0 ? g.L[mu] - 1 : co[mu] - 1;
  const uint32_t idx_b = (uint32_t)(cb_[0] + g.L[0] * (cb_[1] + g.L[1] * (cb_[2] + g.L[2] * cb_[3])));
  const bool second = gl >= 2;  // lanes g = 0, 1 write link a; g = 2, 3 link b
  const uint32_t idx = second ? idx_b : idx_a;
  const double sg = second ? sb : sa;
  double2 m[9];
#pragma unroll
  for (int e = 0; e < 9; ++e) m[e] = cscale(second ? mb[e] : ma[e], sg);
  const size_t lo = (size_t)mu * vol + idx;
  if (!a.lie) {
    // G = M^dag, the two lanes of a link split its nine entries
    double2* G = a.G + lo * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e)
      if ((e & 1) == (gl & 1)) {
        const double2 v = cconj(m[3 * (e % 3) + e / 3]);
        G[e] = a.add ? cadd(G[e], v) : v;
      }
    return;
  }
  if (gl & 1) return;
  // the link itself: U = 2 eta b_f L_a, or U = (-2 eta b_e L_b)^dag
  double2 u[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (LDS_LINKS)
        u[3 * r + b] = second ? cconj(cscale(lds[sl * kLinkPitch + (4 + mu) * 9 + 3 * b + r],
                                             -2.0 * eta * be))
                              : cscale(lds[sl * kLinkPitch + mu * 9 + 3 * r + b], 2.0 * eta * bf);
      else
        u[3 * r + b] = second ? cconj(cscale(lb[3 * b + r], -2.0 * eta * be))
                              : cscale(la[3 * r + b], 2.0 * eta * bf);
    }
  double2 w[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double2 t = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) t = cfma(u[3 * r + k], m[3 * k + b], t);
      w[3 * r + b] = t;
    }
  double f[8];
  f[0] = 0.5 * (w[3].y + w[1].y);
  f[1] = 0.5 * (-(w[3].x) + w[1].x);
  f[2] = 0.5 * (w[0].y - w[4].y);
  f[3] = 0.5 * (w[6].y + w[2].y);
  f[4] = 0.5 * (-(w[6].x) + w[2].x);
  f[5] = 0.5 * (w[7].y + w[5].y);
  f[6] = 0.5 * (-(w[7].x) + w[5].x);
  f[7] = 0.5 / sqrt(3.0) * (w[0].y + w[4].y - 2.0 * w[8].y);
  double* F = a.F + lo * 8;
#pragma unroll
  for (int k = 0; k < 8; ++k) F[k] = a.add ? F[k] + f[k] : f[k];
}

}  // namespace

extern "C" int bms_force(bms_ctx* c, int n, int ns, const double* alpha, const void* X, void* out,
                         int flags) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 1 || ns > BMS_MAX_SHIFTS) return set_err(c, BMS_EINVAL, "bad n_shifts");
  if (!alpha || !X || !out) return set_err(c, BMS_EINVAL, "null pointer");
  if (flags < 0 || flags > (BMS_FORCE_LIE | BMS_FORCE_ADD)) return set_err(c, BMS_EINVAL, "bad flags");
  for (int s = 0; s < ns; ++s)
    if (!std::isfinite(alpha[s])) return set_err(c, BMS_EINVAL, "alpha[%d] not finite", s);
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  if (c->nlinks != 8)
    return set_err(c, BMS_EINVAL, "the force is defined for the unimproved operator only");
  int rc;
  if ((rc = stream_begin(c))) return rc;
  const size_t blk = (size_t)c->vh * 3 * n;
  const bool fused = c->force_variant != 0;
  void* Y = nullptr;
  if (!fused && (rc = scratch_buf(c, S_Y, blk * ns * sizeof(double2), &Y))) return rc;
  ForceArgs a;
  memset(&a, 0, sizeof a);
  a.g = c->geom;
  for (int i = 0; i < 4; ++i) a.bc[i] = c->bc[i];
  a.n = n;
  a.ns = ns;
  a.sbl = c->sbl;
  a.lie = (flags & BMS_FORCE_LIE) != 0;
  a.add = (flags & BMS_FORCE_ADD) != 0;
  a.X = (const double2*)X;
  a.Y = (const double2*)Y;
  a.links = (const double2*)c->links64.p;
  a.pstride = (size_t)c->nblk * 72 << c->sbl;
  a.G = (double2*)out;
  a.F = (double*)out;
  for (int s = 0; s < ns; ++s) a.alpha[s] = alpha[s];
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (c->timing) {
    // the whole call is timed (for variant 0 its D_oe hops included)
    HIP_TRY(c, hipEventCreate(&ev[0]));
    HIP_TRY(c, hipEventCreate(&ev[1]));
    HIP_TRY(c, hipEventRecord(ev[0], c->stream));
  }
  if (fused) {
    // 16 lanes per odd site. Variants: 1 links in registers, loads one
    // column ahead; 2 (default) links in LDS, loads two columns ahead.
    // Measured at 16^3 x 32, K = 128: 511 and 499 us (hops + per-link
    // kernel, variant 0: 998 us)
    const dim3 grid((c->vh + kForceSites - 1) / kForceSites);
    const int fv = c->force_variant < 0 ? 2 : c->force_variant;
    if (fv == 1)
      k_force_fused<1, false, 2><<<grid, BMS_WG, 0, c->stream>>>(a);
    else
      k_force_fused<2, true, 2><<<grid, BMS_WG, 0, c->stream>>>(a);
  } else {
    // Y = D_oe X per shift, then a lane group per link (the block width
    // rounded up to a power of two, at most 16)
    for (int s = 0; s < ns; ++s)
      HIP_TRY(c, launch_hop<double>(c, 1, n, (const double2*)X + s * blk, (double2*)Y + s * blk,
                                    nullptr, 0.0, 1.0, nullptr));
    int lpl = 1;
    while (lpl < n && lpl < 16) lpl <<= 1;
    const uint32_t nthr = 4u * (uint32_t)c->vol * (uint32_t)lpl;
    k_force<<<(nthr + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>(a, lpl);
  }
  HIP_TRY(c, hipGetLastError());
  if (c->timing) {
    // algorithmic bytes: every solution read once, the 4V FP64 links once, the output
    HIP_TRY(c, hipEventRecord(ev[1], c->stream));
    HIP_TRY(c, hipEventSynchronize(ev[1]));
    float ms = 0;
    HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
    const double vol = (double)c->vol;
    c->kt_ms[BMS_KERNEL_FORCE] += ms;
    c->kt_launches[BMS_KERNEL_FORCE] += 1;
    c->kt_bytes[BMS_KERNEL_FORCE] += (double)ns * blk * sizeof(double2) + 4 * vol * 9 * 16 +
                                     (a.lie ? 4 * vol * 8 * 8 : 4 * vol * 9 * 16);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
  }
  return stream_end(c);
}
