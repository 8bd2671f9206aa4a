// Gauge-field kernels of an RHMC trajectory (the gauge part of the HMC
// Hamiltonian of Sec. II and its molecular dynamics, Sec. IV):
//   Wilson action   S_g = beta sum_{x, mu<nu} (1 - Re Tr U_mu nu(x) / 3),
//                   U_mu nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
//   gauge force     F^a = -dS_g/d omega^a for U_mu(x) -> exp(i omega^a T^a) U_mu(x),
//                   T^a = lambda_a / 2: with the staple sum A_mu(x) of the six
//                   plaquettes through the link, F^a = -(beta/3) Im Tr(T^a U A),
//                   added into the momenta as P += scale F
//   link update     U <- exp(i eps P^a T^a) U
//   kinetic energy  1/2 sum (P^a)^2
// Links U[mu][idx][3][3] complex128 (lexicographic idx, periodic), momenta
// P[mu][idx][8] float64. One thread per site or link; the two sums finish in
// the fixed-order partial-sum kernel, so they are reproducible.
#include <cmath>

#include "blas.h"

namespace {

struct M3 {
  double2 e[9];
};

__device__ __forceinline__ M3 ld(const double2* p) {
  M3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) m.e[k] = p[k];
  return m;
}

// a b, a b^dag, a^dag b
__device__ __forceinline__ M3 mm(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(a.e[3 * i + k], b.e[3 * k + j], s);
      r.e[3 * i + j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 mmd(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(a.e[3 * i + k], cconj(b.e[3 * j + k]), s);
      r.e[3 * i + j] = s;
    }
  return r;
}
__device__ __forceinline__ M3 mdm(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0, 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cjfma(a.e[3 * k + i], b.e[3 * k + j], s);
      r.e[3 * i + j] = s;
    }
  return r;
}
__device__ __forceinline__ double re_tr(const M3& a) { return a.e[0].x + a.e[4].x + a.e[8].x; }

struct Lat {
  int L[4];
  int stride[4];
  int vol;
};

__device__ __forceinline__ void coords(const Lat& g, int idx, int* c) {
  c[0] = idx % g.L[0];
  c[1] = (idx / g.L[0]) % g.L[1];
  c[2] = (idx / (g.L[0] * g.L[1])) % g.L[2];
  c[3] = idx / (g.L[0] * g.L[1] * g.L[2]);
}
// lexicographic index of the site k steps from c in direction mu (|k| <= L)
__device__ __forceinline__ int nbr(const Lat& g, int idx, const int* c, int mu, int k) {
  int v = c[mu] + k;
  int d = k;
  if (v < 0) d += g.L[mu];
  if (v >= g.L[mu]) d -= g.L[mu];
  return idx + d * g.stride[mu];
}
__device__ __forceinline__ const double2* lk(const double2* U, const Lat& g, int mu, int idx) {
  return U + ((size_t)mu * g.vol + idx) * 9;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = BMS_WG / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  return red[0];
}

// per block: sum over its sites of sum_{mu<nu} (1 - Re Tr U_mu nu / 3)
__global__ __launch_bounds__(BMS_WG) void k_wilson(const double2* __restrict__ U, Lat g,
                                                   double2* __restrict__ partials) {
  __shared__ double red[BMS_WG];
  const int idx = blockIdx.x * BMS_WG + threadIdx.x;
  double acc = 0;
  if (idx < g.vol) {
    int c[4];
    coords(g, idx, c);
    for (int mu = 0; mu < 4; ++mu)
      for (int nu = mu + 1; nu < 4; ++nu) {
        const M3 a = mm(ld(lk(U, g, mu, idx)), ld(lk(U, g, nu, nbr(g, idx, c, mu, 1))));
        const M3 b = mm(ld(lk(U, g, nu, idx)), ld(lk(U, g, mu, nbr(g, idx, c, nu, 1))));
        acc += 1.0 - re_tr(mmd(a, b)) / 3.0;
      }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s, 0);
}

// Im Tr(T^a W) for the eight generators T^a = lambda_a / 2
__device__ __forceinline__ void im_tr_t(const M3& w, double* f) {
  const double2* e = w.e;
  f[0] = 0.5 * (e[3].y + e[1].y);
  f[1] = 0.5 * (-e[3].x + e[1].x);
  f[2] = 0.5 * (e[0].y - e[4].y);
  f[3] = 0.5 * (e[6].y + e[2].y);
  f[4] = 0.5 * (-e[6].x + e[2].x);
  f[5] = 0.5 * (e[7].y + e[5].y);
  f[6] = 0.5 * (-e[7].x + e[5].x);
  f[7] = 0.5 / sqrt(3.0) * (e[0].y + e[4].y - 2.0 * e[8].y);
}

// P[mu][x] += scale * F^a, F^a = -(beta/3) Im Tr(T^a U_mu(x) A_mu(x)), one thread per link
__global__ __launch_bounds__(BMS_WG) void k_gauge_force(const double2* __restrict__ U, Lat g,
                                                        double beta, double scale,
                                                        double* __restrict__ P) {
  const int t = blockIdx.x * BMS_WG + threadIdx.x;
  if (t >= 4 * g.vol) return;
  const int mu = t / g.vol, idx = t - mu * g.vol;
  int c[4];
  coords(g, idx, c);
  const int xp = nbr(g, idx, c, mu, 1);
  M3 A;
#pragma unroll
  for (int k = 0; k < 9; ++k) A.e[k] = make_double2(0, 0);
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    // up: U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
    const int xn = nbr(g, idx, c, nu, 1);
    const M3 up = mmd(mmd(ld(lk(U, g, nu, xp)), ld(lk(U, g, mu, xn))), ld(lk(U, g, nu, idx)));
    // down: U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)
    const int xm = nbr(g, idx, c, nu, -1);
    int cm[4] = {c[0], c[1], c[2], c[3]};
    cm[nu] = c[nu] == 0 ? g.L[nu] - 1 : c[nu] - 1;
    const int xpm = nbr(g, xm, cm, mu, 1);
    // = (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
    const M3 down = mdm(mm(ld(lk(U, g, mu, xm)), ld(lk(U, g, nu, xpm))), ld(lk(U, g, nu, xm)));
#pragma unroll
    for (int k = 0; k < 9; ++k) A.e[k] = cadd(A.e[k], cadd(up.e[k], down.e[k]));
  }
  const M3 w = mm(ld(lk(U, g, mu, idx)), A);
  double f[8];
  im_tr_t(w, f);
  double* p = P + (size_t)t * 8;
  const double k = -scale * beta / 3.0;
#pragma unroll
  for (int a = 0; a < 8; ++a) p[a] += k * f[a];
}

// E = exp(i X) for Hermitian X by scaling and squaring: Y = X / 2^s with
// |Y|_F <= 1/4, the Taylor series of exp(i Y) to order 16 (remainder below
// 4^-17 / 17!), then s squarings.
__device__ M3 exp_i(const M3& X) {
  double nf = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) nf += X.e[k].x * X.e[k].x + X.e[k].y * X.e[k].y;
  nf = sqrt(nf);
  int s = 0;
  while (nf > 0.25 && s < 60) {
    nf *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
  M3 iy;  // i Y
#pragma unroll
  for (int k = 0; k < 9; ++k) iy.e[k] = make_double2(-X.e[k].y * sc, X.e[k].x * sc);
  M3 E, term;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    E.e[k] = make_double2(k % 4 == 0 ? 1.0 : 0.0, 0);
    term.e[k] = E.e[k];
  }
  for (int j = 1; j <= 16; ++j) {
    term = mm(term, iy);
    const double inv = 1.0 / j;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      term.e[k] = cscale(term.e[k], inv);
      E.e[k] = cadd(E.e[k], term.e[k]);
    }
  }
  for (int k = 0; k < s; ++k) E = mm(E, E);
  return E;
}

// U_mu(x) <- exp(i eps P^a T^a) U_mu(x), one thread per link
__global__ __launch_bounds__(BMS_WG) void k_link_update(double2* __restrict__ U,
                                                        const double* __restrict__ P, int nlink,
                                                        double eps) {
  const int t = blockIdx.x * BMS_WG + threadIdx.x;
  if (t >= nlink) return;
  const double* p = P + (size_t)t * 8;
  const double h = 0.5 * eps, r3 = 1.0 / sqrt(3.0);
  M3 X;
  X.e[0] = make_double2(h * (p[2] + r3 * p[7]), 0);
  X.e[4] = make_double2(h * (-p[2] + r3 * p[7]), 0);
  X.e[8] = make_double2(h * (-2.0 * r3 * p[7]), 0);
  X.e[1] = make_double2(h * p[0], -h * p[1]);
  X.e[3] = make_double2(h * p[0], h * p[1]);
  X.e[2] = make_double2(h * p[3], -h * p[4]);
  X.e[6] = make_double2(h * p[3], h * p[4]);
  X.e[5] = make_double2(h * p[5], -h * p[6]);
  X.e[7] = make_double2(h * p[5], h * p[6]);
  double2* u = U + (size_t)t * 9;
  const M3 E = exp_i(X);
  const M3 n = mm(E, ld(u));
#pragma unroll
  for (int k = 0; k < 9; ++k) u[k] = n.e[k];
}

// per block: 1/2 sum of squares of its momenta
__global__ __launch_bounds__(BMS_WG) void k_kinetic(const double* __restrict__ P, size_t n,
                                                    double2* __restrict__ partials) {
  __shared__ double red[BMS_WG];
  double acc = 0;
  for (size_t i = (size_t)blockIdx.x * BMS_WG + threadIdx.x; i < n;
       i += (size_t)gridDim.x * BMS_WG)
    acc += P[i] * P[i];
  const double s = block_sum(0.5 * acc, red);
  if (threadIdx.x == 0) partials[blockIdx.x] = make_double2(s, 0);
}

Lat lat_of(const bms_ctx* c) {
  Lat g;
  for (int i = 0; i < 4; ++i) g.L[i] = c->dims[i];
  g.stride[0] = 1;
  g.stride[1] = c->dims[0];
  g.stride[2] = c->dims[0] * c->dims[1];
  g.stride[3] = c->dims[0] * c->dims[1] * c->dims[2];
  g.vol = (int)c->vol;
  return g;
}

constexpr int kKineticBlocks = 1024;

// a one-entry grid reduction read back to the host
int reduce_to_host(bms_ctx* c, double2* partials, int nb, double* out) {
  void* o;
  int rc = scratch_buf(c, S_RES, 64, &o);
  if (rc) return rc;
  HIP_TRY(c, launch_sum_partials(c->stream, partials, nb, 1, (double2*)o, nullptr, nullptr));
  double2 h;
  HIP_TRY(c, hipMemcpyAsync(&h, o, sizeof h, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *out = h.x;
  return BMS_OK;
}

}  // namespace

int gauge_action_dev(bms_ctx* c, double beta, const void* U, double* S) {
  const Lat g = lat_of(c);
  const int nb = (g.vol + BMS_WG - 1) / BMS_WG;
  void* pp;
  int rc = scratch_buf(c, S_PART, (size_t)nb * sizeof(double2) + 64, &pp);
  if (rc) return rc;
  k_wilson<<<nb, BMS_WG, 0, c->stream>>>((const double2*)U, g, (double2*)pp);
  HIP_TRY(c, hipGetLastError());
  double s;
  if ((rc = reduce_to_host(c, (double2*)pp, nb, &s))) return rc;
  *S = beta * s;
  return BMS_OK;
}

int gauge_force_dev(bms_ctx* c, double beta, const void* U, void* P, double scale) {
  const Lat g = lat_of(c);
  const int n = 4 * g.vol;
  k_gauge_force<<<(n + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>((const double2*)U, g, beta,
                                                                    scale, (double*)P);
  HIP_TRY(c, hipGetLastError());
  return BMS_OK;
}

int link_update_dev(bms_ctx* c, double eps, const void* P, void* U) {
  const int n = 4 * (int)c->vol;
  k_link_update<<<(n + BMS_WG - 1) / BMS_WG, BMS_WG, 0, c->stream>>>((double2*)U,
                                                                    (const double*)P, n, eps);
  HIP_TRY(c, hipGetLastError());
  return BMS_OK;
}

int kinetic_dev(bms_ctx* c, const void* P, double* K) {
  const size_t n = (size_t)4 * c->vol * 8;
  const int nb = (int)std::min<size_t>(kKineticBlocks, (n + BMS_WG - 1) / BMS_WG);
  void* pp;
  int rc = scratch_buf(c, S_PART, (size_t)nb * sizeof(double2) + 64, &pp);
  if (rc) return rc;
  k_kinetic<<<nb, BMS_WG, 0, c->stream>>>((const double*)P, n, (double2*)pp);
  HIP_TRY(c, hipGetLastError());
  return reduce_to_host(c, (double2*)pp, nb, K);
}

extern "C" int bms_gauge_action(bms_ctx* c, double beta, const void* U, double* S) {
  if (!c) return BMS_EINVAL;
  if (!U || !S) return set_err(c, BMS_EINVAL, "null pointer");
  if (!std::isfinite(beta)) return set_err(c, BMS_EINVAL, "beta not finite");
  int rc = stream_begin(c);
  if (rc) return rc;
  if ((rc = gauge_action_dev(c, beta, U, S))) return rc;
  return stream_end(c);
}

extern "C" int bms_gauge_force(bms_ctx* c, double beta, const void* U, void* P, double scale) {
  if (!c) return BMS_EINVAL;
  if (!U || !P) return set_err(c, BMS_EINVAL, "null pointer");
  if (!std::isfinite(beta) || !std::isfinite(scale))
    return set_err(c, BMS_EINVAL, "beta or scale not finite");
  int rc = stream_begin(c);
  if (rc) return rc;
  if ((rc = gauge_force_dev(c, beta, U, P, scale))) return rc;
  return stream_end(c);
}

extern "C" int bms_gauge_update(bms_ctx* c, double eps, const void* P, void* U) {
  if (!c) return BMS_EINVAL;
  if (!U || !P) return set_err(c, BMS_EINVAL, "null pointer");
  if (!std::isfinite(eps)) return set_err(c, BMS_EINVAL, "eps not finite");
  int rc = stream_begin(c);
  if (rc) return rc;
  if ((rc = link_update_dev(c, eps, P, U))) return rc;
  return stream_end(c);
}

extern "C" int bms_kinetic_energy(bms_ctx* c, const void* P, double* K) {
  if (!c) return BMS_EINVAL;
  if (!P || !K) return set_err(c, BMS_EINVAL, "null pointer");
  int rc = stream_begin(c);
  if (rc) return rc;
  if ((rc = kinetic_dev(c, P, K))) return rc;
  return stream_end(c);
}
