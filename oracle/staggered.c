/*
 * Test infrastructure only: the plain FP64 CPU oracle.
 *
 * Nothing in the product path may link, load or call this file. It exists so
 * that tests, the smoke check and the CPU baseline of the benchmark can
 * compare the HIP library with an obviously correct implementation written
 * straight from the paper's definitions. It shares no code, header or table
 * with the HIP library.
 *
 * What it computes (de Forcrand & Keegan, "Rational Hybrid Monte Carlo with
 * Block Solvers and Multiple Pseudofermions"):
 *
 *  - The unimproved staggered operator used in Sec. IV (the paper names it but
 *    does not write it out; this is the textbook form):
 *      (D psi)(x) = 1/2 sum_mu eta_mu(x) [ b U_mu(x) psi(x+mu)
 *                                          - b U_mu(x-mu)^dag psi(x-mu) ]
 *    with eta_mu(x) = (-1)^(x_0+...+x_{mu-1}), direction order (x,y,z,t),
 *    and b = bc[mu] on a link that crosses the lattice boundary, 1 elsewhere.
 *    M = m + D; the even-odd preconditioned normal operator on even sites is
 *      A = M^dag M |_even = m^2 - D_eo D_oe.
 *  - An improved, less local variant (the paper's outlook, Sec. V): one-hop
 *    links V (in place of U) plus three-hop links W,
 *      (D psi)(x) = 1/2 sum_mu eta_mu(x) [ b V_mu(x) psi(x+mu) - b V_mu(x-mu)^dag psi(x-mu)
 *                                  + b3 W_mu(x) psi(x+3mu) - b3 W_mu(x-3mu)^dag psi(x-3mu) ]
 *    where b3 is the product of the boundary factors of the three unit steps
 *    the three-hop link spans; the coefficients of an improvement scheme (for
 *    the Naik term 9/8 and -1/24) are folded into V and W by the caller.
 *    W = NULL gives the unimproved operator.
 *  - Conjugate gradient on (A + sigma) x = b (Sec. III, the CG paragraph).
 *  - Multi-shift CG for all shifts at once (Sec. III, the SCG paragraph):
 *    shifted residuals are kept collinear with the unshifted one through a
 *    scalar recurrence for the collinearity factor zeta.
 *  - The link derivative of the pseudofermion action S = sum_i phi_i^dag r(A)
 *    phi_i with r(A) = a0 + sum_j a_j (A + s_j)^-1 (eq. RA and eq. force):
 *      dS = -2 sum_ij a_j Re[ y_ij^dag dD_oe x_ij ],
 *      x_ij = (A + s_j)^-1 phi_i (even sites), y_ij = D_oe x_ij (odd sites).
 *    Written per link as dS = sum Re Tr[dU_mu(w) M_mu(w)] with
 *      M_mu(w) = -eta_mu(w) b sum a_j x(w+mu) y(w)^dag   (w odd)
 *      M_mu(w) = +eta_mu(w) b sum a_j y(w+mu) x(w)^dag   (w even)
 *    the gradient returned is G = M^dag, i.e. G_ab = dS/dRe U_ab + i dS/dIm U_ab.
 *
 * Layouts (all complex numbers are interleaved double pairs re, im):
 *   site index   idx = x + Lx*(y + Ly*(z + Lz*t)), parity (x+y+z+t)&1,
 *                checkerboard index cb = idx>>1 (all extents even).
 *   gauge field  U[mu][idx][a][b]            (4*V*9 complex)
 *   half vector  v[cb][color]                (V/2*3 complex)
 *   gradient     G[mu][idx][a][b]            (4*V*9 complex)
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static inline cplx c_add(cplx a, cplx b) { cplx r = {a.re + b.re, a.im + b.im}; return r; }
static inline cplx c_sub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static inline cplx c_mul(cplx a, cplx b) {
  cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
  return r;
}
/* conj(a) * b */
static inline cplx c_cjmul(cplx a, cplx b) {
  cplx r = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
  return r;
}
static inline cplx c_scale(cplx a, double s) { cplx r = {a.re * s, a.im * s}; return r; }

/* ---- geometry --------------------------------------------------------- */

static long volume(const int *dims) {
  return (long)dims[0] * dims[1] * dims[2] * dims[3];
}

static void coords_of(const int *dims, long idx, int *c) {
  for (int mu = 0; mu < 4; ++mu) {
    c[mu] = (int)(idx % dims[mu]);
    idx /= dims[mu];
  }
}

static long index_of(const int *dims, const int *c) {
  return c[0] + (long)dims[0] * (c[1] + (long)dims[1] * (c[2] + (long)dims[2] * c[3]));
}

/* lexicographic index of the site of parity `par` with checkerboard index cb */
static long site_of_cb(const int *dims, long cb, int par) {
  long idx = 2 * cb;
  int c[4];
  coords_of(dims, idx, c);
  int p = (c[0] + c[1] + c[2] + c[3]) & 1;
  return p == par ? idx : idx + 1;
}

static double eta(const int *c, int mu) {
  int s = 0;
  for (int nu = 0; nu < mu; ++nu) s += c[nu];
  return (s & 1) ? -1.0 : 1.0;
}

/* neighbour of c in direction mu, dir = +1 or -1; returns the boundary factor
 * of the link that is crossed */
static double neighbour(const int *dims, const int *bc, const int *c, int mu, int dir, int *nc) {
  for (int k = 0; k < 4; ++k) nc[k] = c[k];
  double b = 1.0;
  if (dir > 0) {
    if (c[mu] == dims[mu] - 1) { nc[mu] = 0; b = (double)bc[mu]; }
    else nc[mu] = c[mu] + 1;
  } else {
    if (c[mu] == 0) { nc[mu] = dims[mu] - 1; b = (double)bc[mu]; }
    else nc[mu] = c[mu] - 1;
  }
  return b;
}

static const cplx *link(const cplx *U, const int *dims, int mu, long idx) {
  return U + ((long)mu * volume(dims) + idx) * 9;
}

/* ---- operator ------------------------------------------------------- */

/* out(z) = (D psi)(z) for every site z of parity par_out; psi lives on the
 * other parity. */
void ora_dslash_half_imp(const int *dims, const int *bc, const double *Ud, const double *Wd,
                         int par_out, const double *in_d, double *out_d) {
  const cplx *U = (const cplx *)Ud;
  const cplx *W = (const cplx *)Wd;
  const cplx *in = (const cplx *)in_d;
  cplx *out = (cplx *)out_d;
  long vh = volume(dims) / 2;
#pragma omp parallel for schedule(static)
  for (long s = 0; s < vh; ++s) {
    long idx = site_of_cb(dims, s, par_out);
    int c[4], nc[4];
    coords_of(dims, idx, c);
    cplx acc[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int mu = 0; mu < 4; ++mu) {
      double e = 0.5 * eta(c, mu);
      /* forward: + U_mu(x) psi(x+mu) */
      double bf = neighbour(dims, bc, c, mu, +1, nc);
      long nf = index_of(dims, nc);
      const cplx *uf = link(U, dims, mu, idx);
      const cplx *pf = in + (nf >> 1) * 3;
      for (int a = 0; a < 3; ++a) {
        cplx t = {0, 0};
        for (int b = 0; b < 3; ++b) t = c_add(t, c_mul(uf[3 * a + b], pf[b]));
        acc[a] = c_add(acc[a], c_scale(t, e * bf));
      }
      /* backward: - U_mu(x-mu)^dag psi(x-mu) */
      double bb = neighbour(dims, bc, c, mu, -1, nc);
      long nb = index_of(dims, nc);
      const cplx *ub = link(U, dims, mu, nb);
      const cplx *pb = in + (nb >> 1) * 3;
      for (int a = 0; a < 3; ++a) {
        cplx t = {0, 0};
        /* (U^dag)_ab = conj(U_ba) */
        for (int b = 0; b < 3; ++b) t = c_add(t, c_cjmul(ub[3 * b + a], pb[b]));
        acc[a] = c_sub(acc[a], c_scale(t, e * bb));
      }
      if (!W) continue;
      /* three-hop terms: walk three unit steps, multiplying their boundary factors */
      int c3[4], tmp[4];
      double b3 = 1.0;
      for (int k = 0; k < 4; ++k) c3[k] = c[k];
      for (int st = 0; st < 3; ++st) {
        b3 *= neighbour(dims, bc, c3, mu, +1, tmp);
        for (int k = 0; k < 4; ++k) c3[k] = tmp[k];
      }
      const cplx *wf = link(W, dims, mu, idx);
      const cplx *qf = in + (index_of(dims, c3) >> 1) * 3;
      for (int a = 0; a < 3; ++a) {
        cplx t = {0, 0};
        for (int b = 0; b < 3; ++b) t = c_add(t, c_mul(wf[3 * a + b], qf[b]));
        acc[a] = c_add(acc[a], c_scale(t, e * b3));
      }
      b3 = 1.0;
      for (int k = 0; k < 4; ++k) c3[k] = c[k];
      for (int st = 0; st < 3; ++st) {
        b3 *= neighbour(dims, bc, c3, mu, -1, tmp);
        for (int k = 0; k < 4; ++k) c3[k] = tmp[k];
      }
      long n3 = index_of(dims, c3);
      const cplx *wb = link(W, dims, mu, n3);
      const cplx *qb = in + (n3 >> 1) * 3;
      for (int a = 0; a < 3; ++a) {
        cplx t = {0, 0};
        for (int b = 0; b < 3; ++b) t = c_add(t, c_cjmul(wb[3 * b + a], qb[b]));
        acc[a] = c_sub(acc[a], c_scale(t, e * b3));
      }
    }
    for (int a = 0; a < 3; ++a) out[s * 3 + a] = acc[a];
  }
}

void ora_dslash_half(const int *dims, const int *bc, const double *Ud, int par_out,
                     const double *in_d, double *out_d) {
  ora_dslash_half_imp(dims, bc, Ud, NULL, par_out, in_d, out_d);
}

/* out = (A + sigma) in = (m^2 + sigma) in - D_eo D_oe in, on even sites */
void ora_mdagm_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
                   double sigma, const double *in_d, double *out_d) {
  long n = volume(dims) / 2 * 3;
  double *tmp = (double *)malloc(sizeof(double) * 2 * n);
  double *tmp2 = (double *)malloc(sizeof(double) * 2 * n);
  ora_dslash_half_imp(dims, bc, U, W, 1, in_d, tmp);   /* D_oe: even -> odd */
  ora_dslash_half_imp(dims, bc, U, W, 0, tmp, tmp2);   /* D_eo: odd -> even */
  double d = mass * mass + sigma;
  for (long i = 0; i < 2 * n; ++i) out_d[i] = d * in_d[i] - tmp2[i];
  free(tmp);
  free(tmp2);
}

void ora_mdagm(const int *dims, const int *bc, const double *U, double mass, double sigma,
               const double *in_d, double *out_d) {
  ora_mdagm_imp(dims, bc, U, NULL, mass, sigma, in_d, out_d);
}

/* ---- linear algebra helpers (plain loops) ------------------------------ */

static double dot_re(long n, const cplx *a, const cplx *b) {
  double s = 0;
  for (long i = 0; i < n; ++i) s += a[i].re * b[i].re + a[i].im * b[i].im;
  return s;
}

static double norm2(long n, const cplx *a) { return dot_re(n, a, a); }

/* ---- CG on (A + sigma) x = b, starting from x = 0 ------------------------ */
/* Returns the number of iterations; *true_rel receives |b - (A+s)x| / |b|. */
int ora_cg_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
               double sigma, const double *b_d, double *x_d, double tol, int maxiter,
               double *true_rel) {
  long n = volume(dims) / 2 * 3;
  const cplx *b = (const cplx *)b_d;
  cplx *x = (cplx *)x_d;
  cplx *r = (cplx *)malloc(sizeof(cplx) * n);
  cplx *p = (cplx *)malloc(sizeof(cplx) * n);
  cplx *ap = (cplx *)malloc(sizeof(cplx) * n);
  for (long i = 0; i < n; ++i) { x[i].re = x[i].im = 0; r[i] = b[i]; p[i] = b[i]; }
  double bb = norm2(n, b);
  double rr = bb;
  int k = 0;
  if (bb > 0) {
    while (k < maxiter && rr > tol * tol * bb) {
      ora_mdagm_imp(dims, bc, U, W, mass, sigma, (const double *)p, (double *)ap);
      double alpha = rr / dot_re(n, p, ap);
      for (long i = 0; i < n; ++i) {
        x[i] = c_add(x[i], c_scale(p[i], alpha));
        r[i] = c_sub(r[i], c_scale(ap[i], alpha));
      }
      double rr_new = norm2(n, r);
      double beta = rr_new / rr;
      rr = rr_new;
      for (long i = 0; i < n; ++i) p[i] = c_add(r[i], c_scale(p[i], beta));
      ++k;
    }
  }
  if (true_rel) {
    ora_mdagm_imp(dims, bc, U, W, mass, sigma, x_d, (double *)ap);
    double s = 0;
    for (long i = 0; i < n; ++i) {
      cplx d = c_sub(b[i], ap[i]);
      s += d.re * d.re + d.im * d.im;
    }
    *true_rel = bb > 0 ? sqrt(s / bb) : 0.0;
  }
  free(r);
  free(p);
  free(ap);
  return k;
}

/* ---- multi-shift CG -------------------------------------------------- */
/*
 * Solves (A + shifts[s]) x_s = b for all s from x_s = 0. shifts[0] must be
 * the smallest shift: the unshifted recurrence runs on it. For s > 0 the
 * residual of system s is zeta_s r, with zeta from the standard multi-shift
 * relation (derived from matching the three-term CG recurrences):
 *   zeta_{k+1} = zeta_k zeta_{k-1} a_{k-1} /
 *       ( zeta_{k-1} a_{k-1} (1 + a_k d_s) + a_k b_{k-1} (zeta_{k-1} - zeta_k) )
 *   a^s_k = a_k zeta_{k+1}/zeta_k,  b^s_k = b_k (zeta_{k+1}/zeta_k)^2
 * with d_s = shifts[s] - shifts[0]. Iterates until every system's residual
 * |zeta_s| |r| <= tol |b|. x has layout x[s][cb][color]. Returns iterations;
 * true_rel[s] receives the true relative residual of each system.
 */
int ora_mscg_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
                 int nshift, const double *shifts, const double *b_d, double *x_d, double tol,
                 int maxiter, double *true_rel) {
  long n = volume(dims) / 2 * 3;
  const cplx *b = (const cplx *)b_d;
  cplx *x = (cplx *)x_d;
  cplx *r = (cplx *)malloc(sizeof(cplx) * n);
  cplx *ap = (cplx *)malloc(sizeof(cplx) * n);
  cplx *p = (cplx *)malloc(sizeof(cplx) * n * nshift);
  double *zeta = (double *)malloc(sizeof(double) * nshift);
  double *zeta_old = (double *)malloc(sizeof(double) * nshift);
  int *active = (int *)malloc(sizeof(int) * nshift);
  for (int s = 0; s < nshift; ++s) {
    zeta[s] = zeta_old[s] = 1.0;
    active[s] = 1;
    for (long i = 0; i < n; ++i) {
      x[s * n + i].re = x[s * n + i].im = 0;
      p[s * n + i] = b[i];
    }
  }
  for (long i = 0; i < n; ++i) r[i] = b[i];
  double bb = norm2(n, b);
  double rr = bb;
  double a_old = 1.0, b_old = 0.0;
  int k = 0;
  if (bb > 0) {
    for (; k < maxiter; ++k) {
      int any = 0;
      for (int s = 0; s < nshift; ++s) {
        if (active[s] && zeta[s] * zeta[s] * rr <= tol * tol * bb) active[s] = 0;
        any |= active[s];
      }
      if (!any) break;
      ora_mdagm_imp(dims, bc, U, W, mass, shifts[0], (const double *)p, (double *)ap);
      double a = rr / dot_re(n, p, ap);
      /* shifted coefficients use zeta_k, zeta_{k-1}, a_{k-1}, b_{k-1} */
      for (int s = 1; s < nshift; ++s) {
        if (!active[s]) continue;
        double d = shifts[s] - shifts[0];
        double znew = zeta[s] * zeta_old[s] * a_old /
                      (zeta_old[s] * a_old * (1.0 + a * d) + a * b_old * (zeta_old[s] - zeta[s]));
        double as = a * znew / zeta[s];
        for (long i = 0; i < n; ++i) x[s * n + i] = c_add(x[s * n + i], c_scale(p[s * n + i], as));
        zeta_old[s] = zeta[s];
        zeta[s] = znew;
      }
      for (long i = 0; i < n; ++i) {
        x[i] = c_add(x[i], c_scale(p[i], a));
        r[i] = c_sub(r[i], c_scale(ap[i], a));
      }
      double rr_new = norm2(n, r);
      double beta = rr_new / rr;
      rr = rr_new;
      for (long i = 0; i < n; ++i) p[i] = c_add(r[i], c_scale(p[i], beta));
      for (int s = 1; s < nshift; ++s) {
        if (!active[s]) continue;
        double ratio = zeta[s] / zeta_old[s];
        double bs = beta * ratio * ratio;
        for (long i = 0; i < n; ++i)
          p[s * n + i] = c_add(c_scale(r[i], zeta[s]), c_scale(p[s * n + i], bs));
      }
      a_old = a;
      b_old = beta;
    }
  }
  if (true_rel) {
    for (int s = 0; s < nshift; ++s) {
      ora_mdagm_imp(dims, bc, U, W, mass, shifts[s], (const double *)(x + s * n), (double *)ap);
      double t = 0;
      for (long i = 0; i < n; ++i) {
        cplx dd = c_sub(b[i], ap[i]);
        t += dd.re * dd.re + dd.im * dd.im;
      }
      true_rel[s] = bb > 0 ? sqrt(t / bb) : 0.0;
    }
  }
  free(r);
  free(ap);
  free(p);
  free(zeta);
  free(zeta_old);
  free(active);
  return k;
}

/* ---- force: link gradient of S = sum_v coef[v] x_v^dag ... ---------------- */
int ora_cg(const int *dims, const int *bc, const double *U, double mass, double sigma,
           const double *b_d, double *x_d, double tol, int maxiter, double *true_rel) {
  return ora_cg_imp(dims, bc, U, NULL, mass, sigma, b_d, x_d, tol, maxiter, true_rel);
}

int ora_mscg(const int *dims, const int *bc, const double *U, double mass, int nshift,
             const double *shifts, const double *b_d, double *x_d, double tol, int maxiter,
             double *true_rel) {
  return ora_mscg_imp(dims, bc, U, NULL, mass, nshift, shifts, b_d, x_d, tol, maxiter, true_rel);
}

/*
 * x has layout x[v][cb][color] for nvec even-site solutions x_v = (A+s_v)^-1 phi
 * with residue coef[v]. Accumulates the per-link matrix M_mu(w) of the header
 * comment over all v and writes G = M^dag into g[mu][idx][a][b] (overwritten).
 */
void ora_force(const int *dims, const int *bc, const double *Ud, int nvec, const double *coef,
               const double *x_d, double *g_d) {
  const cplx *x = (const cplx *)x_d;
  cplx *g = (cplx *)g_d;
  long V = volume(dims);
  long vh = V / 2;
  long n = vh * 3;
  cplx *m = (cplx *)calloc((size_t)4 * V * 9, sizeof(cplx));
  cplx *y = (cplx *)malloc(sizeof(cplx) * n);
  for (int v = 0; v < nvec; ++v) {
    const cplx *xv = x + (long)v * n;
    ora_dslash_half(dims, bc, Ud, 1, (const double *)xv, (double *)y); /* y = D_oe x */
#pragma omp parallel for schedule(static)
    for (long idx = 0; idx < V; ++idx) {
      int c[4], nc[4];
      coords_of(dims, idx, c);
      int par = (c[0] + c[1] + c[2] + c[3]) & 1;
      for (int mu = 0; mu < 4; ++mu) {
        double bf = neighbour(dims, bc, c, mu, +1, nc);
        long nidx = index_of(dims, nc);
        double f = eta(c, mu) * bf * coef[v];
        const cplx *col, *row;  /* M += f * col row^dag */
        if (par == 1) {         /* w odd: -eta b a x(w+mu) y(w)^dag */
          f = -f;
          col = xv + (nidx >> 1) * 3;
          row = y + (idx >> 1) * 3;
        } else {                /* w even: +eta b a y(w+mu) x(w)^dag */
          col = y + (nidx >> 1) * 3;
          row = xv + (idx >> 1) * 3;
        }
        cplx *mm = m + ((long)mu * V + idx) * 9;
        for (int a = 0; a < 3; ++a)
          for (int bb = 0; bb < 3; ++bb) {
            cplx t = c_cjmul(row[bb], col[a]); /* col[a] * conj(row[b]) */
            mm[3 * a + bb] = c_add(mm[3 * a + bb], c_scale(t, f));
          }
      }
    }
  }
  for (long l = 0; l < 4 * V; ++l)
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb) {
        cplx t = m[l * 9 + 3 * bb + a];
        t.im = -t.im;
        g[l * 9 + 3 * a + bb] = t;
      }
  free(m);
  free(y);
}
