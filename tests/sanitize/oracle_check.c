/* Test infrastructure: exercises every exported routine of the C oracle
 * (oracle/staggered.c) on a small lattice, for a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer. Besides the sanitizers' own checks it tests
 * what holds exactly: D_eo = -D_oe^dag (the staggered hop is anti-Hermitian),
 * A = m^2 - D_eo D_oe is Hermitian, and CG / multi-shift CG meet their
 * tolerance in the true residual. Prints "ok" and returns 0 on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void ora_dslash_half_imp(const int *dims, const int *bc, const double *Ud, const double *Wd,
                         int par_out, const double *in_d, double *out_d);
void ora_dslash_half(const int *dims, const int *bc, const double *Ud, int par_out,
                     const double *in_d, double *out_d);
void ora_mdagm_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
                   double sigma, const double *in_d, double *out_d);
void ora_mdagm(const int *dims, const int *bc, const double *U, double mass, double sigma,
               const double *in_d, double *out_d);
int ora_cg_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
               double sigma, const double *b_d, double *x_d, double tol, int maxiter,
               double *true_rel);
int ora_mscg_imp(const int *dims, const int *bc, const double *U, const double *W, double mass,
                 int nshift, const double *shifts, const double *b_d, double *x_d, double tol,
                 int maxiter, double *true_rel);
int ora_cg(const int *dims, const int *bc, const double *U, double mass, double sigma,
           const double *b_d, double *x_d, double tol, int maxiter, double *true_rel);
int ora_mscg(const int *dims, const int *bc, const double *U, double mass, int nshift,
             const double *shifts, const double *b_d, double *x_d, double tol, int maxiter,
             double *true_rel);
void ora_force(const int *dims, const int *bc, const double *Ud, int nvec, const double *coef,
               const double *x_d, double *g_d);

static unsigned long long rng = 88172645463325252ULL;
static double urand(void) {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (double)(rng >> 11) / 9007199254740992.0 - 0.5;
}
static double *randv(long n) {
  double *v = (double *)malloc(sizeof(double) * n);
  for (long i = 0; i < n; ++i) v[i] = urand();
  return v;
}
/* Re and Im of a^dag b over n complex numbers */
static void cdot(long n, const double *a, const double *b, double *re, double *im) {
  double r = 0, m = 0;
  for (long i = 0; i < n; ++i) {
    r += a[2 * i] * b[2 * i] + a[2 * i + 1] * b[2 * i + 1];
    m += a[2 * i] * b[2 * i + 1] - a[2 * i + 1] * b[2 * i];
  }
  *re = r;
  *im = m;
}

static int fail(const char *what, double v) {
  printf("FAILED %s: %g\n", what, v);
  return 1;
}

int main(void) {
  const int dims[4] = {4, 2, 2, 6}, bc[4] = {1, 1, 1, -1};
  const long V = 4L * 2 * 2 * 6, vh = V / 2, n = 3 * vh;
  /* generic complex links (the identities below do not need SU(3)) */
  double *U = randv(4 * V * 9 * 2), *W = randv(4 * V * 9 * 2);
  double *e = randv(2 * n), *o = randv(2 * n);
  double *t1 = randv(2 * n), *t2 = randv(2 * n);
  double r1, i1, r2, i2;
  int bad = 0;
  for (int imp = 0; imp < 2; ++imp) {
    const double *w = imp ? W : NULL;
    /* <o, D_oe e> = -conj <e, D_eo o> */
    ora_dslash_half_imp(dims, bc, U, w, 1, e, t1);
    ora_dslash_half_imp(dims, bc, U, w, 0, o, t2);
    cdot(n, o, t1, &r1, &i1);
    cdot(n, e, t2, &r2, &i2);
    if (fabs(r1 + r2) + fabs(i1 - i2) > 1e-12 * (fabs(r1) + fabs(i1) + 1))
      bad |= fail("anti-Hermitian hop", fabs(r1 + r2) + fabs(i1 - i2));
    /* <o, A e> = conj <e, A o> for even-site o, e */
    ora_mdagm_imp(dims, bc, U, w, 0.1, 0.2, e, t1);
    ora_mdagm_imp(dims, bc, U, w, 0.1, 0.2, o, t2);
    cdot(n, o, t1, &r1, &i1);
    cdot(n, e, t2, &r2, &i2);
    if (fabs(r1 - r2) + fabs(i1 + i2) > 1e-11 * (fabs(r1) + fabs(i1) + 1))
      bad |= fail("Hermitian A", fabs(r1 - r2) + fabs(i1 + i2));
  }
  ora_dslash_half(dims, bc, U, 1, e, t1);
  ora_mdagm(dims, bc, U, 0.3, 0.0, e, t2);
  /* CG and multi-shift CG: true residuals within tol */
  double rel = 1, rels[3] = {1, 1, 1};
  double *x = (double *)calloc(2 * n, sizeof(double));
  int it = ora_cg(dims, bc, U, 0.5, 0.1, e, x, 1e-10, 2000, &rel);
  if (!(it > 0 && rel <= 1e-10)) bad |= fail("cg residual", rel);
  it = ora_cg_imp(dims, bc, U, W, 0.5, 0.1, e, x, 1e-10, 4000, &rel);
  if (!(it > 0 && rel <= 1e-10)) bad |= fail("improved cg residual", rel);
  const double sh[3] = {0.0, 0.05, 0.7};
  double *xs = (double *)calloc(3 * 2 * n, sizeof(double));
  it = ora_mscg(dims, bc, U, 0.5, 3, sh, e, xs, 1e-10, 2000, rels);
  for (int s = 0; s < 3; ++s)
    if (!(it > 0 && rels[s] <= 1e-10)) bad |= fail("mscg residual", rels[s]);
  it = ora_mscg_imp(dims, bc, U, W, 0.5, 3, sh, e, xs, 1e-10, 4000, rels);
  for (int s = 0; s < 3; ++s)
    if (!(it > 0 && rels[s] <= 1e-10)) bad |= fail("improved mscg residual", rels[s]);
  /* force of two solution vectors: finite output */
  const double coef[2] = {0.3, -0.2};
  double *g = (double *)malloc(sizeof(double) * 4 * V * 9 * 2);
  ora_force(dims, bc, U, 2, coef, xs, g);
  for (long i = 0; i < 4 * V * 9 * 2; ++i)
    if (!isfinite(g[i])) {
      bad |= fail("force not finite", (double)i);
      break;
    }
  free(U);
  free(W);
  free(e);
  free(o);
  free(t1);
  free(t2);
  free(x);
  free(xs);
  free(g);
  if (!bad) printf("ok\n");
  return bad;
}
