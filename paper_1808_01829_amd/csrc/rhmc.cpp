// bms_rhmc_trajectory: one RHMC trajectory on the GPU (Sec. II; the run
// settings of Sec. IV), every step in the library's kernels:
//   heatbath     phi = r_hb(A) eta (block multi-shift solve at tol_hb),
//   energies     H = 1/2 sum (P^a)^2 + S_g(U) + S_f(U, phi) with the accept
//                rational at tol_hb,
//   MD           two-level second-order Omelyan integration: the fermion
//                force (force rational, solves at tol_md) on the outer level
//                with step tau / n_steps; each outer drift of the links is n_gauge
//                inner Omelyan steps of the Wilson gauge force; adjacent kicks
//                of consecutive steps are merged,
//   final H and dH.
// The caller draws P and eta, keeps a copy of U and decides acceptance.
#include <string.h>

#include <cmath>
#include <vector>

#include "internal.h"

namespace {

struct Traj {
  bms_ctx* c;
  const bms_rhmc_params* p;
  void* U;
  void* P;
  void* phi;
  void* X;
  bms_opts o_md, o_hb;
  bms_rhmc_result* r;
};

int fermion_action(Traj& t, double* S) {
  const bms_rhmc_params& p = *t.p;
  int rc = bms_set_gauge(t.c, t.U);
  if (rc) return rc;
  bms_stats st;
  memset(&st, 0, sizeof st);
  rc = bms_solve(t.c, p.mass, p.n, p.ns_acc, p.beta_acc, p.tol_hb, p.max_iter, &t.o_hb, t.phi,
                 t.X, &st);
  t.r->iterations += st.iterations;
  t.r->max_residual_hb = std::max(t.r->max_residual_hb, st.max_true_residual);
  if (rc) return rc;
  std::vector<double> s(p.n);
  if ((rc = bms_action(t.c, p.n, p.ns_acc, p.a0_acc, p.alpha_acc, t.phi, t.X, s.data())))
    return rc;
  double sum = 0;
  for (double v : s) sum += v;
  *S = sum;
  return BMS_OK;
}

// P += e F_f(U, phi)
int fermion_kick(Traj& t, double e) {
  const bms_rhmc_params& p = *t.p;
  if (p.n == 0 || e == 0) return BMS_OK;
  int rc = bms_set_gauge(t.c, t.U);
  if (rc) return rc;
  bms_stats st;
  memset(&st, 0, sizeof st);
  rc = bms_solve(t.c, p.mass, p.n, p.ns_md, p.beta_md, p.tol_md, p.max_iter, &t.o_md, t.phi, t.X,
                 &st);
  t.r->iterations += st.iterations;
  t.r->force_evals += 1;
  if (rc) return rc;
  // the force is linear in the residues: e F = F(e alpha)
  std::vector<double> al(p.ns_md);
  for (int j = 0; j < p.ns_md; ++j) al[j] = e * p.alpha_md[j];
  return bms_force(t.c, p.n, p.ns_md, al.data(), t.X, t.P, BMS_FORCE_LIE | BMS_FORCE_ADD);
}

// Omelyan steps of the gauge part for a drift of the links over time `len`
int gauge_drift(Traj& t, double len) {
  const bms_rhmc_params& p = *t.p;
  const int m = p.n_gauge;
  const double g = len / m, lam = p.lambda;
  int rc;
  if ((rc = gauge_force_dev(t.c, p.beta, t.U, t.P, lam * g))) return rc;
  for (int k = 0; k < m; ++k) {
    if ((rc = link_update_dev(t.c, 0.5 * g, t.P, t.U))) return rc;
    if ((rc = gauge_force_dev(t.c, p.beta, t.U, t.P, (1.0 - 2.0 * lam) * g))) return rc;
    if ((rc = link_update_dev(t.c, 0.5 * g, t.P, t.U))) return rc;
    if ((rc = gauge_force_dev(t.c, p.beta, t.U, t.P, (k < m - 1 ? 2.0 : 1.0) * lam * g))) return rc;
  }
  return BMS_OK;
}

int energies(Traj& t, double* K, double* Sg, double* Sf) {
  int rc;
  if ((rc = kinetic_dev(t.c, t.P, K))) return rc;
  if ((rc = gauge_action_dev(t.c, t.p->beta, t.U, Sg))) return rc;
  *Sf = 0;
  if (t.p->n > 0 && (rc = fermion_action(t, Sf))) return rc;
  return BMS_OK;
}

bool finite_all(int n, const double* v) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

extern "C" void bms_default_rhmc_params(bms_rhmc_params* p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->beta = 5.12;
  p->mass = 0.05;
  p->n = 1;
  p->tau = 1.0;
  p->n_steps = 10;
  p->n_gauge = 3;
  p->lambda = 1.0 / 6.0;
  p->tol_hb = 1e-14;
  p->tol_md = 1e-7;
  p->precision_md = BMS_PREC_F64;
  p->max_iter = 100000;
}

extern "C" int bms_rhmc_trajectory(bms_ctx* c, const bms_rhmc_params* p, void* U, void* P,
                                   const void* eta, bms_rhmc_result* r) {
  if (!c) return BMS_EINVAL;
  if (!p || !U || !P || !r) return set_err(c, BMS_EINVAL, "null pointer");
  if (p->n < 0 || p->n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [0, 32]");
  if (p->n > 0 && !eta) return set_err(c, BMS_EINVAL, "eta is NULL");
  if (!(p->tau > 0) || p->n_steps < 1 || p->n_gauge < 1 || !std::isfinite(p->tau))
    return set_err(c, BMS_EINVAL, "need tau > 0, n_steps >= 1, n_gauge >= 1");
  if (!std::isfinite(p->beta) || !std::isfinite(p->lambda) || !std::isfinite(p->mass))
    return set_err(c, BMS_EINVAL, "beta, lambda and mass must be finite");
  if (p->n > 0) {
    const int ns[3] = {p->ns_hb, p->ns_acc, p->ns_md};
    const double* al[3] = {p->alpha_hb, p->alpha_acc, p->alpha_md};
    const double* be[3] = {p->beta_hb, p->beta_acc, p->beta_md};
    for (int k = 0; k < 3; ++k) {
      if (ns[k] < 1 || ns[k] > BMS_MAX_SHIFTS || !al[k] || !be[k])
        return set_err(c, BMS_EINVAL, "rational approximation %d: bad pole count or NULL", k);
      if (!finite_all(ns[k], al[k]) || !finite_all(ns[k], be[k]))
        return set_err(c, BMS_EINVAL, "rational approximation %d: non-finite coefficient", k);
    }
    if (!(p->tol_hb > 0 && p->tol_hb < 1) || !(p->tol_md > 0 && p->tol_md < 1))
      return set_err(c, BMS_EINVAL, "tolerances must be in (0, 1)");
    if (p->precision_md != BMS_PREC_F64 && p->precision_md != BMS_PREC_MIXED)
      return set_err(c, BMS_EINVAL, "precision_md must be BMS_PREC_F64 or BMS_PREC_MIXED");
  }
  memset(r, 0, sizeof *r);
  int rc = stream_begin(c);
  if (rc) return rc;
  Traj t;
  t.c = c;
  t.p = p;
  t.U = U;
  t.P = P;
  t.r = r;
  t.phi = t.X = nullptr;
  bms_default_opts(&t.o_hb);
  bms_default_opts(&t.o_md);
  t.o_md.precision = p->precision_md;
  if (p->n > 0) {
    const size_t blk = (size_t)3 * c->vh * p->n;
    const int nsx = std::max(p->ns_hb, std::max(p->ns_acc, p->ns_md));
    if ((rc = scratch_buf(c, S_PHI, blk * sizeof(double2), &t.phi))) return rc;
    if ((rc = scratch_buf(c, S_XR, (size_t)nsx * blk * sizeof(double2), &t.X))) return rc;
    // heatbath phi = r_hb(A) eta
    if ((rc = bms_set_gauge(c, U))) return rc;
    bms_stats st;
    memset(&st, 0, sizeof st);
    rc = bms_rational_apply(c, p->mass, p->n, p->ns_hb, p->a0_hb, p->alpha_hb, p->beta_hb,
                            p->tol_hb, p->max_iter, &t.o_hb, eta, t.X, t.phi, &st);
    r->iterations += st.iterations;
    r->max_residual_hb = st.max_true_residual;
    if (rc) return rc;
  }
  if ((rc = energies(t, &r->K0, &r->Sg0, &r->Sf0))) return rc;
  // two-level Omelyan integration over tau
  const double h = p->tau / p->n_steps, lam = p->lambda;
  if ((rc = fermion_kick(t, lam * h))) return rc;
  for (int k = 0; k < p->n_steps; ++k) {
    if ((rc = gauge_drift(t, 0.5 * h))) return rc;
    if ((rc = fermion_kick(t, (1.0 - 2.0 * lam) * h))) return rc;
    if ((rc = gauge_drift(t, 0.5 * h))) return rc;
    if ((rc = fermion_kick(t, (k < p->n_steps - 1 ? 2.0 : 1.0) * lam * h))) return rc;
  }
  if ((rc = energies(t, &r->K1, &r->Sg1, &r->Sf1))) return rc;
  r->H0 = r->K0 + r->Sg0 + r->Sf0;
  r->H1 = r->K1 + r->Sg1 + r->Sf1;
  r->dH = r->H1 - r->H0;
  if (!std::isfinite(r->dH)) return set_err(c, BMS_ENAN, "non-finite energy in the trajectory");
  return stream_end(c);
}
