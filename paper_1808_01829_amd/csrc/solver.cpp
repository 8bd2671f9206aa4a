// bms_solve: host driver of the block multi-shift solver (Algorithm 1).
//
// Per iteration the device runs
//   hop D_oe P^(0) -> W1;  hop D_eo W1 -> W = (m^2 + s0) P^(0) - D_eo W1
//   G_k = P^(0)H W                          (Gram, FP64)
//   alpha_k, beta^(s)_k, alpha^(s)_k        (small kernel, one WG per shift)
//   G_V = V^H V, V = Q_{k-1} - W alpha_k    (Cholesky-QR Gram, FP64)
//   rho_k, delta_k, delta^(s)_k, Mp[s]       (small kernel, convergence)
//   Q_k, X^(s), P^(s) for all active shifts (fused update)
// The host only enqueues chunks of iterations (optionally as a captured
// hipGraph) and reads a small flag block between chunks; stopping, freezing
// of converged shifts and the iteration limit are decided on the device.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "blas.h"

namespace {

enum Slot {
  S_TMP = 0,  // used by bms_apply_mdagm
  S_W1,
  S_W,
  S_Q,
  S_P,
  S_X,
  S_SMALL,
  S_PART,
  S_M,
  S_FLAGS,
  S_RES,
  S_X64,
  S_B32,
  S_LOG,
  S_COUNT
};

struct Work {
  int rows, n, ns;
  size_t blk;  // complex elements per block vector
  void *W1, *W, *Q, *P, *X, *Mx, *Mp;
  SmallState sm;
  SolverFlags* flags;
  double2* partials;
  int* counters;  // [0] gram, [1] cholqr gram, [2] residual / misc
  double2* Rinv;
  int nb;
};

template <typename T>
int alloc_work(bms_ctx* c, int n, int ns, int max_iter, Work& w) {
  int rc;
  w.n = n;
  w.ns = ns;
  w.rows = 3 * c->vh;
  w.blk = (size_t)w.rows * n;
  size_t es = sizeof(cplx<T>);
  if ((rc = scratch_buf(c, S_W1, w.blk * es, &w.W1))) return rc;
  if ((rc = scratch_buf(c, S_W, w.blk * es, &w.W))) return rc;
  if ((rc = scratch_buf(c, S_Q, w.blk * es, &w.Q))) return rc;
  if ((rc = scratch_buf(c, S_P, w.blk * es * ns, &w.P))) return rc;
  if ((rc = scratch_buf(c, S_X, w.blk * es * ns, &w.X))) return rc;
  size_t nn = (size_t)n * n;
  size_t small_elems = 2 * nn + 2 * nn + 5 * nn + 2 * ns * nn + 2 * nn + n;
  void* sp;
  if ((rc = scratch_buf(c, S_SMALL, small_elems * sizeof(double2) + 64, &sp))) return rc;
  double2* d = (double2*)sp;
  w.sm.Gb = d;
  d += 2 * nn;
  w.sm.rhob = d;
  d += 2 * nn;
  w.sm.alpha = d;
  d += nn;
  w.sm.rhoinv = d;
  d += nn;
  w.sm.delta = d;
  d += nn;
  w.sm.Ggram = d;
  d += nn;
  w.sm.Gqr = d;
  d += nn;
  w.sm.beta_s = d;
  d += ns * nn;
  w.sm.alpha_s = d;
  d += ns * nn;
  w.sm.tmp = d;
  d += nn;
  w.Rinv = d;
  d += nn;
  w.sm.norm0 = (double*)d;
  w.nb = gram_blocks(w.rows, n);
  void* pp;
  if ((rc = scratch_buf(c, S_PART, (size_t)w.nb * nn * sizeof(double2) + 64, &pp))) return rc;
  w.partials = (double2*)pp;
  void* mp;
  if ((rc = scratch_buf(c, S_M, 2 * ns * nn * es, &mp))) return rc;
  w.Mx = mp;
  w.Mp = (char*)mp + ns * nn * es;
  void* fp;
  if ((rc = scratch_buf(c, S_FLAGS, sizeof(SolverFlags) + 64, &fp))) return rc;
  w.flags = (SolverFlags*)fp;
  w.counters = (int*)((char*)fp + sizeof(SolverFlags));
  w.sm.counter = w.counters + 3;
  void* lp;
  if ((rc = scratch_buf(c, S_LOG, (size_t)max_iter * sizeof(int) + 64, &lp))) return rc;
  w.sm.nact_log = (int*)lp;
  return BMS_OK;
}

struct HostFlags {
  SolverFlags f;
};

// kernel classes of the 7 launches of one iteration (timing)
const int kIterKernel[7] = {BMS_KERNEL_HOP,   BMS_KERNEL_HOP,    BMS_KERNEL_GRAM,  BMS_KERNEL_SMALL,
                            BMS_KERNEL_CHOLQR, BMS_KERNEL_SMALL, BMS_KERNEL_UPDATE};

template <typename T>
int enqueue_iteration(bms_ctx* c, const Work& w, const SmallParams& sp, double mass,
                      hipEvent_t* ev) {
  const int* skip = &w.flags->stop;
  cplx<T>* P0 = (cplx<T>*)w.P;
#define MARK(i) \
  if (ev) HIP_TRY(c, hipEventRecord(ev[i], c->stream))
  MARK(0);
  HIP_TRY(c, launch_hop<T>(c, 1, w.n, P0, w.W1, nullptr, 0.0, 1.0, skip));
  MARK(1);
  HIP_TRY(c, launch_hop<T>(c, 0, w.n, w.W1, w.W, P0, mass * mass + sp.sigma[0], -1.0, skip));
  MARK(2);
  HIP_TRY(c, launch_gram<T>(c->stream, w.rows, w.n, P0, w.W, w.sm.Ggram, w.partials,
                            w.counters + 0, w.nb, skip));
  MARK(3);
  HIP_TRY(c, launch_small_alpha<T>(c->stream, sp, w.sm, w.flags, (cplx<T>*)w.Mx));
  MARK(4);
  HIP_TRY(c, launch_cholqr_gram<T>(c->stream, w.rows, w.n, w.Q, w.W, w.sm.alpha, w.sm.Gqr,
                                   w.partials, w.counters + 1, w.nb, skip));
  MARK(5);
  HIP_TRY(c, launch_small_rho<T>(c->stream, sp, w.sm, w.flags, (cplx<T>*)w.Mp));
  MARK(6);
  UpdateArgs<T, T> ua;
  ua.rows = w.rows;
  ua.n = w.n;
  ua.ns = w.ns;
  ua.Q = (cplx<T>*)w.Q;
  ua.W = (const cplx<T>*)w.W;
  ua.alpha = w.sm.alpha;
  ua.rhoinv = w.sm.rhoinv;
  ua.P = (cplx<T>*)w.P;
  ua.X = (cplx<T>*)w.X;
  ua.Mx = (const cplx<T>*)w.Mx;
  ua.Mp = (const cplx<T>*)w.Mp;
  ua.flags = w.flags;
  for (int s = 0; s < BMS_MAX_SHIFTS; ++s) ua.xidx[s] = s < w.ns ? s : 0;
  HIP_TRY(c, (launch_update<T, T>(c->stream, ua)));
  MARK(7);
#undef MARK
  return BMS_OK;
}

// Q_0 delta_0 = B by Cholesky-QR applied twice; P^(s) = Q_0, X^(s) = 0.
template <typename T>
int enqueue_setup(bms_ctx* c, const Work& w, const SmallParams& sp, const void* B) {
  size_t es = sizeof(cplx<T>);
  // grid-completion counters must start at zero (they are left at zero after use)
  HIP_TRY(c, launch_fill_zero(c->stream, w.counters, 64));
  HIP_TRY(c, launch_fill_zero(c->stream, w.X, w.blk * es * w.ns));
  HIP_TRY(c, launch_gram<T>(c->stream, w.rows, w.n, B, B, w.sm.Ggram, w.partials, w.counters + 0,
                            w.nb, nullptr));
  HIP_TRY(c, launch_small_init(c->stream, sp, w.sm, w.flags, w.sm.Ggram, w.Rinv));
  HIP_TRY(c, launch_block_matmul<T>(c->stream, w.rows, w.n, B, w.Rinv, w.W));
  HIP_TRY(c, launch_gram<T>(c->stream, w.rows, w.n, w.W, w.W, w.sm.Ggram, w.partials,
                            w.counters + 0, w.nb, nullptr));
  HIP_TRY(c, launch_small_init_pass2(c->stream, sp, w.sm, w.flags, w.sm.Ggram, w.Rinv));
  HIP_TRY(c, launch_block_matmul<T>(c->stream, w.rows, w.n, w.W, w.Rinv, w.Q));
  for (int s = 0; s < w.ns; ++s)
    HIP_TRY(c, hipMemcpyAsync((char*)w.P + s * w.blk * es, w.Q, w.blk * es,
                              hipMemcpyDeviceToDevice, c->stream));
  return BMS_OK;
}

__attribute__((unused)) static int map_device_error(int e) { return e; }

}  // namespace

// true relative residuals |b_i - (A + s)x_i| / |b_i| of user-ordered solutions
int true_residuals(bms_ctx* c, double mass, int n, int ns, const double* shifts, const void* B,
                   const void* X, double* res_host) {
  int rc;
  int rows = 3 * c->vh;
  size_t blk = (size_t)rows * n;
  void *t1, *t2, *out;
  if ((rc = scratch_buf(c, S_W1, blk * sizeof(double2), &t1))) return rc;
  if ((rc = scratch_buf(c, S_W, blk * sizeof(double2), &t2))) return rc;
  if ((rc = scratch_buf(c, S_RES, (size_t)ns * n * sizeof(double2) + 64, &out))) return rc;
  int nb = gram_blocks(rows, n);
  void* pp;
  if ((rc = scratch_buf(c, S_PART, (size_t)nb * n * n * sizeof(double2) + 64, &pp))) return rc;
  void* fp;
  if ((rc = scratch_buf(c, S_FLAGS, sizeof(SolverFlags) + 64, &fp))) return rc;
  int* counter = (int*)((char*)fp + sizeof(SolverFlags)) + 2;
  for (int s = 0; s < ns; ++s) {
    const double2* xs = (const double2*)X + s * blk;
    HIP_TRY(c, launch_hop<double>(c, 1, n, xs, t1, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<double>(c, 0, n, t1, t2, xs, mass * mass + shifts[s], -1.0, nullptr));
    HIP_TRY(c, launch_resid_norms(c->stream, rows, n, B, t2, (double2*)out + (size_t)s * n,
                                  (double2*)pp, counter, nb));
  }
  std::vector<double2> h((size_t)ns * n);
  HIP_TRY(c, hipMemcpyAsync(h.data(), out, h.size() * sizeof(double2), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < h.size(); ++i)
    res_host[i] = h[i].y > 0 ? std::sqrt(h[i].x / h[i].y) : std::sqrt(h[i].x);
  return BMS_OK;
}

static int validate_solve(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                          double tol, int max_iter, const bms_opts* o, const void* B,
                          const void* X) {
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 1 || ns > BMS_MAX_SHIFTS)
    return set_err(c, BMS_EINVAL, "n_shifts must be in [1, %d]", BMS_MAX_SHIFTS);
  if (!shifts) return set_err(c, BMS_EINVAL, "shifts is NULL");
  for (int s = 0; s < ns; ++s)
    if (!(shifts[s] >= 0) || !std::isfinite(shifts[s]))
      return set_err(c, BMS_EINVAL, "shift %d is negative or not finite", s);
  if (!std::isfinite(mass)) return set_err(c, BMS_EINVAL, "mass not finite");
  if (!(tol > 0) || !(tol < 1)) return set_err(c, BMS_EINVAL, "tol must be in (0, 1)");
  if (max_iter < 1) return set_err(c, BMS_EINVAL, "max_iter must be >= 1");
  if (!B || !X) return set_err(c, BMS_EINVAL, "null B or X");
  if (B == X) return set_err(c, BMS_EINVAL, "B and X must not alias");
  if (o) {
    if (o->precision != BMS_PREC_F64 && o->precision != BMS_PREC_MIXED)
      return set_err(c, BMS_EINVAL, "opts.precision must be BMS_PREC_F64 or BMS_PREC_MIXED");
    if (o->check_interval < 1 || o->check_interval > 4096)
      return set_err(c, BMS_EINVAL, "opts.check_interval must be in [1, 4096]");
    if (o->qr_passes < 1 || o->qr_passes > 2)
      return set_err(c, BMS_EINVAL, "opts.qr_passes must be 1 or 2");
    if (o->precision == BMS_PREC_MIXED && o->reliable_interval < 1)
      return set_err(c, BMS_EINVAL, "opts.reliable_interval must be >= 1");
    if (o->max_refine < 0) return set_err(c, BMS_EINVAL, "opts.max_refine must be >= 0");
  }
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  return BMS_OK;
}

template <typename T>
static int solve_f64(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                     int max_iter, const bms_opts& o, const void* B, void* X, bms_stats* st) {
  int rc;
  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return shifts[a] < shifts[b]; });
  SmallParams sp;
  memset(&sp, 0, sizeof sp);
  sp.n = n;
  sp.ns = ns;
  sp.max_iter = max_iter;
  sp.tol = tol;
  double ft = o.freeze_tol > 0 ? o.freeze_tol : tol;
  sp.freeze_tol = ft < tol ? ft : tol;
  // a computed Gram resolves pivots only down to ~eps * trace
  sp.breakdown_tol = 10.0 * n * 2.220446049250313e-16;
  for (int s = 0; s < ns; ++s) sp.sigma[s] = shifts[order[s]];
  Work w;
  if ((rc = alloc_work<T>(c, n, ns, max_iter, w))) return rc;
  if ((rc = enqueue_setup<T>(c, w, sp, B))) return rc;
  SolverFlags hf;
  int K = o.check_interval;
  long enqueued = 0;
  if (c->timing && (int)c->evpool.size() < 8 * K) {
    size_t old = c->evpool.size();
    c->evpool.resize(8 * K);
    for (size_t i = old; i < c->evpool.size(); ++i) HIP_TRY(c, hipEventCreate(&c->evpool[i]));
  }
  std::vector<float> upd_ms;  // per completed iteration, update kernel time
  while (true) {
    for (int k = 0; k < K; ++k)
      if ((rc = enqueue_iteration<T>(c, w, sp, mass, c->timing ? &c->evpool[8 * k] : nullptr)))
        return rc;
    HIP_TRY(c, hipMemcpyAsync(&hf, w.flags, sizeof hf, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->timing) {
      double G = 72.0 * c->vol * sizeof(T);
      double S = (double)w.blk * sizeof(cplx<T>);
      const double kbytes[7] = {G + 2 * S, G + 3 * S, 2 * S, 0, 2 * S, 0, 0};
      for (int k = 0; k < K; ++k) {
        if (enqueued + k >= hf.iter) break;  // launches after the stop did no work
        for (int i = 0; i < 7; ++i) {
          float ms = 0;
          HIP_TRY(c, hipEventElapsedTime(&ms, c->evpool[8 * k + i], c->evpool[8 * k + i + 1]));
          int kc = kIterKernel[i];
          c->kt_ms[kc] += ms;
          c->kt_launches[kc] += 1;
          c->kt_bytes[kc] += kbytes[i];
          if (i == 6) upd_ms.push_back(ms);
        }
      }
    }
    enqueued += K;
    if (hf.stop) break;
    if (enqueued > (long)max_iter + 2L * K)  // the device stops itself at max_iter
      return set_err(c, BMS_EHIP, "device iteration control did not stop (iter %d)", hf.iter);
  }
  if (c->timing && hf.iter > 0) {
    std::vector<int> nact(hf.iter);
    HIP_TRY(c, hipMemcpyAsync(nact.data(), w.sm.nact_log, hf.iter * sizeof(int),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double S = (double)w.blk * sizeof(cplx<T>);
    for (int k = 0; k < hf.iter; ++k) c->kt_bytes[BMS_KERNEL_UPDATE] += (3.0 + 4.0 * nact[k]) * S;
  }
  // solutions back to the caller's shift order
  size_t bytes = w.blk * sizeof(double2);
  for (int s = 0; s < ns; ++s)
    HIP_TRY(c, hipMemcpyAsync((char*)X + (size_t)order[s] * bytes, (char*)w.X + (size_t)s * bytes,
                              bytes, hipMemcpyDeviceToDevice, c->stream));
  std::vector<double> res((size_t)ns * n);
  if ((rc = true_residuals(c, mass, n, ns, shifts, B, X, res.data()))) return rc;
  double mx = 0;
  for (double r : res) mx = std::max(mx, std::isfinite(r) ? r : 1e300);
  if (st) {
    st->iterations = hf.iter;
    st->hop_calls = 2 * hf.iter + 2 * ns;
    st->reliable_updates = 0;
    st->refine_iterations = 0;
    st->converged = mx <= tol;
    st->max_true_residual = mx;
    if (st->true_residual) memcpy(st->true_residual, res.data(), res.size() * sizeof(double));
  }
  if (hf.error) return set_err(c, hf.error, "device reported %s after %d iterations",
                               bms_error_string(hf.error), hf.iter);
  if (mx > tol)
    return set_err(c, BMS_ENOCONV, "max true residual %.3e > tol %.3e after %d iterations", mx,
                   tol, hf.iter);
  return BMS_OK;
}

extern "C" int bms_solve(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                         int max_iter, const bms_opts* opts, const void* B, void* X,
                         bms_stats* st) {
  if (!c) return BMS_EINVAL;
  int rc = validate_solve(c, mass, n, ns, shifts, tol, max_iter, opts, B, X);
  if (rc) return rc;
  bms_opts o;
  bms_default_opts(&o);
  if (opts) o = *opts;
  if ((rc = stream_begin(c))) return rc;
  if (o.precision == BMS_PREC_F64)
    rc = solve_f64<double>(c, mass, n, ns, shifts, tol, max_iter, o, B, X, st);
  else
    rc = set_err(c, BMS_EINVAL, "BMS_PREC_MIXED not available yet");
  int rc2 = stream_end(c);
  return rc ? rc : rc2;
}

extern "C" int bms_action(bms_ctx* c, int n, int ns, double a0, const double* alpha,
                          const void* B, const void* X, double* S) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 0 || ns > BMS_MAX_SHIFTS) return set_err(c, BMS_EINVAL, "bad n_shifts");
  if ((ns > 0 && (!alpha || !X)) || !B || !S) return set_err(c, BMS_EINVAL, "null pointer");
  int rc;
  if ((rc = stream_begin(c))) return rc;
  int rows = 3 * c->vh;
  void *al, *out, *pp, *fp;
  if ((rc = scratch_buf(c, S_RES, (size_t)(n + BMS_MAX_SHIFTS) * sizeof(double2) + 64, &out)))
    return rc;
  al = (double2*)out + n;
  int nb = gram_blocks(rows, n);
  if ((rc = scratch_buf(c, S_PART, (size_t)nb * n * n * sizeof(double2) + 64, &pp))) return rc;
  if ((rc = scratch_buf(c, S_FLAGS, sizeof(SolverFlags) + 64, &fp))) return rc;
  int* counter = (int*)((char*)fp + sizeof(SolverFlags)) + 2;
  if (ns > 0)
    HIP_TRY(c, hipMemcpyAsync(al, alpha, ns * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_action(c->stream, rows, n, ns, a0, (const double*)al, B, X, (double2*)out,
                           (double2*)pp, counter, nb));
  std::vector<double2> h(n);
  HIP_TRY(c, hipMemcpyAsync(h.data(), out, n * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) S[i] = h[i].x;
  return stream_end(c);
}
