// bms_solve: host driver of the block multi-shift solver (Algorithm 1).
//
// Per iteration the device runs
//   hop D_oe P^(0) -> W1;  hop D_eo W1 -> W = (m^2 + s0) P^(0) - D_eo W1
//   G4 = [P^H W, Q^H W, W^H W, Q^H Q]        (one pass, FP64)
//   alpha_k, beta^(s)_k, alpha^(s)_k, rho_k, delta^(s)_k, convergence
//                                            (one work-group per shift)
//   [explicit V^H V and rho_k, only if the expansion lost its pivot]
//   Q_k, X^(s), P^(s) for all active shifts  (fused update)
// The host only enqueues chunks of iterations and reads a small flag block
// between chunks; stopping, freezing of converged shifts and the iteration
// limit are decided on the device.
//
// Precision control. In BMS_PREC_MIXED the block vectors and the operator
// are FP32 (the n x n algebra stays FP64): every reliable_interval iterations
// the FP32 increments of every X^(s) are added into FP64 solutions and the
// unshifted residual is replaced by the true FP64 one (re-factored by
// Cholesky-QR). In both precisions, after the main solve every shift whose
// true FP64 residual misses tol is refined by defect correction: its residual
// block, column-normalised, is solved for with the same solver and added back.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "blas.h"

namespace {

const double kEps = 2.220446049250313e-16;
const double kEps32 = 1.1920928955078125e-07;
// the solver flags, then the arrival counter of the small-step blocks
const size_t kFlagsBytes = sizeof(SolverFlags) + 64;

// partial sums of a grid reduction over nb blocks of P entries
size_t part_bytes(int nb, int P) { return (size_t)nb * P * sizeof(double2) + 64; }

struct Work {
  int rows, n, ns;
  int win;     // update window of the shifts s >= 1 (1: every iteration)
  size_t blk;  // complex elements per block vector
  void *W1, *W, *Q, *P, *X, *Mx, *Mp, *Wm;
  SmallState sm;
  SolverFlags* flags;
  double2* partials;
  double2* Rinv;
  double2* Gtmp;
  int nb;
};

// Update window of the shifts s >= 1: the matrix-core update (variants -1, 4,
// 5 at n = 8, 16) applies each shift's X and P updates once per window of
// iterations; its length is the longest the kernel stages (4 in FP64, 8 in
// FP32) that divides the chunk of iterations between host checks, so that
// every window closes at a chunk's end (where the mixed solver's reliable
// update needs every X). Variant 6, the vector kernels and one shift: 1.
int update_window(const bms_ctx* c, int n, int ns, int elem_bytes, int check_interval) {
  const int uv = c->update_variant;
  if (ns < 2 || !update_mfma_supported(n) || !(uv < 0 || uv == 4 || uv == 5)) return 1;
  int w = elem_bytes == 8 ? update_mfma_max_win<double>() : update_mfma_max_win<float>();
  w = std::min(w, BMS_MAX_WIN);
  while (w > 1 && check_interval % w) w >>= 1;
  return w;
}

// n x n FP64 entries of the small state (SmallState), the window state included
size_t small_elems(int n, int ns) {
  const size_t nn = (size_t)n * n;
  return 2 * nn + 2 * nn + 8 * nn + 2 * ns * nn + 3 * nn + n + 1 +
         (size_t)2 * ns * 2 * BMS_MAX_WIN * nn;
}

template <typename T>
int alloc_work(bms_ctx* c, int n, int ns, int max_iter, int win, Work& w) {
  int rc;
  w.n = n;
  w.ns = ns;
  w.win = win;
  w.rows = 3 * c->vh;
  w.blk = (size_t)w.rows * n;
  size_t es = sizeof(cplx<T>);
  if ((rc = scratch_buf(c, S_W1, w.blk * es, &w.W1))) return rc;
  if ((rc = scratch_buf(c, S_W, w.blk * es, &w.W))) return rc;
  // Q_j in ring buffer j % win
  if ((rc = scratch_buf(c, S_Q, w.blk * es * win, &w.Q))) return rc;
  if ((rc = scratch_buf(c, S_P, w.blk * es * ns, &w.P))) return rc;
  if ((rc = scratch_buf(c, S_X, w.blk * es * ns, &w.X))) return rc;
  size_t nn = (size_t)n * n;
  void* sp;
  if ((rc = scratch_buf(c, S_SMALL, small_elems(n, ns) * sizeof(double2) + 64, &sp))) return rc;
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
  w.sm.G4 = d;
  d += 4 * nn;
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
  w.Gtmp = d;
  d += nn;
  w.sm.norm0 = (double*)d;
  w.sm.rel_last = (double*)d + n;
  d += n + 1;
  w.sm.wst = d;
  w.nb = gram_blocks(w.rows, n, c->num_cu);
  void* pp;
  if ((rc = scratch_buf(c, S_PART, part_bytes(w.nb, 4 * nn), &pp))) return rc;
  w.partials = (double2*)pp;
  void* mp;
  if ((rc = scratch_buf(c, S_M, (2 + 2 * BMS_MAX_WIN) * ns * nn * es, &mp))) return rc;
  w.Mx = mp;
  w.Mp = (char*)mp + ns * nn * es;
  w.Wm = (char*)mp + 2 * ns * nn * es;
  void* fp;
  if ((rc = scratch_buf(c, S_FLAGS, kFlagsBytes, &fp))) return rc;
  w.flags = (SolverFlags*)fp;
  w.sm.counter = (int*)((char*)fp + sizeof(SolverFlags));
  void* lp;
  if ((rc = scratch_buf(c, S_LOG, (size_t)max_iter * sizeof(int) + 64, &lp))) return rc;
  w.sm.upd_log = (int*)lp;
  return BMS_OK;
}

// kernel classes of the 7 launches of one iteration (timing)
const int kIterKernel[7] = {BMS_KERNEL_HOP,   BMS_KERNEL_HOP,   BMS_KERNEL_GRAM,  BMS_KERNEL_SMALL,
                            BMS_KERNEL_CHOLQR, BMS_KERNEL_SMALL, BMS_KERNEL_UPDATE};

template <typename T>
UpdateArgs<T, T> update_args(const Work& w) {
  UpdateArgs<T, T> ua;
  ua.rows = w.rows;
  ua.n = w.n;
  ua.ns = w.ns;
  ua.Q = (cplx<T>*)w.Q;
  ua.Qring = (cplx<T>*)w.Q;
  ua.W = (const cplx<T>*)w.W;
  ua.alpha = w.sm.alpha;
  ua.rhoinv = w.sm.rhoinv;
  ua.P = (cplx<T>*)w.P;
  ua.X = (cplx<T>*)w.X;
  ua.Mx = (const cplx<T>*)w.Mx;
  ua.Mp = (const cplx<T>*)w.Mp;
  ua.Wm = (const cplx<T>*)w.Wm;
  ua.wst = w.sm.wst;
  ua.win = w.win;
  ua.flags = w.flags;
  for (int s = 0; s < BMS_MAX_SHIFTS; ++s) ua.xidx[s] = s < w.ns ? s : 0;
  return ua;
}

// ev: NULL, or 8 timing events recorded around the 7 launches (direct
// launches only: event-record nodes of a replayed graph carry no usable
// timestamps on this runtime, measured).
// k: the iteration's index (Q_k is in ring buffer k % win).
template <typename T>
int enqueue_iteration(bms_ctx* c, const Work& w, const SmallParams& sp, double mass, long k,
                      hipEvent_t* ev) {
  const int* skip = &w.flags->stop;
  cplx<T>* P0 = (cplx<T>*)w.P;
  const cplx<T>* Qk = (const cplx<T>*)w.Q + (size_t)(k % w.win) * w.blk;
#define MARK(i) \
  if (ev) HIP_TRY(c, hipEventRecord(ev[i], c->stream))
  MARK(0);
  HIP_TRY(c, launch_hop<T>(c, 1, w.n, P0, w.W1, nullptr, 0.0, 1.0, skip));
  MARK(1);
  HIP_TRY(c, launch_hop<T>(c, 0, w.n, w.W1, w.W, P0, mass * mass + sp.sigma[0], -1.0, skip));
  MARK(2);
  HIP_TRY(c, launch_gram4<T>(c->stream, w.rows, w.n, P0, Qk, w.W, w.sm.G4, w.partials, w.nb,
                             skip, c->gram_variant, c->num_cu));
  MARK(3);
  HIP_TRY(c, launch_small_iter<T>(c->stream, sp, w.sm, w.flags, (cplx<T>*)w.Mx,
                                  (cplx<T>*)w.Mp, (cplx<T>*)w.Wm));
  MARK(4);
  // explicit Cholesky-QR Gram, only when the expansion lost its pivot
  HIP_TRY(c, launch_cholqr_gram<T>(c->stream, w.rows, w.n, Qk, w.W, w.sm.alpha, w.sm.Gqr,
                                   w.partials, w.nb, &w.flags->need_explicit));
  MARK(5);
  HIP_TRY(c, launch_small_rho_explicit<T>(c->stream, sp, w.sm, w.flags, (cplx<T>*)w.Mp,
                                          (cplx<T>*)w.Wm));
  MARK(6);
  const UpdateArgs<T, T> ua = update_args<T>(w);
  // built-in default: the matrix-core kernel where it exists (n = 8, 16), else
  // four row chunks with one coefficient column at a time
  const int uv = c->update_variant;
  if (update_mfma_supported(w.n) && (uv < 0 || uv >= 4))
    HIP_TRY(c, launch_update_mfma<T>(c->stream, ua, uv == 5));
  else
    HIP_TRY(c, (launch_update_fast<T, T>(c->stream, ua, uv < 0 || uv >= 4 ? 2 : uv)));
  MARK(7);
#undef MARK
  return BMS_OK;
}

// Q_0 delta_0 = B by Cholesky-QR applied twice; P^(s) = Q_0, X^(s) = 0.
template <typename T>
int enqueue_setup(bms_ctx* c, const Work& w, const SmallParams& sp, const void* B) {
  size_t es = sizeof(cplx<T>);
  // the small-step arrival counter must start at zero (it is left at zero after use)
  HIP_TRY(c, launch_fill_zero(c->stream, w.sm.counter, 16));
  HIP_TRY(c, launch_fill_zero(c->stream, w.X, w.blk * es * w.ns));
  HIP_TRY(c, launch_gram<double>(c->stream, w.rows, w.n, B, B, w.sm.G4, w.partials, w.nb,
                                 nullptr));
  HIP_TRY(c, launch_small_init(c->stream, sp, w.sm, w.flags, w.sm.G4, w.Rinv));
  HIP_TRY(c, launch_block_matmul_d<T>(c->stream, w.rows, w.n, B, w.Rinv, w.W, nullptr));
  HIP_TRY(c, launch_gram<T>(c->stream, w.rows, w.n, w.W, w.W, w.sm.G4, w.partials, w.nb,
                            nullptr));
  HIP_TRY(c, launch_small_init_pass2(c->stream, sp, w.sm, w.flags, w.sm.G4, w.Rinv));
  HIP_TRY(c, launch_block_matmul<T>(c->stream, w.rows, w.n, w.W, w.Rinv, w.Q));
  for (int s = 0; s < w.ns; ++s)
    HIP_TRY(c, hipMemcpyAsync((char*)w.P + s * w.blk * es, w.Q, w.blk * es,
                              hipMemcpyDeviceToDevice, c->stream));
  return BMS_OK;
}

// MIXED: FP32 increments into the FP64 solutions, then the unshifted true
// residual replaces the iterated one.
// (Called between chunks of iterations, where Q_k is in ring buffer 0.)
int enqueue_reliable(bms_ctx* c, const Work& w, const SmallParams& sp, double mass, const void* B,
                     void* Xout, const int* xmap, void* R1, void* R2, void* R0, bool flush_only) {
  const int* skip = &w.flags->stop;
  HIP_TRY(c, launch_flush(c->stream, w.rows, w.n, w.ns, w.X, Xout, xmap,
                          flush_only ? nullptr : skip));
  if (flush_only) return BMS_OK;
  const double2* X0 = (const double2*)Xout + (size_t)xmap[0] * w.blk;
  HIP_TRY(c, launch_hop<double>(c, 1, w.n, X0, R1, nullptr, 0.0, 1.0, skip));
  HIP_TRY(c, launch_hop<double>(c, 0, w.n, R1, R2, X0, mass * mass + sp.sigma[0], -1.0, skip));
  HIP_TRY(c, launch_resid_block(c->stream, w.rows, w.n, B, R2, nullptr, nullptr, R0, skip));
  HIP_TRY(c, launch_gram<double>(c->stream, w.rows, w.n, R0, R0, w.Gtmp, w.partials, w.nb,
                                 skip));
  HIP_TRY(c, launch_small_reliable(c->stream, sp, w.sm, w.flags, w.Gtmp, w.Rinv));
  HIP_TRY(c, launch_block_matmul_d<float>(c->stream, w.rows, w.n, R0, w.Rinv, w.Q,
                                          &w.flags->rel_skip));
  // one shift and a large jump: the search direction restarts from the new Q
  HIP_TRY(c, launch_copy_if(c->stream, w.P, w.Q, w.blk * sizeof(float2), &w.flags->rel_restart));
  return BMS_OK;
}

struct CoreResult {
  int iters = 0;
  int error = 0;  // final failure (initial QR)
  int soft = 0;   // the iteration stopped early on breakdown / non-finite values
  int reliable = 0;
  bool diverged = false;  // the mixed iteration's true residual grew (stopped softly)
  bool exhausted = false; // FP32 loop stopped at twice the block Krylov dimension
  bool extended = false;  // the FP64 phase went on to the final tolerance
};

// Everything the kernels of one iteration receive by value or address: a
// captured chunk of iterations can be replayed while this is unchanged.
template <typename T>
std::string chunk_key(const bms_ctx* c, const Work& w, const SmallParams& sp, double mass, int K) {
  struct {
    const void* p[16];
    double mass;
    int K, n, ns, nb, hop_v, gram_v, upd_v, prec, nlinks;
    HopCfg hop_cfg[2];
    SmallParams sp;
    SmallState sm;
  } k;
  memset(&k, 0, sizeof k);
  const bool two = c->links_two_rows && c->nlinks == 8;
  const void* ptrs[16] = {w.W1, w.W, w.Q, w.P, w.X, w.Mx, w.Mp, w.flags, w.partials, w.sm.counter,
                          two ? c->links64r.p : c->links64.p, two ? c->links32r.p : c->links32.p,
                          w.Wm, w.sm.wst, two ? c->lsign.p : nullptr, nullptr};
  for (int i = 0; i < 16; ++i) k.p[i] = ptrs[i];
  k.mass = mass;
  k.K = K;
  k.n = w.n;
  k.ns = w.ns;
  k.nb = w.nb;
  k.hop_v = c->hop_variant;
  k.gram_v = c->gram_variant;
  k.upd_v = c->update_variant;
  k.prec = (int)sizeof(T);
  k.nlinks = c->nlinks;
  k.hop_cfg[0] = c->hop_cfg[0];
  k.hop_cfg[1] = c->hop_cfg[1];
  k.sp = sp;
  k.sm = w.sm;
  return std::string((const char*)&k, sizeof k);
}

// Enqueue K iterations: replayed from a captured hipGraph when allowed (the
// chunk holds kernel launches only), else launched directly (always while
// per-kernel timing is on, with events between the kernels).
template <typename T>
int enqueue_chunk(bms_ctx* c, const Work& w, const SmallParams& sp, double mass, int K,
                  bool use_graph) {
  if (!use_graph || c->timing) {
    for (int k = 0; k < K; ++k) {
      // chunks start at multiples of K, which win divides: k % win is the
      // iteration's ring position
      int rc = enqueue_iteration<T>(c, w, sp, mass, k, c->timing ? &c->evpool[8 * k] : nullptr);
      if (rc) return rc;
    }
    return BMS_OK;
  }
  std::string key = chunk_key<T>(c, w, sp, mass, K);
  if (!c->graph_exec || c->graph_key != key) {
    if (c->graph_exec) {
      HIP_TRY(c, hipStreamSynchronize(c->stream));  // an earlier replay may still run
      HIP_TRY(c, hipGraphExecDestroy(c->graph_exec));
      c->graph_exec = nullptr;
    }
    c->graph_key.clear();
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = BMS_OK;
    for (int k = 0; k < K && rc == BMS_OK; ++k)
      rc = enqueue_iteration<T>(c, w, sp, mass, k, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return set_err(c, BMS_EHIP, "stream capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph_exec = nullptr;
      return set_err(c, BMS_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    c->graph_key = key;
  }
  HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
  return BMS_OK;
}

// One block multi-shift solve from X = 0. sigma[] ascending; the solution of
// sigma[s] is written to Xout + xmap[s] * blk (FP64), which must not alias B.
template <typename T>
int solve_core(bms_ctx* c, double mass, int n, int ns, const double* sigma, const int* xmap,
               double tol, int max_iter, const bms_opts& o, const void* B, void* Xout,
               CoreResult& cr, double extend_tol = 0.0) {
  int rc;
  const bool mixed = sizeof(T) == 4;
  SmallParams sp;
  memset(&sp, 0, sizeof sp);
  sp.n = n;
  sp.ns = ns;
  sp.max_iter = max_iter;
  // In exact arithmetic block CG ends within ceil(rows / n) iterations (the
  // block Krylov space is then the whole space). An FP32 loop still running
  // at twice that has lost the recurrence to rounding and creeps along (seen
  // on 8^4 with n = 16 at m = 0.01: 42 000 FP32 iterations against 538 in
  // FP64), so it stops there and the caller finishes in FP64 (the FP32-only
  // solve through its full FP64 restart, the two-phase solve by redoing the
  // correction solve in FP64).
  const long kdim = (3L * c->vh + n - 1) / n;
  if (mixed && 2 * kdim < max_iter) sp.max_iter = (int)(2 * kdim);
  // The recurrence's residual estimate drifts from the true residual by
  // rounding; stopping (and freezing) at tol/2 leaves that margin.
  sp.tol = 0.5 * tol;
  double ft = o.freeze_tol > 0 ? o.freeze_tol : sp.tol;
  sp.freeze_tol = ft < sp.tol ? ft : sp.tol;
  // a computed Gram resolves pivots only down to ~eps * trace, eps of the
  // block vectors' precision (FP32 blocks in the mixed solver)
  sp.breakdown_tol = 10.0 * n * (mixed ? kEps32 : kEps);
  for (int s = 0; s < ns; ++s) sp.sigma[s] = sigma[s];
  sp.win = update_window(c, n, ns, (int)sizeof(T), o.check_interval);
  Work w;
  if ((rc = alloc_work<T>(c, n, ns, max_iter, sp.win, w))) return rc;
  void *R1 = nullptr, *R2 = nullptr, *R0 = nullptr;
  if (mixed) {
    size_t b64 = w.blk * sizeof(double2);
    if ((rc = scratch_buf(c, S_R1, b64, &R1))) return rc;
    if ((rc = scratch_buf(c, S_R2, b64, &R2))) return rc;
    if ((rc = scratch_buf(c, S_R0, b64, &R0))) return rc;
    for (int s = 0; s < ns; ++s)
      HIP_TRY(c, launch_fill_zero(c->stream, (double2*)Xout + (size_t)xmap[s] * w.blk,
                                  w.blk * sizeof(double2)));
  }
  if ((rc = enqueue_setup<T>(c, w, sp, B))) return rc;
  SolverFlags hf;
  const int K = o.check_interval;
  long enqueued = 0, last_rel = 0;
  if (c->timing && (int)c->evpool.size() < 8 * K) {
    size_t old = c->evpool.size();
    c->evpool.resize(8 * K);
    for (size_t i = old; i < c->evpool.size(); ++i) HIP_TRY(c, hipEventCreate(&c->evpool[i]));
  }
  while (true) {
    if ((rc = enqueue_chunk<T>(c, w, sp, mass, K, o.use_graph != 0))) return rc;
    if (mixed && enqueued + K - last_rel >= o.reliable_interval) {
      if ((rc = enqueue_reliable(c, w, sp, mass, B, Xout, xmap, R1, R2, R0, false))) return rc;
      last_rel = enqueued + K;
    }
    HIP_TRY(c, hipMemcpyAsync(&hf, w.flags, sizeof hf, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->timing) {
      // links read by one half hop: nine entries, or six for two-row links
      const int epl = c->links_two_rows && c->nlinks == 8 ? 6 : 9;
      double G = (double)epl * c->nlinks * c->vol * sizeof(T);
      double S = (double)w.blk * sizeof(cplx<T>);
      // the explicit Cholesky-QR Gram (slot 4) normally exits at once: no bytes
      const double kbytes[7] = {G + 2 * S, G + 3 * S, 3 * S, 0, 0, 0, 0};
      for (int k = 0; k < K; ++k) {
        if (enqueued + k >= hf.iter) break;  // launches after the stop did no work
        for (int i = 0; i < 7; ++i) {
          float ms = 0;
          HIP_TRY(c, hipEventElapsedTime(&ms, c->evpool[8 * k + i], c->evpool[8 * k + i + 1]));
          int kc = kIterKernel[i];
          c->kt_ms[kc] += ms;
          c->kt_launches[kc] += 1;
          c->kt_bytes[kc] += kbytes[i];
        }
      }
    }
    enqueued += K;
    if (hf.stop) break;
    // extend_tol > 0 (the FP64 phase of the mixed solver): once the block
    // Krylov space is half spanned the residual block sits in the few modes
    // left, its columns nearly dependent, and the last iterations converge
    // fast; an FP32 phase started from it would have to rebuild that space
    // (and its Cholesky-QR loses rank), so this solve goes on to extend_tol.
    if (extend_tol > 0 && !cr.extended && 2L * hf.iter >= kdim) {
      sp.tol = 0.5 * extend_tol;
      sp.freeze_tol = std::min(sp.freeze_tol, sp.tol);
      cr.extended = true;
    }
    if (enqueued > (long)max_iter + 2L * K)  // the device stops itself at max_iter
      return set_err(c, BMS_EHIP, "device iteration control did not stop (iter %d)", hf.iter);
  }
  // increments the two-iteration update still holds back
  // windows the solve ended with still open
  if (w.win > 1) HIP_TRY(c, launch_update_drain<T>(c->stream, update_args<T>(w)));
  if (c->timing && hf.iter > 0) {
    std::vector<int> units(hf.iter);
    HIP_TRY(c, hipMemcpyAsync(units.data(), w.sm.upd_log, hf.iter * sizeof(int),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double S = (double)w.blk * sizeof(cplx<T>);
    // matrix-core flops of one complex right product of a row block by an
    // n x n matrix: three real products (rows n^2 FMA each) for n = 16, one
    // real product by the 2n x 2n form (rows (2n)^2 FMA) for n = 8
    const double prod = n == 16 ? 6.0 * w.rows * n * n : 2.0 * w.rows * (2.0 * n) * (2.0 * n);
    const bool mf = update_mfma_supported(n) && (c->update_variant < 0 || c->update_variant >= 4);
    for (int k = 0; k < hf.iter; ++k) {
      const double b = (units[k] & 0xffff) * S;
      c->kt_bytes[BMS_KERNEL_UPDATE] += b;
      double f64 = 0, f32 = 0;
      if (mf) {
        f64 = 2 * prod;  // the Q step, FP64
        (mixed ? f32 : f64) += (units[k] >> 16) * prod;
      }
      c->kt_flops64[BMS_KERNEL_UPDATE] += f64;
      c->kt_flops32[BMS_KERNEL_UPDATE] += f32;
      c->kt_upd_launch.push_back(b);
      c->kt_upd_launch.push_back(f64);
      c->kt_upd_launch.push_back(f32);
    }
  }
  if (mixed) {
    if ((rc = enqueue_reliable(c, w, sp, mass, B, Xout, xmap, R1, R2, R0, true))) return rc;
  } else {
    size_t bytes = w.blk * sizeof(double2);
    for (int s = 0; s < ns; ++s)
      HIP_TRY(c, hipMemcpyAsync((char*)Xout + (size_t)xmap[s] * bytes,
                                (char*)w.X + (size_t)s * bytes, bytes, hipMemcpyDeviceToDevice,
                                c->stream));
  }
  cr.iters = hf.iter;
  cr.reliable = hf.rel_count;
  cr.diverged = hf.diverged != 0;
  bool all_conv = true;
  for (int s = 0; s < ns; ++s) all_conv = all_conv && hf.conv[s];
  if (sp.max_iter < max_iter && hf.iter >= sp.max_iter && !all_conv) {
    cr.exhausted = true;
    cr.diverged = true;  // no usable FP32 result: the caller goes on in FP64
  }
  (mixed ? c->it_f32 : c->it_f64) += hf.iter;
  c->hop_work += 2L * hf.iter + 2L * hf.rel_count;
  // A breakdown or non-finite value inside the iteration stops it with the
  // last finite iterate in X (the update of that step is skipped); the true
  // residual check and defect correction then decide. Only a failure of the
  // initial QR (linearly dependent columns of B) is final.
  if (hf.error && hf.iter == 0) cr.error = hf.error;
  else if (hf.error) cr.soft = hf.error;
  return BMS_OK;
}

}  // namespace

// Size every workspace slot that a solve of n columns, ns shifts and max_iter
// iterations can touch, in any phase and precision (FP64 blocks are the
// larger), and the event pool of per-kernel timing. Called serially for each
// context before bms_solve_batch starts its threads, so that no solve grows a
// buffer (hipFree, hipMalloc, hipMemset) while another captures a graph.
static int validate_solve(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                          double tol, int max_iter, const bms_opts* o, const void* B,
                          const void* X);

int solve_reserve(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                  int max_iter, const bms_opts* opts, const void* B, const void* X) {
  // a call that bms_solve rejects on the host reserves nothing (and reports
  // its error from bms_solve)
  if (validate_solve(c, mass, n, ns, shifts, tol, max_iter, opts, B, X) != BMS_OK) {
    c->last_error.clear();
    return BMS_OK;
  }
  bms_opts o;
  bms_default_opts(&o);
  if (opts) o = *opts;
  const int check_interval = o.check_interval;
  int rc;
  if ((rc = ensure_device(c))) return rc;
  const size_t rows = (size_t)3 * c->vh, blk = rows * n, nn = (size_t)n * n, e = sizeof(double2);
  void* p;
  const struct {
    int slot;
    size_t bytes;
  } need[] = {
      {S_W1, blk * e},
      {S_W, blk * e},
      {S_Q, blk * std::max(e * update_window(c, n, ns, 8, check_interval),
                           sizeof(float2) * update_window(c, n, ns, 4, check_interval))},
      {S_P, blk * e * ns},
      {S_X, blk * e * ns},
      {S_SMALL, small_elems(n, ns) * e + 64},
      {S_PART, std::max(part_bytes(gram_blocks((int)rows, n, c->num_cu), 4 * (int)nn),
                        part_bytes(gram_blocks((int)rows, 1, c->num_cu), 4))},
      {S_M, (2 + 2 * BMS_MAX_WIN) * ns * nn * e},
      {S_FLAGS, kFlagsBytes},
      {S_LOG, (size_t)max_iter * sizeof(int) + 64},
      {S_R1, blk * e},
      {S_R2, blk * e},
      {S_R0, blk * e},
      {S_RES, std::max({(size_t)ns * n * e, 2 * nn * e, (size_t)(n + BMS_MAX_SHIFTS) * e}) + 64},
      {S_RB, blk * e},
      {S_E, blk * e},
      {S_COLS, 3 * n * sizeof(double) + 64},
      {S_RBC, rows * e},
      {S_EC, rows * e},
      {S_E2, (size_t)ns * blk * e},
      {S_CMAT, nn * e + 64},
  };
  for (const auto& q : need)
    if ((rc = scratch_buf(c, q.slot, q.bytes, &p))) return rc;
  if (c->timing && (int)c->evpool.size() < 8 * check_interval) {
    size_t old = c->evpool.size();
    c->evpool.resize(8 * check_interval);
    for (size_t i = old; i < c->evpool.size(); ++i) HIP_TRY(c, hipEventCreate(&c->evpool[i]));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return BMS_OK;
}

// Per shift s and column i of user-ordered solutions: rn2[s][i] = |b_i - (A+s)x_i|^2
// and bn2[i] = |b_i|^2.
static int residual_norms(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                          const void* B, const void* X, std::vector<double>& rn2,
                          std::vector<double>& bn2) {
  int rc;
  int rows = 3 * c->vh;
  size_t blk = (size_t)rows * n;
  void *t1, *t2, *out;
  if ((rc = scratch_buf(c, S_R1, blk * sizeof(double2), &t1))) return rc;
  if ((rc = scratch_buf(c, S_R2, blk * sizeof(double2), &t2))) return rc;
  if ((rc = scratch_buf(c, S_RES, (size_t)ns * n * sizeof(double2) + 64, &out))) return rc;
  int nb = gram_blocks(rows, n, c->num_cu);
  void* pp;
  if ((rc = scratch_buf(c, S_PART, part_bytes(nb, 4 * n * n), &pp))) return rc;
  for (int s = 0; s < ns; ++s) {
    const double2* xs = (const double2*)X + s * blk;
    HIP_TRY(c, launch_hop<double>(c, 1, n, xs, t1, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<double>(c, 0, n, t1, t2, xs, mass * mass + shifts[s], -1.0, nullptr));
    HIP_TRY(c, launch_resid_norms(c->stream, rows, n, B, t2, (double2*)out + (size_t)s * n,
                                  (double2*)pp, nb));
  }
  c->hop_work += 2L * ns;
  std::vector<double2> h((size_t)ns * n);
  HIP_TRY(c, hipMemcpyAsync(h.data(), out, h.size() * sizeof(double2), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  rn2.resize((size_t)ns * n);
  bn2.resize(n);
  for (size_t i = 0; i < h.size(); ++i) rn2[i] = h[i].x;
  for (int i = 0; i < n; ++i) bn2[i] = h[i].y;
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
  if (max_iter < 1 || max_iter > 10000000)
    return set_err(c, BMS_EINVAL, "max_iter must be in [1, 1e7]");
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
    if (!(o->mixed_switch == o->mixed_switch))
      return set_err(c, BMS_EINVAL, "opts.mixed_switch must be a number");
    if (o->max_refine < 0) return set_err(c, BMS_EINVAL, "opts.max_refine must be >= 0");
  }
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  return BMS_OK;
}

int solve_validate(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                   int max_iter, const bms_opts* o, const void* B, const void* X) {
  return validate_solve(c, mass, n, ns, shifts, tol, max_iter, o, B, X);
}

// x = G^-1 b for Hermitian positive definite G (n x n, row-major) and n
// right-hand sides b (columns of the n x n matrix B): Cholesky on the host.
// Fails (false) when a pivot falls below 1e-12 of G's largest diagonal entry.
static bool host_hpd_solve(int n, std::vector<double2>& G, std::vector<double2>& Bm) {
  std::vector<double2> L((size_t)n * n, make_double2(0, 0));
  double gmax = 0;
  for (int j = 0; j < n; ++j) gmax = std::max(gmax, G[j * n + j].x);
  auto mul = [](double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); };
  auto cjm = [](double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); };
  for (int j = 0; j < n; ++j) {
    double d = G[j * n + j].x;
    for (int k = 0; k < j; ++k) d -= L[j * n + k].x * L[j * n + k].x + L[j * n + k].y * L[j * n + k].y;
    if (!(d > 1e-12 * gmax)) return false;
    d = std::sqrt(d);
    L[j * n + j] = make_double2(d, 0);
    for (int i = j + 1; i < n; ++i) {
      double2 v = G[i * n + j];
      for (int k = 0; k < j; ++k) {
        double2 t = cjm(L[j * n + k], L[i * n + k]);  // L_ik conj(L_jk)
        v.x -= t.x;
        v.y -= t.y;
      }
      L[i * n + j] = make_double2(v.x / d, v.y / d);
    }
  }
  for (int c = 0; c < n; ++c) {  // L L^H x = b, column c
    std::vector<double2> y(n);
    for (int i = 0; i < n; ++i) {
      double2 v = Bm[i * n + c];
      for (int k = 0; k < i; ++k) {
        double2 t = mul(L[i * n + k], y[k]);
        v.x -= t.x;
        v.y -= t.y;
      }
      y[i] = make_double2(v.x / L[i * n + i].x, v.y / L[i * n + i].x);
    }
    for (int i = n - 1; i >= 0; --i) {
      double2 v = y[i];
      for (int k = i + 1; k < n; ++k) {
        double2 t = cjm(L[k * n + i], Bm[k * n + c]);  // conj(L_ki) x_k
        v.x -= t.x;
        v.y -= t.y;
      }
      Bm[i * n + c] = make_double2(v.x / L[i * n + i].x, v.y / L[i * n + i].x);
    }
  }
  return true;
}

// The FP32 phase of the mixed solver. After the FP64 block multi-shift phase
// has brought the smallest shift to the switch residual, every shift that is
// still updated shares its residual block up to a right factor: R_s = R_0 C_s
// (R_s = Q delta^(s) with one Q for all shifts). One FP32 block multi-shift
// solve of (A + sigma_s) E_s = R' for the column-normalised R' = R_0 D^-1 then
// corrects all of them: X_s += E_s C'_s with C'_s = (R'^H R')^-1 R'^H R_s, the
// least-squares right factor (exact up to the FP64 phase's rounding). Shifts
// already converged are left to the per-shift defect correction. In FP32 a
// shifted solution drifts from its recurrence by about eps_32 times its
// condition number times the residual it starts from, which is why the FP64
// phase runs first: started from the switch residual, that drift stays near
// the target. Returns BMS_OK without changing X when it does not apply.
static int mixed_phase2(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                        const int* order, double tol, int max_iter, const bms_opts& o,
                        const void* B, void* X, int& iters, int& reliable) {
  int rc;
  std::vector<double> rn2, bn2;
  if ((rc = residual_norms(c, mass, n, ns, shifts, B, X, rn2, bn2))) return rc;
  auto worst = [&](int s) {
    double m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, std::sqrt(rn2[s * n + i] / bn2[i]));
    return m;
  };
  const int s0 = order[0];
  if (!(worst(s0) > tol) || !(worst(s0) < 1.0)) return BMS_OK;
  // the shifts still updated by the FP64 phase (their residuals are well above
  // tol; frozen ones sit near tol and go to the defect correction)
  std::vector<int> act;
  double wmax = 0;
  for (int k = 0; k < ns; ++k) {
    int s = order[k];
    if (k == 0 || worst(s) > 10.0 * tol) {
      act.push_back(s);
      wmax = std::max(wmax, worst(s));
    }
  }
  const int na = (int)act.size();
  int rows = 3 * c->vh;
  size_t blk = (size_t)rows * n;
  void *RB, *E, *E2, *cols, *t1, *t2, *res, *pp, *cm;
  if ((rc = scratch_buf(c, S_RB, blk * sizeof(double2), &RB))) return rc;
  if ((rc = scratch_buf(c, S_E, blk * sizeof(double2), &E))) return rc;
  if ((rc = scratch_buf(c, S_COLS, 3 * n * sizeof(double) + 64, &cols))) return rc;
  if ((rc = scratch_buf(c, S_R1, blk * sizeof(double2), &t1))) return rc;
  if ((rc = scratch_buf(c, S_R2, blk * sizeof(double2), &t2))) return rc;
  if ((rc = scratch_buf(c, S_RES, (size_t)2 * n * n * sizeof(double2) + 64, &res))) return rc;
  if ((rc = scratch_buf(c, S_CMAT, (size_t)n * n * sizeof(double2) + 64, &cm))) return rc;
  int nb = gram_blocks(rows, n, c->num_cu);
  if ((rc = scratch_buf(c, S_PART, part_bytes(nb, 4 * n * n), &pp))) return rc;
  // R' = (B - (A + s0) X_0) D^-1, D = diag |r_i| (B's column where r_i = 0)
  std::vector<double> h(3 * n);
  for (int i = 0; i < n; ++i) {
    double rn = std::sqrt(rn2[s0 * n + i]), bn = std::sqrt(bn2[i]);
    h[i] = rn > 0 ? 1.0 / rn : 0.0;
    h[n + i] = bn > 0 ? 1.0 / bn : 1.0;
    h[2 * n + i] = rn;
  }
  HIP_TRY(c, hipMemcpyAsync(cols, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  auto apply_a = [&](int s) -> int {
    const double2* xs = (const double2*)X + (size_t)s * blk;
    HIP_TRY(c, launch_hop<double>(c, 1, n, xs, t1, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<double>(c, 0, n, t1, t2, xs, mass * mass + shifts[s], -1.0, nullptr));
    c->hop_work += 2;
    return BMS_OK;
  };
  if ((rc = apply_a(s0))) return rc;
  HIP_TRY(c, launch_resid_block(c->stream, rows, n, B, t2, (const double*)cols,
                                (const double*)cols + n, RB, nullptr));
  // C'_s from the Grams R'^H R' and R'^H R_s
  std::vector<double2> G00((size_t)n * n), G0s((size_t)n * n);
  HIP_TRY(c, launch_gram<double>(c->stream, rows, n, RB, RB, (double2*)res, (double2*)pp, nb,
                                 nullptr));
  HIP_TRY(c, hipMemcpyAsync(G00.data(), res, G00.size() * sizeof(double2), hipMemcpyDeviceToHost,
                            c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<std::vector<double2>> C(na);
  for (int a = 0; a < na; ++a) {
    const int s = act[a];
    if ((rc = apply_a(s))) return rc;
    HIP_TRY(c, launch_resid_block(c->stream, rows, n, B, t2, nullptr, nullptr, E, nullptr));
    HIP_TRY(c, launch_gram<double>(c->stream, rows, n, RB, E, (double2*)res, (double2*)pp, nb,
                                   nullptr));
    HIP_TRY(c, hipMemcpyAsync(G0s.data(), res, G0s.size() * sizeof(double2),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    std::vector<double2> G = G00;
    if (!host_hpd_solve(n, G, G0s)) return BMS_OK;  // R' rank-deficient: leave it to refinement
    C[a] = G0s;
  }
  // one FP32 multi-shift solve on R' for all of them (ascending shifts)
  std::vector<double> sig(na);
  std::vector<int> xm(na);
  for (int a = 0; a < na; ++a) {
    sig[a] = shifts[act[a]];
    xm[a] = a;
  }
  if ((rc = scratch_buf(c, S_E2, (size_t)na * blk * sizeof(double2), &E2))) return rc;
  double t2tol = std::min(0.5, std::max(0.5 * tol / wmax, 1e-13));
  bms_opts o2 = o;
  o2.freeze_tol = 0.0;
  CoreResult cr;
  if ((rc = solve_core<float>(c, mass, n, na, sig.data(), xm.data(), t2tol, max_iter, o2, RB, E2,
                              cr)))
    return rc;
  iters += cr.iters;
  reliable += cr.reliable;
  if (cr.exhausted) {
    // the FP32 recurrence ran out of Krylov space (small lattices, where the
    // block spans it within a few hundred iterations): the same correction
    // solve in FP64, which keeps what the FP64 phase reached
    if ((rc = solve_core<double>(c, mass, n, na, sig.data(), xm.data(), t2tol, max_iter, o2, RB,
                                 E2, cr)))
      return rc;
    iters += cr.iters;
    reliable += cr.reliable;
  }
  // a failed, diverged or softly stopped (breakdown, non-finite values) FP32
  // phase gives no usable correction: X stays as the FP64 phase left it
  if (cr.error || cr.diverged || cr.soft) return BMS_OK;
  std::vector<double> ones(n, 1.0);
  HIP_TRY(c, hipMemcpyAsync(cols, ones.data(), n * sizeof(double), hipMemcpyHostToDevice,
                            c->stream));
  for (int a = 0; a < na; ++a) {
    HIP_TRY(c, hipMemcpyAsync(cm, C[a].data(), (size_t)n * n * sizeof(double2),
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, launch_block_matmul_d<double>(c->stream, rows, n, (const double2*)E2 + a * blk,
                                             (const double2*)cm, E, nullptr));
    HIP_TRY(c, launch_axpy_cols(c->stream, rows, n, (double2*)X + (size_t)act[a] * blk, E,
                                (const double*)cols));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return BMS_OK;
}

template <typename T>
static int solve_precision(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                           double tol, int max_iter, const bms_opts& o, const void* B, void* X,
                           bms_stats* st) {
  int rc;
  std::vector<int> order(ns);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return shifts[a] < shifts[b]; });
  std::vector<double> sig(ns);
  for (int s = 0; s < ns; ++s) sig[s] = shifts[order[s]];
  CoreResult cr;
  int refine_iters = 0, reliable = 0;
  c->it_f64 = c->it_f32 = c->hop_work = c->rel_work = 0;
  // MIXED: an FP64 block multi-shift phase down to the switch residual (every
  // shift kept updated until the final tolerance), then the FP32 phase
  const bool two_phase = sizeof(T) == 4 && o.mixed_switch > tol && o.mixed_switch < 1.0;
  int first_iters = 0;
  if (two_phase) {
    bms_opts o1 = o;
    o1.freeze_tol = o.freeze_tol > 0 ? std::min(o.freeze_tol, 0.5 * tol) : 0.5 * tol;
    if ((rc = solve_core<double>(c, mass, n, ns, sig.data(), order.data(), o.mixed_switch,
                                 max_iter, o1, B, X, cr, tol)))
      return rc;
    first_iters = cr.iters;
    if (!cr.error && !cr.extended &&
        (rc = mixed_phase2(c, mass, n, ns, shifts, order.data(), tol, max_iter, o, B, X,
                           refine_iters, reliable)))
      return rc;
  } else {
    if ((rc = solve_core<T>(c, mass, n, ns, sig.data(), order.data(), tol, max_iter, o, B, X, cr)))
      return rc;
    first_iters = cr.iters;
  }
  reliable += cr.reliable;
  bool fell_back = false;
  if (sizeof(T) == 4 && cr.diverged) {
    // the FP32 iteration diverged or stalled: solve all shifts again in FP64
    // (one multi-shift solve is cheaper than refining every shift on its own)
    refine_iters += cr.iters;
    CoreResult c64;
    if ((rc = solve_core<double>(c, mass, n, ns, sig.data(), order.data(), tol, max_iter, o, B, X,
                                 c64)))
      return rc;
    cr = c64;
    cr.reliable = reliable;
    fell_back = true;
  }
  std::vector<double> rn2, bn2;
  if ((rc = residual_norms(c, mass, n, ns, shifts, B, X, rn2, bn2))) return rc;
  // defect correction of the shifts that miss tol. In the mixed solver the
  // corrections run in FP32 unless a shift's FP32 correction diverged or did
  // not gain a factor 10, then in FP64; a shift whose residual is worse than
  // that of X = 0 (a diverged main iteration) restarts from X = 0.
  const bool mixed = sizeof(T) == 4;
  std::vector<char> use64(ns, fell_back || cr.extended ? 1 : 0);
  int rows = 3 * c->vh;
  size_t blk = (size_t)rows * n;
  for (int round = 0; round < o.max_refine && !cr.error; ++round) {
    std::vector<int> bad;
    std::vector<double> before(ns, 0.0);
    for (int s = 0; s < ns; ++s) {
      double m = 0;
      for (int i = 0; i < n; ++i) m = std::max(m, std::sqrt(rn2[s * n + i] / bn2[i]));
      before[s] = m;
      if (!(m <= tol)) bad.push_back(s);
    }
    if (bad.empty()) break;
    void *RB, *E, *cols, *t1, *t2;
    if ((rc = scratch_buf(c, S_RB, blk * sizeof(double2), &RB))) return rc;
    if ((rc = scratch_buf(c, S_E, blk * sizeof(double2), &E))) return rc;
    if ((rc = scratch_buf(c, S_COLS, 3 * n * sizeof(double) + 64, &cols))) return rc;
    if ((rc = scratch_buf(c, S_R1, blk * sizeof(double2), &t1))) return rc;
    if ((rc = scratch_buf(c, S_R2, blk * sizeof(double2), &t2))) return rc;
    for (int s : bad) {
      if (!(before[s] <= 1.0)) {
        // worse than no solution at all (or not finite): start again from 0
        HIP_TRY(c, launch_fill_zero(c->stream, (double2*)X + s * blk, blk * sizeof(double2)));
        for (int i = 0; i < n; ++i) rn2[s * n + i] = bn2[i];
      }
      // column-normalised residual R'_i = r_i / |r_i| (B's column if r_i = 0)
      std::vector<double> h(3 * n);
      double worst = 0;
      for (int i = 0; i < n; ++i) {
        double rn = std::sqrt(rn2[s * n + i]), bn = std::sqrt(bn2[i]);
        h[i] = rn > 0 ? 1.0 / rn : 0.0;
        h[n + i] = bn > 0 ? 1.0 / bn : 1.0;
        h[2 * n + i] = rn;
        worst = std::max(worst, rn / bn);
      }
      const double2* xs = (const double2*)X + s * blk;
      HIP_TRY(c, hipMemcpyAsync(cols, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice,
                                c->stream));
      HIP_TRY(c, launch_hop<double>(c, 1, n, xs, t1, nullptr, 0.0, 1.0, nullptr));
      HIP_TRY(c, launch_hop<double>(c, 0, n, t1, t2, xs, mass * mass + shifts[s], -1.0, nullptr));
      c->hop_work += 2;
      HIP_TRY(c, launch_resid_block(c->stream, rows, n, B, t2, (const double*)cols,
                                    (const double*)cols + n, RB, nullptr));
      double tin = 0.5 * tol / worst;
      tin = std::min(0.5, std::max(tin, 1e-13));
      CoreResult ci;
      int zero = 0;
      double sg = shifts[s];
      const bool in64 = !mixed || use64[s];
      if (in64)
        rc = solve_core<double>(c, mass, n, 1, &sg, &zero, tin, max_iter, o, RB, E, ci);
      else
        rc = solve_core<T>(c, mass, n, 1, &sg, &zero, tin, max_iter, o, RB, E, ci);
      if (rc) return rc;
      refine_iters += ci.iters;
      reliable += ci.reliable;
      if (ci.diverged) {
        use64[s] = 1;  // E is not a usable correction; FP64 next round
        continue;
      }
      if (ci.error == BMS_EBREAKDOWN) {
        // the normalised residual columns are nearly dependent (typically a
        // few lowest modes left): refine them one column at a time
        void *bc, *ec;
        if ((rc = scratch_buf(c, S_RBC, (size_t)rows * sizeof(double2), &bc))) return rc;
        if ((rc = scratch_buf(c, S_EC, (size_t)rows * sizeof(double2), &ec))) return rc;
        for (int i = 0; i < n; ++i) {
          if (!(h[2 * n + i] > 0.5 * tol * std::sqrt(bn2[i]))) continue;
          double ti = std::min(0.5, std::max(0.5 * tol * std::sqrt(bn2[i]) / h[2 * n + i], 1e-13));
          HIP_TRY(c, launch_gather_col(c->stream, rows, n, i, RB, bc));
          CoreResult cc;
          if (in64)
            rc = solve_core<double>(c, mass, 1, 1, &sg, &zero, ti, max_iter, o, bc, ec, cc);
          else
            rc = solve_core<T>(c, mass, 1, 1, &sg, &zero, ti, max_iter, o, bc, ec, cc);
          if (rc) return rc;
          refine_iters += cc.iters;
          reliable += cc.reliable;
          if (cc.diverged) {
            use64[s] = 1;
            continue;
          }
          if (cc.error) {
            cr.error = cc.error;
            break;
          }
          HIP_TRY(c, launch_scatter_axpy_col(c->stream, rows, n, i, (double2*)X + s * blk, ec,
                                             h[2 * n + i]));
        }
        if (cr.error) break;
        continue;
      }
      if (ci.error) {
        cr.error = ci.error;
        break;
      }
      HIP_TRY(c, launch_axpy_cols(c->stream, rows, n, (double2*)X + s * blk, E,
                                  (const double*)cols + 2 * n));
    }
    if ((rc = residual_norms(c, mass, n, ns, shifts, B, X, rn2, bn2))) return rc;
    if (mixed)
      for (int s : bad) {
        double m = 0;
        for (int i = 0; i < n; ++i) m = std::max(m, std::sqrt(rn2[s * n + i] / bn2[i]));
        if (!(m <= 0.1 * before[s]) && !(m <= tol)) use64[s] = 1;
      }
  }
  double mx = 0;
  std::vector<double> res((size_t)ns * n);
  for (int s = 0; s < ns; ++s)
    for (int i = 0; i < n; ++i) {
      double r = bn2[i] > 0 ? std::sqrt(rn2[s * n + i] / bn2[i]) : std::sqrt(rn2[s * n + i]);
      res[s * n + i] = r;
      mx = std::max(mx, std::isfinite(r) ? r : 1e300);
    }
  if (st) {
    const long total = c->it_f64 + c->it_f32;
    st->iterations = (int)total;
    st->multishift_iterations = first_iters;
    st->refine_iterations = (int)(total - first_iters);
    st->iterations_f64 = (int)c->it_f64;
    st->iterations_f32 = (int)c->it_f32;
    st->hop_calls = (int)c->hop_work;
    st->reliable_updates = reliable;
    st->converged = mx <= tol;
    st->max_true_residual = mx;
    if (st->true_residual) memcpy(st->true_residual, res.data(), res.size() * sizeof(double));
  }
  if (cr.error)
    return set_err(c, cr.error, "device reported %s in the initial QR", bms_error_string(cr.error));
  if (!(mx < 1e300))
    return set_err(c, BMS_ENAN, "non-finite true residual after %d iterations", cr.iters);
  if (mx > tol)
    return set_err(c, BMS_ENOCONV, "max true residual %.3e > tol %.3e after %d iterations", mx,
                   tol, cr.iters);
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
    rc = solve_precision<double>(c, mass, n, ns, shifts, tol, max_iter, o, B, X, st);
  else
    rc = solve_precision<float>(c, mass, n, ns, shifts, tol, max_iter, o, B, X, st);
  int rc2 = stream_end(c);
  return rc ? rc : rc2;
}

extern "C" int bms_rational_apply(bms_ctx* c, double mass, int n, int ns, double a0,
                                  const double* alpha, const double* shifts, double tol,
                                  int max_iter, const bms_opts* opts, const void* B, void* X,
                                  void* out, bms_stats* st) {
  if (!c) return BMS_EINVAL;
  int rc = validate_solve(c, mass, n, ns, shifts, tol, max_iter, opts, B, X);
  if (rc) return rc;
  if (!alpha || !out) return set_err(c, BMS_EINVAL, "null alpha or out");
  if (out == X) return set_err(c, BMS_EINVAL, "out and X must not alias");
  if (!std::isfinite(a0)) return set_err(c, BMS_EINVAL, "a0 not finite");
  for (int s = 0; s < ns; ++s)
    if (!std::isfinite(alpha[s])) return set_err(c, BMS_EINVAL, "alpha[%d] not finite", s);
  rc = bms_solve(c, mass, n, ns, shifts, tol, max_iter, opts, B, X, st);
  if (rc != BMS_OK) return rc;
  if ((rc = stream_begin(c))) return rc;
  HIP_TRY(c, launch_rational_combine(c->stream, (size_t)3 * c->vh * n, ns, a0, alpha, B, X, out));
  return stream_end(c);
}

extern "C" int bms_action(bms_ctx* c, int n, int ns, double a0, const double* alpha,
                          const void* B, const void* X, double* S) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 0 || ns > BMS_MAX_SHIFTS) return set_err(c, BMS_EINVAL, "bad n_shifts");
  if ((ns > 0 && (!alpha || !X)) || !B || !S) return set_err(c, BMS_EINVAL, "null pointer");
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  int rc;
  if ((rc = stream_begin(c))) return rc;
  int rows = 3 * c->vh;
  void *al, *out, *pp;
  if ((rc = scratch_buf(c, S_RES, (size_t)(n + BMS_MAX_SHIFTS) * sizeof(double2) + 64, &out)))
    return rc;
  al = (double2*)out + n;
  int nb = gram_blocks(rows, n, c->num_cu);
  if ((rc = scratch_buf(c, S_PART, part_bytes(nb, 4 * n * n), &pp))) return rc;
  if (ns > 0)
    HIP_TRY(c, hipMemcpyAsync(al, alpha, ns * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, launch_action(c->stream, rows, n, ns, a0, (const double*)al, B, X, (double2*)out,
                           (double2*)pp, nb));
  std::vector<double2> h(n);
  HIP_TRY(c, hipMemcpyAsync(h.data(), out, n * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) S[i] = h[i].x;
  return stream_end(c);
}
