// Drivers above bms_solve: kernel-variant autotuning on the caller's problem
// and a batch of independent solves (one context and stream each) run
// concurrently on one GPU.
#include <string.h>

#include <thread>
#include <vector>

#include "internal.h"

namespace {

int* variant_slot(bms_ctx* c, int kernel) {
  switch (kernel) {
    case BMS_KERNEL_HOP: return &c->hop_variant;
    case BMS_KERNEL_GRAM: return &c->gram_variant;
    case BMS_KERNEL_UPDATE: return &c->update_variant;
    case BMS_KERNEL_FORCE: return &c->force_variant;
    default: return nullptr;
  }
}

// candidate variants of a kernel class for block width n (all accepted by
// bms_set_variant; ones that do not apply fall back to a default kernel and
// simply time like it)
std::vector<int> candidates(int kernel, int n) {
  const bool quad = n == 4 || n == 8 || n == 16 || n == 32;
  const bool mf = n == 8 || n == 16;
  switch (kernel) {
    // -1 (the built-in default) picks per precision, which one fixed variant
    // cannot do for the mixed solver's FP64 and FP32 phases
    case BMS_KERNEL_HOP: return quad ? std::vector<int>{-1, 1, 3, 0, 2} : std::vector<int>{-1, 0, 2};
    case BMS_KERNEL_GRAM: return mf ? std::vector<int>{2, 1, 3} : std::vector<int>{0};
    case BMS_KERNEL_UPDATE: return mf ? std::vector<int>{4, 6, 5, 2, 0} : std::vector<int>{2};
    default: return {};
  }
}

}  // namespace

extern "C" int bms_get_variant(const bms_ctx* c, int kernel, int* variant) {
  if (!c || !variant) return BMS_EINVAL;
  int* v = variant_slot(const_cast<bms_ctx*>(c), kernel);
  if (!v) return BMS_EINVAL;
  *variant = *v;
  return BMS_OK;
}

extern "C" int bms_autotune(bms_ctx* c, double mass, int n, int ns, const double* shifts,
                            int precision, int iters, const void* B, void* X) {
  if (!c) return BMS_EINVAL;
  if (precision != BMS_PREC_F64 && precision != BMS_PREC_MIXED)
    return set_err(c, BMS_EINVAL, "precision must be BMS_PREC_F64 or BMS_PREC_MIXED");
  if (iters < 1 || iters > 4096) return set_err(c, BMS_EINVAL, "iters must be in [1, 4096]");
  bms_opts o;
  bms_default_opts(&o);
  o.precision = precision;
  o.max_refine = 0;
  o.reliable_interval = 1 << 30;  // time the iteration kernels only
  const bool timing_was = c->timing;
  const int kinds[3] = {BMS_KERNEL_HOP, BMS_KERNEL_GRAM, BMS_KERNEL_UPDATE};
  for (int kind : kinds) {
    int* slot = variant_slot(c, kind);
    std::vector<int> cand = candidates(kind, n);
    int best = *slot;
    double best_us = 1e300;
    for (int v : cand) {
      *slot = v;
      bms_timing_enable(c, 1);
      bms_stats st;
      memset(&st, 0, sizeof st);
      // a target far below reach: exactly `iters` iterations are run
      int rc = bms_solve(c, mass, n, ns, shifts, 1e-300, iters, &o, B, X, &st);
      if (rc != BMS_OK && rc != BMS_ENOCONV && rc != BMS_EBREAKDOWN && rc != BMS_ENAN) {
        bms_timing_enable(c, timing_was);
        c->timing = timing_was;
        return rc;
      }
      if (c->kt_launches[kind] > 0) {
        double us = 1e3 * c->kt_ms[kind] / (double)c->kt_launches[kind];
        if (us < best_us) {
          best_us = us;
          best = v;
        }
      }
    }
    *slot = best;
  }
  bms_timing_enable(c, timing_was);
  c->timing = timing_was;
  return BMS_OK;
}

extern "C" int bms_solve_batch(int nprob, bms_ctx* const* ctxs, const double* mass, const int* n,
                               const int* n_shifts, const double* const* shifts, const double* tol,
                               const int* max_iter, const bms_opts* opts, const void* const* B,
                               void* const* X, bms_stats* stats, int* status) {
  if (nprob < 1 || nprob > 64 || !ctxs || !mass || !n || !n_shifts || !shifts || !tol ||
      !max_iter || !B || !X || !status)
    return BMS_EINVAL;
  for (int i = 0; i < nprob; ++i) {
    if (!ctxs[i]) return BMS_EINVAL;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return BMS_EINVAL;  // a context serves one solve at a time
  }
  // All workspace first, one context after another: a solve that grew a
  // buffer inside a thread would free and allocate device memory while a
  // sibling thread captures its iteration chunk into a hipGraph.
  for (int i = 0; i < nprob; ++i) {
    int rc = solve_reserve(ctxs[i], mass[i], n[i], n_shifts[i], shifts[i], tol[i], max_iter[i],
                           opts ? &opts[i] : nullptr, B[i], X[i]);
    if (rc) {
      for (int j = 0; j < nprob; ++j) status[j] = j == i ? rc : BMS_OK;
      return rc;
    }
  }
  std::vector<std::thread> th;
  th.reserve(nprob);
  for (int i = 0; i < nprob; ++i)
    th.emplace_back([=]() {
      status[i] = bms_solve(ctxs[i], mass[i], n[i], n_shifts[i], shifts[i], tol[i], max_iter[i],
                            opts ? &opts[i] : nullptr, B[i], X[i], stats ? &stats[i] : nullptr);
    });
  for (auto& t : th) t.join();
  for (int i = 0; i < nprob; ++i)
    if (status[i] != BMS_OK) return status[i];
  return BMS_OK;
}
