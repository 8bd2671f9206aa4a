// Drivers above bms_solve: kernel-variant autotuning on the caller's problem
// and a batch of independent solves (one context and stream each) run
// concurrently on one GPU.
#include <stdio.h>
#include <string.h>

#include <string>

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

namespace {

// Events around `reps` pairs of half hops (D_oe then D_eo with the aux
// epilogue) on the workspace blocks, in the current hop variant and
// configuration: microseconds per pair.
template <typename T>
int time_hop_pair(bms_ctx* c, int n, void* e_in, void* o_mid, void* e_out, int reps, double* us) {
  hipEvent_t ev[2];
  HIP_TRY(c, hipEventCreate(&ev[0]));
  HIP_TRY(c, hipEventCreate(&ev[1]));
  HIP_TRY(c, launch_hop<T>(c, 1, n, e_in, o_mid, nullptr, 0.0, 1.0, nullptr));  // warm-up
  HIP_TRY(c, launch_hop<T>(c, 0, n, o_mid, e_out, e_in, 0.5, -1.0, nullptr));
  HIP_TRY(c, hipEventRecord(ev[0], c->stream));
  for (int r = 0; r < reps; ++r) {
    HIP_TRY(c, launch_hop<T>(c, 1, n, e_in, o_mid, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<T>(c, 0, n, o_mid, e_out, e_in, 0.5, -1.0, nullptr));
  }
  HIP_TRY(c, hipEventRecord(ev[1], c->stream));
  HIP_TRY(c, hipEventSynchronize(ev[1]));
  float ms = 0;
  HIP_TRY(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  *us = 1e3 * ms / reps;
  return BMS_OK;
}

// Search of the hop's traversal for one precision: natural order and several
// tile shapes, each with 0..4 resident work-groups per compute unit and with
// and without non-temporal link loads, plus the per-group kernel. Keeps the
// fastest (variant and configuration); returns its time per hop pair.
int tune_hop(bms_ctx* c, int n, bool fp64, double* best_us) {
  const size_t blk = (size_t)3 * c->vh * n;
  void *e_in, *o_mid, *e_out;
  int rc;
  if ((rc = scratch_buf(c, S_R2, blk * sizeof(double2), &e_in))) return rc;
  if ((rc = scratch_buf(c, S_R1, blk * sizeof(double2), &o_mid))) return rc;
  if ((rc = scratch_buf(c, S_R0, blk * sizeof(double2), &e_out))) return rc;
  const int tiles[][3] = {{0, 0, 0},  {8, 8, 4},  {8, 8, 8}, {16, 8, 4}, {8, 16, 4},
                          {4, 8, 8},  {16, 16, 2}, {4, 4, 8}, {8, 4, 8},  {16, 8, 2}};
  const int slot = fp64 ? 0 : 1;
  const HopCfg keep = c->hop_cfg[slot];
  const int keep_v = c->hop_variant;
  HopCfg best = keep;
  int best_v = keep_v;
  double bus = 1e300;
  const int reps = 3;
  for (int v : {-1, 0}) {
    c->hop_variant = v;
    for (const auto& t : tiles) {
      if (t[0] > 0 && !hop_tiling_valid(c, n, t[0], t[1], t[2])) continue;
      for (int cap = 0; cap <= 4; ++cap)
        for (int nt = 0; nt <= 1; ++nt) {
          if (cap > 0 && hop_cap_lds(c, cap) == 0) continue;  // cap not applicable here
          HopCfg h;
          h.ty = t[0];
          h.tz = t[0] > 0 ? t[1] : 8;
          h.tt = t[0] > 0 ? t[2] : 4;
          h.cap = cap;
          h.nt = nt;
          c->hop_cfg[slot] = h;
          double us = 0;
          rc = fp64 ? time_hop_pair<double>(c, n, e_in, o_mid, e_out, reps, &us)
                    : time_hop_pair<float>(c, n, e_in, o_mid, e_out, reps, &us);
          if (rc) {
            c->hop_cfg[slot] = keep;
            c->hop_variant = keep_v;
            return rc;
          }
          if (us < bus) {
            bus = us;
            best = h;
            best_v = v;
          }
        }
    }
  }
  c->hop_cfg[slot] = best;
  c->hop_variant = best_v;
  *best_us = bus;
  return BMS_OK;
}

std::string tune_key(bms_ctx* c, int n, int ns, int precision) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    size_t colon = arch.find(':');
    if (colon != std::string::npos) arch.resize(colon);
  }
  // links per site and rows read per link: the hop's traffic, and so its
  // best traversal, depend on them
  const int rows = c->links_two_rows && c->nlinks == 8 ? 2 : 3;
  char buf[256];
  snprintf(buf, sizeof buf, "%s|%d,%d,%d,%d|%d|%d|%d|L%dr%d", arch.c_str(), c->dims[0], c->dims[1],
           c->dims[2], c->dims[3], n, ns, precision, c->nlinks, rows);
  return buf;
}

// The last cache line with this key, applied to the context; false if none.
bool cache_lookup(bms_ctx* c, const std::string& key) {
  FILE* f = fopen(c->tune_cache.c_str(), "r");
  if (!f) return false;
  char line[1024];
  const std::string want = "{\"key\": \"" + key + "\",";
  bool found = false;
  int hv = -1, gv = -1, uv = -1, h64[5], h32[5];
  while (fgets(line, sizeof line, f)) {
    if (strncmp(line, want.c_str(), want.size()) != 0) continue;
    int a, b, d, e[5], g[5];
    if (sscanf(line + want.size(),
               " \"hop\": %d, \"gram\": %d, \"update\": %d, \"hop_f64\": [%d, %d, %d, %d, %d], "
               "\"hop_f32\": [%d, %d, %d, %d, %d]",
               &a, &b, &d, &e[0], &e[1], &e[2], &e[3], &e[4], &g[0], &g[1], &g[2], &g[3],
               &g[4]) == 13) {
      found = true;
      hv = a;
      gv = b;
      uv = d;
      memcpy(h64, e, sizeof h64);
      memcpy(h32, g, sizeof h32);
    }
  }
  fclose(f);
  if (!found) return false;
  c->hop_variant = hv;
  c->gram_variant = gv;
  c->update_variant = uv;
  bms_set_hop_config(c, BMS_PREC_F64, h64);
  bms_set_hop_config(c, BMS_PREC_F32, h32);
  return true;
}

void cache_append(bms_ctx* c, const std::string& key, const double* us) {
  FILE* f = fopen(c->tune_cache.c_str(), "a");
  if (!f) return;
  const HopCfg& a = c->hop_cfg[0];
  const HopCfg& b = c->hop_cfg[1];
  fprintf(f,
          "{\"key\": \"%s\", \"hop\": %d, \"gram\": %d, \"update\": %d, \"hop_f64\": [%d, %d, %d, "
          "%d, %d], \"hop_f32\": [%d, %d, %d, %d, %d], \"hop_pair_us\": [%.1f, %.1f]}\n",
          key.c_str(), c->hop_variant, c->gram_variant, c->update_variant, a.ty, a.tz, a.tt, a.cap,
          a.nt, b.ty, b.tz, b.tt, b.cap, b.nt, us[0], us[1]);
  fclose(f);
}

}  // namespace

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
  int rc = solve_validate(c, mass, n, ns, shifts, 0.5, iters, &o, B, X);
  if (rc) return rc;
  if ((rc = ensure_device(c))) return rc;
  const std::string key = tune_key(c, n, ns, precision);
  if (!c->tune_cache.empty() && cache_lookup(c, key)) return BMS_OK;
  // 1. the hop's kernel and traversal, per precision the solve uses
  double hop_us[2] = {0, 0};
  if ((rc = stream_begin(c))) return rc;
  if ((rc = tune_hop(c, n, true, &hop_us[0]))) return rc;
  if (precision == BMS_PREC_MIXED && (rc = tune_hop(c, n, false, &hop_us[1]))) return rc;
  // 2. the Gram and update kernels, timed inside real block iterations
  const bool timing_was = c->timing;
  const int kinds[2] = {BMS_KERNEL_GRAM, BMS_KERNEL_UPDATE};
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
      rc = bms_solve(c, mass, n, ns, shifts, 1e-300, iters, &o, B, X, &st);
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
  if (!c->tune_cache.empty()) cache_append(c, key, hop_us);
  return stream_end(c);
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
