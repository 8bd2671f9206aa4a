// C-ABI entry points: context lifecycle, validation, gauge import, operator.
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "internal.h"

int set_err(bms_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->last_error = buf;
  }
  return code;
}

extern "C" void bms_default_opts(bms_opts* o) {
  if (!o) return;
  o->precision = BMS_PREC_F64;
  o->reliable_interval = 50;
  o->freeze_tol = 0.0;
  o->check_interval = 8;
  o->max_refine = 4;
  o->qr_passes = 1;
  o->use_graph = 1;
  o->mixed_switch = 3e-4;
}

extern "C" const char* bms_error_string(int s) {
  switch (s) {
    case BMS_OK: return "BMS_OK";
    case BMS_EINVAL: return "BMS_EINVAL: invalid argument";
    case BMS_ENOMEM: return "BMS_ENOMEM: device allocation failed";
    case BMS_EHIP: return "BMS_EHIP: HIP runtime error";
    case BMS_EBREAKDOWN: return "BMS_EBREAKDOWN: block lost rank (Cholesky pivot not positive)";
    case BMS_ENOCONV: return "BMS_ENOCONV: not converged within max_iter";
    case BMS_ENAN: return "BMS_ENAN: non-finite value";
    case BMS_ESTATE: return "BMS_ESTATE: call out of order";
    default: return "unknown bms status";
  }
}

extern "C" const char* bms_last_error(const bms_ctx* c) { return c ? c->last_error.c_str() : ""; }

extern "C" int bms_create(bms_ctx** out, const int dims[4], const int bc[4], void* stream) {
  if (!out || !dims || !bc) return BMS_EINVAL;
  *out = nullptr;
  long vol = 1;
  for (int i = 0; i < 4; ++i) {
    if (dims[i] < 2 || (dims[i] & 1) || dims[i] > 4096) return BMS_EINVAL;
    if (bc[i] != 1 && bc[i] != -1) return BMS_EINVAL;
    vol *= dims[i];
    if (vol > (1L << 25)) return BMS_EINVAL;
  }
  bms_ctx* c = new (std::nothrow) bms_ctx();
  if (!c) return BMS_ENOMEM;
  for (int i = 0; i < 4; ++i) {
    c->dims[i] = dims[i];
    c->bc[i] = bc[i];
  }
  c->vol = vol;
  c->vh = (int)(vol / 2);
  Geom& g = c->geom;
  for (int i = 0; i < 4; ++i) g.L[i] = dims[i];
  g.hx = dims[0] / 2;
  g.stride[0] = 1;
  g.stride[1] = g.hx;
  g.stride[2] = g.hx * dims[1];
  g.stride[3] = g.hx * dims[1] * dims[2];
  g.vh = c->vh;
  g.d_hx = make_fastdiv(g.hx);
  g.d_ly = make_fastdiv(dims[1]);
  g.d_lz = make_fastdiv(dims[2]);
  c->nblk = (c->vh + (1 << c->sbl) - 1) >> c->sbl;
  c->user_stream = (hipStream_t)stream;
  *out = c;
  return BMS_OK;
}

int ensure_device(bms_ctx* c) {
  if (c->stream) return BMS_OK;
  HIP_TRY(c, hipGetDevice(&c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor,
                                   c->device));
  HIP_TRY(c, hipDeviceGetAttribute(&c->lds_per_block, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                   c->device));
  HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  HIP_TRY(c, hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
  HIP_TRY(c, hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
  return BMS_OK;
}

// order the library stream after the caller's stream
int stream_begin(bms_ctx* c) {
  int rc = ensure_device(c);
  if (rc) return rc;
  HIP_TRY(c, hipEventRecord(c->ev_in, c->user_stream));
  HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_in, 0));
  return BMS_OK;
}

// order the caller's stream after the library stream
int stream_end(bms_ctx* c) {
  HIP_TRY(c, hipEventRecord(c->ev_out, c->stream));
  HIP_TRY(c, hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
  return BMS_OK;
}

int ensure_buf(bms_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes) return BMS_OK;
  if (b.p) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    HIP_TRY(c, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
  }
  HIP_TRY(c, hipMalloc(&b.p, bytes));
  b.bytes = bytes;
  // fresh device memory may hold stale data; counters and flags rely on zero
  HIP_TRY(c, hipMemsetAsync(b.p, 0, bytes, c->stream));
  return BMS_OK;
}

int scratch_buf(bms_ctx* c, int slot, size_t bytes, void** p) {
  if ((int)c->scratch.size() <= slot) c->scratch.resize(slot + 1);
  int rc = ensure_buf(c, c->scratch[slot], bytes < 256 ? 256 : bytes);
  if (rc) return rc;
  *p = c->scratch[slot].p;
  return BMS_OK;
}

extern "C" int bms_destroy(bms_ctx* c) {
  if (!c) return BMS_EINVAL;
  // teardown: a failing release cannot be reported past this point
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->links64.p) (void)hipFree(c->links64.p);
  if (c->links32.p) (void)hipFree(c->links32.p);
  for (DevBuf* b : {&c->links64r, &c->links32r, &c->lsign, &c->lcheck})
    if (b->p) (void)hipFree(b->p);
  for (auto& b : c->scratch)
    if (b.p) (void)hipFree(b.p);
  for (auto e : c->evpool) (void)hipEventDestroy(e);
  if (c->ev_in) (void)hipEventDestroy(c->ev_in);
  if (c->ev_out) (void)hipEventDestroy(c->ev_out);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return BMS_OK;
}

extern "C" int bms_set_gauge(bms_ctx* c, const void* U) {
  if (!c) return BMS_EINVAL;
  if (!U) return set_err(c, BMS_EINVAL, "bms_set_gauge: U is NULL");
  int rc = stream_begin(c);
  if (rc) return rc;
  size_t nlink = (size_t)2 * c->nblk * 72 << c->sbl;
  if ((rc = ensure_buf(c, c->links64, nlink * sizeof(double2)))) return rc;
  if ((rc = ensure_buf(c, c->links32, nlink * sizeof(float2)))) return rc;
  // padding sites of the last block are never read; zero them once
  HIP_TRY(c, launch_fill_zero(c->stream, c->links64.p, nlink * sizeof(double2)));
  HIP_TRY(c, launch_fill_zero(c->stream, c->links32.p, nlink * sizeof(float2)));
  const bool two = c->link_rows == 2;
  if (two) {
    const size_t nrow = (size_t)2 * c->nblk * 48 << c->sbl;
    if ((rc = ensure_buf(c, c->links64r, nrow * sizeof(double2)))) return rc;
    if ((rc = ensure_buf(c, c->links32r, nrow * sizeof(float2)))) return rc;
    if ((rc = ensure_buf(c, c->lsign, (size_t)2 * c->vh * sizeof(uint32_t)))) return rc;
    if ((rc = ensure_buf(c, c->lcheck, 256))) return rc;
    HIP_TRY(c, launch_fill_zero(c->stream, c->links64r.p, nrow * sizeof(double2)));
    HIP_TRY(c, launch_fill_zero(c->stream, c->links32r.p, nrow * sizeof(float2)));
    HIP_TRY(c, launch_fill_zero(c->stream, c->lcheck.p, 16));
  }
  HIP_TRY(c, launch_gauge_import(c, U, c->links64.p, c->links32.p, two ? c->links64r.p : nullptr,
                                 two ? c->links32r.p : nullptr, two ? c->lsign.p : nullptr,
                                 two ? c->lcheck.p : nullptr));
  c->links_two_rows = false;
  c->link_dev = -1;
  if (two) {
    // the hop reads two rows only if every third row is the SU(3) one to 1e-12
    unsigned long long bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, c->lcheck.p, sizeof bits, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    double dev;
    memcpy(&dev, &bits, sizeof dev);
    c->link_dev = dev;
    c->links_two_rows = dev <= 1e-12;
  }
  c->nlinks = 8;
  c->gauge_set = true;
  return stream_end(c);
}

extern "C" int bms_set_link_rows(bms_ctx* c, int rows) {
  if (!c) return BMS_EINVAL;
  if (rows != 2 && rows != 3) return set_err(c, BMS_EINVAL, "link rows must be 2 or 3");
  c->link_rows = rows;
  return BMS_OK;
}

extern "C" int bms_get_link_rows(const bms_ctx* c, int* rows, double* max_dev) {
  if (!c || !rows) return BMS_EINVAL;
  *rows = c->links_two_rows && c->nlinks == 8 ? 2 : 3;
  if (max_dev) *max_dev = c->nlinks == 8 ? c->link_dev : -1;
  return BMS_OK;
}

extern "C" int bms_set_gauge_improved(bms_ctx* c, const void* V, const void* W) {
  if (!c) return BMS_EINVAL;
  if (!V || !W) return set_err(c, BMS_EINVAL, "bms_set_gauge_improved: V or W is NULL");
  for (int i = 0; i < 4; ++i)
    if (c->dims[i] < 4)
      return set_err(c, BMS_EINVAL, "the improved operator needs every extent >= 4");
  int rc = stream_begin(c);
  if (rc) return rc;
  size_t nlink = (size_t)2 * c->nblk * 144 << c->sbl;
  if ((rc = ensure_buf(c, c->links64, nlink * sizeof(double2)))) return rc;
  if ((rc = ensure_buf(c, c->links32, nlink * sizeof(float2)))) return rc;
  HIP_TRY(c, launch_fill_zero(c->stream, c->links64.p, nlink * sizeof(double2)));
  HIP_TRY(c, launch_fill_zero(c->stream, c->links32.p, nlink * sizeof(float2)));
  HIP_TRY(c, launch_gauge_import_improved(c, V, W, c->links64.p, c->links32.p));
  c->links_two_rows = false;
  c->link_dev = -1;
  c->nlinks = 16;
  c->gauge_set = true;
  return stream_end(c);
}

static int check_prec_op(bms_ctx* c, int prec) {
  if (prec != BMS_PREC_F64 && prec != BMS_PREC_F32)
    return set_err(c, BMS_EINVAL, "operator precision must be BMS_PREC_F64 or BMS_PREC_F32");
  return BMS_OK;
}

extern "C" int bms_apply_hop(bms_ctx* c, int parity_out, int n, const void* in, void* out,
                             int prec) {
  if (!c) return BMS_EINVAL;
  if (parity_out != 0 && parity_out != 1) return set_err(c, BMS_EINVAL, "parity_out must be 0 or 1");
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (!in || !out) return set_err(c, BMS_EINVAL, "null vector pointer");
  if (in == out) return set_err(c, BMS_EINVAL, "in and out must not alias");
  int rc = check_prec_op(c, prec);
  if (rc) return rc;
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  if ((rc = stream_begin(c))) return rc;
  if (prec == BMS_PREC_F64)
    HIP_TRY(c, launch_hop<double>(c, parity_out, n, in, out, nullptr, 0.0, 1.0, nullptr));
  else
    HIP_TRY(c, launch_hop<float>(c, parity_out, n, in, out, nullptr, 0.0, 1.0, nullptr));
  return stream_end(c);
}

extern "C" int bms_apply_mdagm(bms_ctx* c, double mass, double sigma, int n, const void* in,
                               void* out, int prec) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (!in || !out) return set_err(c, BMS_EINVAL, "null vector pointer");
  if (in == out) return set_err(c, BMS_EINVAL, "in and out must not alias");
  if (!(mass == mass) || !(sigma == sigma)) return set_err(c, BMS_EINVAL, "mass/sigma is NaN");
  int rc = check_prec_op(c, prec);
  if (rc) return rc;
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  if ((rc = stream_begin(c))) return rc;
  size_t es = prec == BMS_PREC_F64 ? sizeof(double2) : sizeof(float2);
  void* tmp;
  if ((rc = scratch_buf(c, 0, (size_t)c->vh * 3 * n * es, &tmp))) return rc;
  double d = mass * mass + sigma;
  if (prec == BMS_PREC_F64) {
    HIP_TRY(c, launch_hop<double>(c, 1, n, in, tmp, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<double>(c, 0, n, tmp, out, in, d, -1.0, nullptr));
  } else {
    HIP_TRY(c, launch_hop<float>(c, 1, n, in, tmp, nullptr, 0.0, 1.0, nullptr));
    HIP_TRY(c, launch_hop<float>(c, 0, n, tmp, out, in, d, -1.0, nullptr));
  }
  return stream_end(c);
}

extern "C" int bms_timing_enable(bms_ctx* c, int enable) {
  if (!c) return BMS_EINVAL;
  c->timing = enable != 0;
  for (int k = 0; k < BMS_NKERNELS; ++k) {
    c->kt_ms[k] = 0;
    c->kt_launches[k] = 0;
    c->kt_bytes[k] = 0;
    c->kt_flops64[k] = c->kt_flops32[k] = 0;
  }
  c->kt_upd_launch.clear();
  return BMS_OK;
}

extern "C" int bms_timing_read(const bms_ctx* c, int kernel, double* ms, long long* launches,
                               double* bytes) {
  if (!c || kernel < 0 || kernel >= BMS_NKERNELS) return BMS_EINVAL;
  if (ms) *ms = c->kt_ms[kernel];
  if (launches) *launches = c->kt_launches[kernel];
  if (bytes) *bytes = c->kt_bytes[kernel];
  return BMS_OK;
}

extern "C" int bms_timing_flops(const bms_ctx* c, int kernel, double* flops_f64,
                                double* flops_f32) {
  if (!c || kernel < 0 || kernel >= BMS_NKERNELS) return BMS_EINVAL;
  if (flops_f64) *flops_f64 = c->kt_flops64[kernel];
  if (flops_f32) *flops_f32 = c->kt_flops32[kernel];
  return BMS_OK;
}

extern "C" int bms_timing_floor(const bms_ctx* c, int kernel, double hbm_bytes_per_s,
                                double f64_flops_per_s, double f32_flops_per_s,
                                double* seconds) {
  if (!c || kernel < 0 || kernel >= BMS_NKERNELS || !seconds || !(hbm_bytes_per_s > 0) ||
      !(f64_flops_per_s > 0) || !(f32_flops_per_s > 0))
    return BMS_EINVAL;
  double t = 0;
  if (kernel == BMS_KERNEL_UPDATE && !c->kt_upd_launch.empty()) {
    const std::vector<double>& L = c->kt_upd_launch;
    for (size_t i = 0; i + 2 < L.size(); i += 3)
      t += std::max(L[i] / hbm_bytes_per_s, L[i + 1] / f64_flops_per_s + L[i + 2] / f32_flops_per_s);
  } else {
    t = c->kt_bytes[kernel] / hbm_bytes_per_s;
  }
  *seconds = t;
  return BMS_OK;
}

extern "C" int bms_set_variant(bms_ctx* c, int kernel, int variant) {
  if (!c) return BMS_EINVAL;
  if (kernel == BMS_KERNEL_HOP) {
    if (variant < -1 || variant > 4) return set_err(c, BMS_EINVAL, "hop variant must be in [-1, 4]");
    c->hop_variant = variant;
    return BMS_OK;
  }
  if (kernel == BMS_KERNEL_GRAM) {
    if (variant < -1 || variant > 5) return set_err(c, BMS_EINVAL, "gram variant must be in [-1, 5]");
    c->gram_variant = variant;
    return BMS_OK;
  }
  if (kernel == BMS_KERNEL_FORCE) {
    if (variant < -1 || variant > 2) return set_err(c, BMS_EINVAL, "force variant must be in [-1, 2]");
    c->force_variant = variant;
    return BMS_OK;
  }
  if (kernel != BMS_KERNEL_UPDATE) return set_err(c, BMS_EINVAL, "no variants for kernel %d", kernel);
  if (variant < -1 || variant > 6) return set_err(c, BMS_EINVAL, "variant must be in [-1, 6]");
  c->update_variant = variant;
  return BMS_OK;
}

extern "C" int bms_set_hop_config(bms_ctx* c, int precision, const int cfg[5]) {
  if (!c) return BMS_EINVAL;
  if (precision != BMS_PREC_F64 && precision != BMS_PREC_F32)
    return set_err(c, BMS_EINVAL, "precision must be BMS_PREC_F64 or BMS_PREC_F32");
  HopCfg h;
  if (cfg && cfg[0] >= 0) {
    const int ty = cfg[0], tz = cfg[1], tt = cfg[2], cap = cfg[3], nt = cfg[4];
    if (ty > 0 && (tz < 1 || tt < 1 || ty > 4096 || tz > 4096 || tt > 4096))
      return set_err(c, BMS_EINVAL, "tile extents must be >= 1");
    if (cap < -1 || cap > 64) return set_err(c, BMS_EINVAL, "cap must be in [-1, 64]");
    if (nt != 0 && nt != 1) return set_err(c, BMS_EINVAL, "nt must be 0 or 1");
    h.ty = ty;
    h.tz = ty > 0 ? tz : 8;
    h.tt = ty > 0 ? tt : 4;
    h.cap = cap;
    h.nt = nt;
  }
  c->hop_cfg[precision == BMS_PREC_F64 ? 0 : 1] = h;
  return BMS_OK;
}

extern "C" int bms_get_hop_config(const bms_ctx* c, int precision, int cfg[5]) {
  if (!c || !cfg) return BMS_EINVAL;
  if (precision != BMS_PREC_F64 && precision != BMS_PREC_F32) return BMS_EINVAL;
  const HopCfg& h = c->hop_cfg[precision == BMS_PREC_F64 ? 0 : 1];
  cfg[0] = h.ty;
  cfg[1] = h.tz;
  cfg[2] = h.tt;
  cfg[3] = h.cap;
  cfg[4] = h.nt;
  return BMS_OK;
}

extern "C" int bms_set_tune_cache(bms_ctx* c, const char* path) {
  if (!c) return BMS_EINVAL;
  c->tune_cache = path ? path : "";
  return BMS_OK;
}
