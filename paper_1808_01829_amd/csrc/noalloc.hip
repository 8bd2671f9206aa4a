// bms_action_noalloc: the pseudofermion action of bms_action for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc). Its scratch (the residues, the
// per-block partial sums of the grid reduction and the n sums) lives in a
// file-scope device array instead of the context's workspace.
//
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is ever passed to kernels or copies.
// Every call on a device shares that device's array, so calls that overlap
// on one GPU (several streams or host threads) race; nothing in it needs to
// start at zero, since every call writes each entry it reads.
#include <mutex>

#include "blas.h"

namespace {

constexpr size_t kScratchBytes = 1u << 20;  // 1 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};
int g_num_cu[kMaxDevices] = {0};

// Device address of this device's scratch array (taken on first use of the
// device, with it current) and its compute-unit count.
int scratch_for_current_device(bms_ctx* c, unsigned char** p, int* num_cu) {
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return set_err(c, BMS_EINVAL, "bms_action_noalloc: device %d beyond the supported %d", dev,
                   kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    int cu = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
    g_ptr[dev] = ptr;
    g_num_cu[dev] = cu;
  }
  *p = (unsigned char*)g_ptr[dev];
  *num_cu = g_num_cu[dev];
  return BMS_OK;
}

}  // namespace

extern "C" int bms_action_noalloc(bms_ctx* c, int n, int ns, double a0, const double* alpha,
                                  const void* B, const void* X, double* S) {
  if (!c) return BMS_EINVAL;
  if (n < 1 || n > BMS_MAX_RHS) return set_err(c, BMS_EINVAL, "n must be in [1, %d]", BMS_MAX_RHS);
  if (ns < 0 || ns > BMS_MAX_SHIFTS) return set_err(c, BMS_EINVAL, "bad n_shifts");
  if ((ns > 0 && (!alpha || !X)) || !B || !S) return set_err(c, BMS_EINVAL, "null pointer");
  if (!c->gauge_set) return set_err(c, BMS_ESTATE, "no gauge field set");
  unsigned char* base;
  int num_cu;
  int rc = scratch_for_current_device(c, &base, &num_cu);
  if (rc) return rc;
  const int rows = 3 * c->vh;
  // the same reduction shape as bms_action (same blocks, same summation order)
  const int nb = gram_blocks(rows, n, num_cu);
  // layout: n sums | BMS_MAX_SHIFTS residues | nb x n partial sums
  const size_t off_alpha = 256 * ((n * sizeof(double2) + 255) / 256);
  const size_t off_part = off_alpha + 256 * ((BMS_MAX_SHIFTS * sizeof(double) + 255) / 256);
  const size_t need = off_part + (size_t)nb * n * sizeof(double2);
  if (need > kScratchBytes)
    return set_err(c, BMS_EINVAL,
                   "bms_action_noalloc: %zu bytes of scratch needed, the static maximum is %zu",
                   need, kScratchBytes);
  double2* out = (double2*)base;
  double* al = (double*)(base + off_alpha);
  double2* part = (double2*)(base + off_part);
  // the caller's stream, nothing created or allocated
  hipStream_t st = c->user_stream;
  if (ns > 0)
    HIP_TRY(c, hipMemcpyAsync(al, alpha, ns * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_TRY(c, launch_action(st, rows, n, ns, a0, al, B, X, out, part, nb));
  double2 h[BMS_MAX_RHS];
  HIP_TRY(c, hipMemcpyAsync(h, out, n * sizeof(double2), hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  for (int i = 0; i < n; ++i) S[i] = h[i].x;
  return BMS_OK;
}
