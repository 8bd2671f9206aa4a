// Internal declarations of the bms library: context, workspace, launchers.
#pragma once

#include <string>
#include <vector>

#include "../../include/bms.h"
#include "common.h"

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Workspace slots of a context (bms_ctx::scratch), one device buffer each,
// grown on first use of a larger shape and reused.
enum Slot {
  S_TMP = 0,  // odd-site temporary of bms_apply_mdagm
  S_W1,       // D_oe P^(0) (odd sites)
  S_W,        // (A + s0) P^(0)
  S_Q,        // orthonormal residual block Q_k (a ring of window-length buffers)
  S_P,        // directions P^(s)
  S_X,        // solutions X^(s) in the block precision
  S_SMALL,    // n x n FP64 state of the recurrences
  S_PART,     // partial sums of the grid reductions
  S_M,        // per-shift coefficient matrices of the update
  S_FLAGS,    // SolverFlags and the small-step arrival counter
  S_RES,      // residual norms, action sums, n x n Grams read back by the host
  S_LOG,      // per-iteration traffic log of the update
  S_R1,       // FP64 odd temporary
  S_R2,       // FP64 even temporary
  S_R0,       // FP64 true residual (reliable update)
  S_RB,       // FP64 defect-correction right-hand side
  S_E,        // FP64 defect-correction solution
  S_COLS,     // per-column scale factors
  S_RBC,      // one column of S_RB
  S_EC,       // its correction
  S_E2,       // FP64 solutions of the FP32 multi-shift phase
  S_CMAT,     // n x n FP64 coefficient matrix
  S_Y,        // bms_force: Y = D_oe X of every shift (odd sites)
  S_PHI,      // RHMC trajectory: the pseudofermion block phi
  S_XR,       // RHMC trajectory: shifted solutions of phi
  S_COUNT
};

// Device-side solver control block (all written by kernels, read by the host
// between graph chunks).
struct SolverFlags {
  int stop;       // iteration over: converged, max_iter or error (skip flag)
  int halted;     // the update kernel skips too (set one step after stop)
  int error;      // 0 or a BMS_E* code raised on the device
  int iter;       // completed block iterations
  int need_explicit;  // V^H V must come from the explicit Gram this iteration
  int rel_skip;       // the last reliable update kept the iterated residual
  int rel_restart;    // one shift: the last reliable update restarts P^(0) = Q
  int diverged;       // the true residual grew or stalled over reliable updates (soft stop)
  int rel_stall;      // reliable updates in a row without progress of the true residual
  int upd_done;       // `iter` as seen by the last matrix-core update that ran (-1: none)
  int rel_count;      // reliable updates that ran (not skipped after a stop)
  int active[BMS_MAX_SHIFTS];  // shift still updated
  int conv[BMS_MAX_SHIFTS];    // shift converged at the last rho step
  double res[BMS_MAX_SHIFTS];  // max relative residual estimate per shift
  // Deferred update of the shifts (matrix-core update): per shift and slot
  // (the iteration parity the small step writes for the update that follows
  // it), the iterations gathered in the open window and whether the update
  // applies them now.
  int win_j[2][BMS_MAX_SHIFTS];
  int win_flush[2][BMS_MAX_SHIFTS];
  int upd_stop;  // stop as seen by the last matrix-core update that ran
};

// Longest window of the deferred shift update (iterations gathered before the
// update applies them) that the state arrays hold.
constexpr int BMS_MAX_WIN = 8;

// Traversal of the half hop for one precision: tiles of whole x-rows ty x tz
// x tt in y, z, t (ty = 0: natural order; -1: the built-in choice for every
// field), at most `cap` resident work-groups per compute unit (0: no cap;
// -1: built-in by block width), non-temporal link loads (nt = 1).
struct HopCfg {
  int ty = -1, tz = 8, tt = 4;
  int cap = -1;
  int nt = 0;
};
struct HopPlan {
  bool quad = false, tiled = false, nt = false;
  int ty = 8, tz = 8, tt = 4, cap = 0;
  bool stream = false;  // k_hop_s: persistent waves with `depth` hops in flight
  int depth = 0;
};

struct bms_ctx {
  int dims[4];
  int bc[4];
  long vol;
  int vh;
  Geom geom;
  int sbl = 5;  // log2 of the link block (sites per SoA block)
  int nblk;     // link blocks per parity
  hipStream_t user_stream = nullptr;
  hipStream_t stream = nullptr;  // library-owned work stream
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int device = -1;
  int num_cu = 0;  // compute units of the device (set with the stream)
  int lds_per_cu = 0;  // bytes of LDS per compute unit (set with the stream)
  int lds_per_block = 0;  // bytes of LDS one work-group may take
  bool gauge_set = false;
  int nlinks = 8;  // links per site and output parity: 8, or 16 with three-hop links
  DevBuf links64, links32;  // [parity][blocked links] complex
  // The half hop's SU(3) links as their first two rows ([parity][blocked],
  // six entries per link) and per site a mask of the links whose scale
  // (+-1/2 times the phases) is negative; used when link_rows is 2 and every
  // link of the field passed the check at import (links_two_rows).
  DevBuf links64r, links32r, lsign, lcheck;
  int link_rows = 2;            // bms_set_link_rows: 2 (when the field allows) or 3
  bool links_two_rows = false;  // the hop reads links64r / links32r
  double link_dev = -1;         // largest third-row deviation found (-1: not checked)
  std::vector<DevBuf> scratch;  // named by slot index
  std::string last_error;
  // kernel variants (bms_set_variant); -1 = built-in default
  int update_variant = -1;
  int gram_variant = -1;
  int hop_variant = -1;
  int force_variant = -1;  // 0: D_oe hops per shift + per-link kernel; else fused
  HopCfg hop_cfg[2];       // [0] FP64, [1] FP32 blocks
  std::string tune_cache;  // bms_autotune's cache file ("" = none)
  // per-kernel timing (bms_timing_enable)
  bool timing = false;
  double kt_ms[BMS_NKERNELS] = {0};
  long long kt_launches[BMS_NKERNELS] = {0};
  double kt_bytes[BMS_NKERNELS] = {0};
  double kt_flops64[BMS_NKERNELS] = {0}, kt_flops32[BMS_NKERNELS] = {0};
  // per update launch: algorithmic bytes, FP64 and FP32 matrix-core flops
  std::vector<double> kt_upd_launch;
  std::vector<hipEvent_t> evpool;
  // graph cache for the iteration chunk
  hipGraphExec_t graph_exec = nullptr;
  std::string graph_key;
  // work done by the current bms_solve (reset at its start, reported in bms_stats)
  long it_f64 = 0, it_f32 = 0, hop_work = 0, rel_work = 0;
};

// error helpers
int set_err(bms_ctx* c, int code, const char* fmt, ...);
#define HIP_TRY(ctx, call)                                                          \
  do {                                                                              \
    hipError_t _e = (call);                                                         \
    if (_e != hipSuccess)                                                           \
      return set_err((ctx), _e == hipErrorOutOfMemory ? BMS_ENOMEM : BMS_EHIP,      \
                     "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), __FILE__, \
                     __LINE__);                                                     \
  } while (0)

int ensure_device(bms_ctx* c);
int ensure_buf(bms_ctx* c, DevBuf& b, size_t bytes);
int scratch_buf(bms_ctx* c, int slot, size_t bytes, void** p);
int stream_begin(bms_ctx* c);
// the host-side argument checks of bms_solve (BMS_OK or the error it returns)
int solve_validate(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                   int max_iter, const bms_opts* o, const void* B, const void* X);
// size every workspace slot a solve of this shape may use (see solver.cpp)
int solve_reserve(bms_ctx* c, double mass, int n, int ns, const double* shifts, double tol,
                  int max_iter, const bms_opts* opts, const void* B, const void* X);
int stream_end(bms_ctx* c);

// gauge-field steps of the RHMC trajectory (gauge.hip), on c->stream
int gauge_action_dev(bms_ctx* c, double beta, const void* U, double* S);
int gauge_force_dev(bms_ctx* c, double beta, const void* U, void* P, double scale);
int link_update_dev(bms_ctx* c, double eps, const void* P, void* U);
int kinetic_dev(bms_ctx* c, const void* P, double* K);

// ---- launchers (all enqueue on c->stream) ---------------------------------
hipError_t launch_gauge_import(const bms_ctx* c, const void* U, void* l64, void* l32,
                               void* r64, void* r32, void* sign, void* dev);
// the improved operator: one-hop links V and three-hop links W (16 per site)
hipError_t launch_gauge_import_improved(const bms_ctx* c, const void* V, const void* W, void* l64,
                                        void* l32);

// out = b * D_{par} in  (+ a * aux if aux)  on n columns; done = optional
// device flag (skip if *done)
HopPlan hop_plan(const bms_ctx* c, int n, bool fp64);
size_t hop_cap_lds(const bms_ctx* c, int cap);
// whether ty x tz x tt tiles of whole x-rows divide this lattice for block width n
bool hop_tiling_valid(const bms_ctx* c, int n, int ty, int tz, int tt);
template <typename T>
hipError_t launch_hop(const bms_ctx* c, int par, int n, const void* in, void* out, const void* aux,
                      double a, double b, const int* skip);

// G (n x n, FP64) = X^H Y over `rows` rows of n complex: nb blocks write
// partial Grams (partials must hold nb*n*n double2), a second kernel sums them.
template <typename T>
hipError_t launch_gram(hipStream_t st, int rows, int n, const void* X, const void* Y, double2* G,
                       double2* partials, int nb, const int* skip);
int gram_blocks(int rows, int n, int num_cu);

// Y = X M (rows x n times n x n, M FP64 on device), optionally Y += (accum)
template <typename T>
hipError_t launch_block_matmul(hipStream_t st, int rows, int n, const void* X, const double2* M,
                               void* Y);

hipError_t launch_fill_zero(hipStream_t st, void* p, size_t bytes);
// dst = src (bytes a multiple of 16) when *run_if is non-zero
hipError_t launch_copy_if(hipStream_t st, void* dst, const void* src, size_t bytes,
                          const int* run_if);
