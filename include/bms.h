/*
 * bms — block multi-shift staggered solver for RHMC on MI355X (gfx950).
 *
 * C ABI of the hot path of de Forcrand & Keegan, "Rational Hybrid Monte Carlo
 * with Block Solvers and Multiple Pseudofermions": applying the even-odd
 * staggered normal operator to a block of n_pf pseudofermions, solving
 * (A + sigma_s) X^(s) = B for all shifts of a rational approximation with the
 * block multi-shift solver SBCGrQ (Algorithm 1), the pseudofermion action
 * (eq. RA inside the action of Sec. II) and its link derivative (eq. force).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status: every function returns BMS_OK (0) or a negative BMS_E* code.
 *   bms_error_string() names a code; bms_last_error() gives the message of
 *   the last failure on a context. Outputs are defined only on BMS_OK, except
 *   where an entry point says otherwise (BMS_ENOCONV, BMS_EBREAKDOWN).
 * Ownership: the caller owns every array. Device arrays are plain device
 *   pointers (hipMalloc'ed or from a framework allocator), contiguous, in the
 *   layouts below; work is ordered on the context's HIP stream. The library
 *   owns only the opaque context and its workspace, which it allocates on
 *   first use of a given shape and reuses. A context is not thread-safe and
 *   serves one stream.
 * Argument errors are detected on the host before any device work is
 *   enqueued and return BMS_EINVAL with nothing written.
 *
 * Lattice and layouts
 * -------------------
 * dims = {Lx, Ly, Lz, Lt}, each even and >= 2; V = Lx*Ly*Lz*Lt, Vh = V/2.
 * Site index idx = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t)&1;
 * checkerboard index cb = idx >> 1.
 * bc = {bx, by, bz, bt}, each +1 or -1: the factor of a link crossing the
 *   lattice boundary in that direction (e.g. {1,1,1,-1} antiperiodic in t).
 * Gauge field U[mu][idx][a][b], complex128 (interleaved re, im): the SU(3)
 *   link from idx to idx + mu. Any complex 3x3 matrices are accepted.
 * Block vector (even or odd sites) v[cb][color][rhs], complex128 for
 *   BMS_PREC_F64 and complex64 for BMS_PREC_F32: site-major, right-hand
 *   side fastest, Vh*3*n complex numbers.
 * Solutions X[shift][cb][color][rhs], complex128, shifts in the caller's order.
 * Link gradient G[mu][idx][a][b], complex128.
 *
 * Operator (Sec. IV names unimproved staggered fermions with even-odd
 * preconditioning; the form is the textbook one):
 *   (D psi)(x) = 1/2 sum_mu eta_mu(x) [ U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu) ]
 *   eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}), boundary links carry bc[mu];
 *   M = m + D,  A = M^dag M on even sites = m^2 - D_eo D_oe.
 */
#ifndef BMS_H
#define BMS_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BMS_OK 0
#define BMS_EINVAL (-1)      /* bad argument (detected before any device work) */
#define BMS_ENOMEM (-2)      /* device allocation failed */
#define BMS_EHIP (-3)        /* a HIP runtime call failed */
#define BMS_EBREAKDOWN (-4)  /* rank-deficient block (Cholesky pivot not positive) */
#define BMS_ENOCONV (-5)     /* max_iter reached before every shift met tol */
#define BMS_ENAN (-6)        /* non-finite value met in the iteration */
#define BMS_ESTATE (-7)      /* call out of order (e.g. no gauge field set) */

/* arithmetic precision */
#define BMS_PREC_F64 0   /* everything in FP64 */
#define BMS_PREC_F32 1   /* operator only: FP32 links, FP32 vectors (complex64 in/out) */
#define BMS_PREC_MIXED 2 /* solver only: FP32 operator and block updates, FP64 small
                            matrices, FP64 reliable updates and defect correction */

#define BMS_MAX_RHS 32    /* largest block width n accepted */
#define BMS_MAX_SHIFTS 64 /* largest number of shifts accepted */

typedef struct bms_ctx bms_ctx;

/* Solver options; bms_default_opts() fills the defaults listed here. */
typedef struct bms_opts {
  int precision;          /* BMS_PREC_F64 (default) or BMS_PREC_MIXED */
  int reliable_interval;  /* MIXED: iterations between FP64 reliable updates (50) */
  double freeze_tol;      /* a shift stops being updated once every column's residual
                             estimate is below this; <= 0 means tol (default 0) */
  int check_interval;     /* iterations between host-side convergence checks (8) */
  int max_refine;         /* MIXED: rounds of per-shift defect correction (4) */
  int qr_passes;          /* Cholesky-QR passes per iteration, 1 or 2 (1) */
  int use_graph;          /* replay each chunk of check_interval iterations from a
                             captured hipGraph (1, default), or launch directly (0);
                             chunks launch directly while timing is enabled */
  double mixed_switch;    /* MIXED: relative residual of the smallest shift at which
                             the FP64 block multi-shift phase hands over to the
                             FP32 one (3e-4); the FP32 phase solves for the
                             remaining residual of every unconverged shift at once.
                             <= tol, or >= 1: FP32 from the start */
} bms_opts;

/* Solver statistics (filled on BMS_OK, BMS_ENOCONV and BMS_EBREAKDOWN). Every
   block iteration of the solve is counted once, in whichever phase ran it:
   iterations = multishift_iterations + refine_iterations
              = iterations_f64 + iterations_f32. */
typedef struct bms_stats {
  int iterations;          /* block iterations of every phase */
  int multishift_iterations; /* of these, the first block multi-shift loop on B
                              (Algorithm 1; in MIXED the FP64 phase down to
                              mixed_switch) */
  int refine_iterations;   /* the iterations after it: the FP32 multi-shift phase
                              (MIXED), an FP64 restart after a diverged FP32 loop,
                              and the per-shift defect correction */
  int iterations_f64;      /* block iterations on FP64 blocks */
  int iterations_f32;      /* block iterations on FP32 blocks */
  int hop_calls;           /* half hops that did work: two per block iteration, two
                              per reliable update, two per shift of each true-residual
                              check or residual formation */
  int reliable_updates;    /* MIXED: FP64 residual replacements that ran */
  int converged;           /* 1 if every shift and column met tol (true FP64 residual) */
  double max_true_residual;/* max over shifts and columns of |b - (A+s)x| / |b| */
  double* true_residual;   /* optional caller array [n_shifts][n]; NULL to skip */
} bms_stats;

void bms_default_opts(bms_opts* opts);

/* Name of a status code (static string). */
const char* bms_error_string(int status);

/* Message of the last failure on ctx (empty if none; valid until the next call). */
const char* bms_last_error(const bms_ctx* ctx);

/*
 * Create a context for one lattice. dims and bc as above; stream is a
 * hipStream_t (NULL = the default stream). Performs no device work; device
 * memory is allocated by bms_set_gauge and the first call of each shape.
 * Errors: BMS_EINVAL for a null ctx, odd or < 2 extents, an extent above 4096,
 * bc not +-1, or a volume above 2^25 sites.
 */
int bms_create(bms_ctx** ctx, const int dims[4], const int bc[4], void* stream);

/* Release the context and all device memory it owns (waits for its stream). */
int bms_destroy(bms_ctx* ctx);

/*
 * Load the gauge field (device pointer, U[mu][idx][a][b] complex128). The
 * library keeps its own copies: per output parity, the 8 links each site's
 * half hop needs, with the 1/2, eta_mu and boundary factors folded in (and
 * the backward links daggered), in FP64 and FP32. U is not referenced after
 * the call returns (the copy is ordered on the stream).
 * With two link rows selected (bms_set_link_rows, the default) the call also
 * keeps the first two rows of every link and checks that each third row is
 * what SU(3) implies, row2 = conj(row0 x row1) for the unscaled matrix, to
 * 1e-12 in every part; when all pass, the half hop reads two rows per link
 * and rebuilds the third (a third fewer link bytes), else it reads all
 * nine entries. That check waits for the import (a host synchronisation).
 */
int bms_set_gauge(bms_ctx* ctx, const void* U);

/*
 * How many rows of each SU(3) link the half hop reads: 2 (default: when the
 * field loaded by bms_set_gauge passes its check) or 3 (always all nine
 * entries). Takes effect at the next bms_set_gauge; BMS_EINVAL for other
 * values. bms_get_link_rows returns in *rows the form the current links are
 * read in: 2, or 3 (also for the improved operator's links, which are not
 * SU(3) matrices), and in *max_dev (may be NULL) the largest difference the
 * last check found between a third row and the SU(3) one (+inf for a value
 * that is not finite; -1 when no check ran).
 */
int bms_set_link_rows(bms_ctx* ctx, int rows);
int bms_get_link_rows(const bms_ctx* ctx, int* rows, double* max_dev);

/*
 * Load the links of the improved, less local staggered operator (the
 * paper's outlook, Sec. V, expects a less local operator to gain more from
 * reading each link once per block): one-hop links V and three-hop links W,
 * both device pointers in the layout of U, the improvement coefficients
 * folded in by the caller (e.g. V = 9/8 x fat links, W = -1/24 x long links
 * for the Naik term):
 *   (D psi)(x) = 1/2 sum_mu eta_mu(x) [ V_mu(x) psi(x+mu) - V_mu(x-mu)^dag psi(x-mu)
 *                                     + W_mu(x) psi(x+3mu) - W_mu(x-3mu)^dag psi(x-3mu) ]
 * with the boundary factor bc[mu] on every link or three-hop link that
 * crosses the lattice boundary. Every later bms_apply_hop, bms_apply_mdagm,
 * bms_solve, bms_rational_apply and bms_autotune acts with it (16 links per
 * site and half hop) until bms_set_gauge loads unimproved links; bms_force
 * then returns BMS_EINVAL. Errors: BMS_EINVAL for NULL pointers or an extent
 * below 4.
 */
int bms_set_gauge_improved(bms_ctx* ctx, const void* V, const void* W);

/*
 * out = D_{parity_out, 1-parity_out} in: the half hop from sites of parity
 * 1-parity_out to sites of parity parity_out (parity_out = 1 gives D_oe,
 * 0 gives D_eo) on n columns. precision BMS_PREC_F64 or BMS_PREC_F32 selects
 * complex128 or complex64 arrays and arithmetic. in and out must not alias.
 */
int bms_apply_hop(bms_ctx* ctx, int parity_out, int n, const void* in, void* out, int precision);

/*
 * out = (A + sigma) in = (m^2 + sigma) in - D_eo D_oe in on even sites for n
 * columns (mass = m). precision as for bms_apply_hop. in and out must not alias.
 */
int bms_apply_mdagm(bms_ctx* ctx, double mass, double sigma, int n, const void* in, void* out,
                    int precision);

/*
 * Block multi-shift solve (Algorithm 1, SBCGrQ): X^(s) = (A + shifts[s])^-1 B
 * for s = 0..n_shifts-1 and all n columns of B at once.
 *   shifts: host array, each >= 0, any order; the smallest one drives the
 *           unshifted recurrence (sigma_0). Duplicates are allowed.
 *   tol:    target relative residual per column and shift, in (0, 1). The
 *           loop runs until every shifted residual estimate |delta^(s) e_i| / |b_i|
 *           is below tol/2 (a margin for the drift between the recurrence and
 *           the true residual); then the true FP64 residuals are computed and
 *           shifts above tol are refined by defect correction.
 *   B:      device block [cb][color][rhs] complex128 (even sites), full column rank.
 *   X:      device output [shift][cb][color][rhs] complex128.
 *   opts:   NULL for defaults. stats: NULL or caller struct.
 * Returns BMS_OK when every column of every shift has true relative residual
 * <= tol; BMS_ENOCONV when max_iter block iterations were not enough (X holds
 * the last iterate, stats the residuals); BMS_EBREAKDOWN when the block lost
 * rank (e.g. linearly dependent columns in B); BMS_ENAN on non-finite values.
 */
int bms_solve(bms_ctx* ctx, double mass, int n, int n_shifts, const double* shifts, double tol,
              int max_iter, const bms_opts* opts, const void* B, void* X, bms_stats* stats);

/*
 * Rational function of the operator applied to a block (eq. RA):
 *   out = r(A) B = a0 B + sum_j alpha[j] (A + shifts[j])^-1 B,
 * e.g. the pseudofermion heatbath phi = r(A) eta with r(x) ~ x^(+p/2) and
 * Gaussian eta (Sec. II), or the accept-step action's solves with
 * r(x) ~ x^(-p) fitted to relative error 1e-15 (the paper runs these at
 * residual 1e-14, Sec. IV). The solutions X^(j) are those of bms_solve (same
 * arguments, same stopping rule and errors, written to the caller's X
 * [shift][cb][color][rhs]); out (device, [cb][color][rhs] complex128, must not
 * alias B or X) is written only on BMS_OK. alpha[] (host) may have any sign
 * (a fit of a positive power has negative residues).
 */
int bms_rational_apply(bms_ctx* ctx, double mass, int n, int n_shifts, double a0,
                       const double* alpha, const double* shifts, double tol, int max_iter,
                       const bms_opts* opts, const void* B, void* X, void* out,
                       bms_stats* stats);

/*
 * Pseudofermion action per column (Sec. II with eq. RA):
 *   S_i = Re phi_i^dag (a0 phi_i + sum_j alpha[j] X^(j) phi-column i),
 * from B (device, complex128 [cb][color][rhs]) and solutions X (device,
 * [shift][cb][color][rhs]). S is a host array of n doubles. Blocks until done.
 */
int bms_action(bms_ctx* ctx, int n, int n_shifts, double a0, const double* alpha, const void* B,
               const void* X, double* S);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): bms_action without
 * any allocation. Same arguments, result and errors as bms_action. Its
 * scratch (residues, partial sums, the n sums; at most 0.55 MB for n = 32) is
 * a static 1 MiB device array per GPU, held until the process ends; the
 * call runs on the context's stream (the one given to bms_create), creates
 * no stream or event and blocks until S is written. Calls that overlap on one
 * GPU (other streams or host threads) share that array and race. A shape
 * whose scratch would exceed 1 MiB is rejected with BMS_EINVAL (none exists
 * within BMS_MAX_RHS).
 */
int bms_action_noalloc(bms_ctx* ctx, int n, int n_shifts, double a0, const double* alpha,
                       const void* B, const void* X, double* S);

#define BMS_FORCE_RAW 0 /* G = dS/dRe U + i dS/dIm U, [mu][idx][3][3] complex128 */
#define BMS_FORCE_LIE 1 /* F^a = -dS/d omega^a for U -> exp(i omega^a T^a) U, T^a = lambda_a/2,
                           [mu][idx][8] float64 */
#define BMS_FORCE_ADD 2 /* or-ed into flags: out += the result instead of out = (e.g. a
                           momentum update P += eps F with alpha scaled by eps) */

/*
 * Link derivative of S = sum_i sum_j alpha[j] phi_i^dag (A + s_j)^-1 phi_i
 * (eq. force) from the solutions X^(j) = (A + s_j)^-1 B (device,
 * [shift][cb][color][rhs] complex128) and host residues alpha[n_shifts]:
 *   dS = -2 sum_ij alpha_j Re[ y_ij^dag dD_oe x_ij ],  y = D_oe x,
 * i.e. per link M_mu(w) = -eta b sum alpha x(w+mu) y(w)^dag (w odd) or
 * +eta b sum alpha y(w+mu) x(w)^dag (w even), returned as G = M^dag
 * (flags = BMS_FORCE_RAW) or F^a = Im Tr[T^a U M] (BMS_FORCE_LIE).
 * out is a device array overwritten in full, or added to with BMS_FORCE_ADD.
 * Defined for the unimproved operator (BMS_EINVAL after bms_set_gauge_improved).
 */
int bms_force(bms_ctx* ctx, int n, int n_shifts, const double* alpha, const void* X, void* out,
              int flags);

/*
 * Gauge-field steps of an RHMC trajectory (the Wilson gauge part of the HMC
 * Hamiltonian, Sec. II and Sec. IV), on the context's lattice. Links U
 * [mu][idx][3][3] complex128 (periodic), momenta P [mu][idx][8] float64
 * (components along T^a = lambda_a / 2), all device pointers.
 *   bms_gauge_action    S = beta sum_{x, mu<nu} (1 - Re Tr U_mu nu(x) / 3) (host double)
 *   bms_gauge_force     P += scale F, F^a = -dS/d omega^a for U -> exp(i omega^a T^a) U,
 *                       i.e. F^a = -(beta/3) Im Tr(T^a U_mu(x) A_mu(x)) with the
 *                       staple sum A of the six plaquettes through the link
 *   bms_gauge_update    U <- exp(i eps P^a T^a) U (every link)
 *   bms_kinetic_energy  K = 1/2 sum (P^a)^2 (host double)
 * The sums block until done. Errors: BMS_EINVAL for NULL or non-finite arguments.
 */
int bms_gauge_action(bms_ctx* ctx, double beta, const void* U, double* S);
int bms_gauge_force(bms_ctx* ctx, double beta, const void* U, void* P, double scale);
int bms_gauge_update(bms_ctx* ctx, double eps, const void* P, void* U);
int bms_kinetic_energy(bms_ctx* ctx, const void* P, double* K);

/* Parameters of bms_rhmc_trajectory; bms_default_rhmc_params fills the
   defaults shown (and NULL coefficient pointers). */
typedef struct bms_rhmc_params {
  double beta;       /* Wilson gauge coupling (5.12) */
  double mass;       /* staggered mass m (0.05) */
  int n;             /* pseudofermions = block width (1); 0 runs pure gauge HMC */
  double tau;        /* trajectory length (1) */
  int n_steps;       /* outer Omelyan steps, fermion force (10) */
  int n_gauge;       /* inner Omelyan steps of the gauge force per outer drift (3) */
  double lambda;     /* Omelyan parameter (1/6) */
  int ns_hb;         /* heatbath r_hb(x) ~ x^(+p/2): a0 + sum alpha/(x + beta) */
  double a0_hb;
  const double* alpha_hb;
  const double* beta_hb;
  int ns_acc;        /* action r(x) ~ x^(-p) for H (heatbath and accept accuracy) */
  double a0_acc;
  const double* alpha_acc;
  const double* beta_acc;
  int ns_md;         /* force r(x) ~ x^(-p) (molecular-dynamics accuracy; a0 drops out) */
  const double* alpha_md;
  const double* beta_md;
  double tol_hb;     /* heatbath and action solves (1e-14) */
  double tol_md;     /* force solves (1e-7) */
  int precision_md;  /* BMS_PREC_F64 (default) or BMS_PREC_MIXED for the force solves */
  int max_iter;      /* block iterations per solve (100000) */
} bms_rhmc_params;

typedef struct bms_rhmc_result {
  double H0, H1, dH;        /* H = K + S_g + S_f before and after the molecular dynamics */
  double K0, K1, Sg0, Sg1, Sf0, Sf1;
  double max_residual_hb;   /* worst true residual of the heatbath and action solves */
  long long iterations;     /* block iterations of every solve */
  int force_evals;          /* fermion-force evaluations */
} bms_rhmc_result;

void bms_default_rhmc_params(bms_rhmc_params* p);

/*
 * One RHMC trajectory (Sec. II; the settings of Sec. IV) with n pseudofermions
 * solved as one block:
 *   heatbath phi = r_hb(A) eta (bms_rational_apply at tol_hb);
 *   H0 = 1/2 sum P^2 + S_g(U) + sum_i phi_i^dag r(A) phi_i (accept rational, tol_hb);
 *   molecular dynamics over tau by the two-level second-order Omelyan scheme:
 *   with h = tau / n_steps, per step P += lambda h F_f, a link drift over h/2,
 *   P += (1 - 2 lambda) h F_f, a drift over h/2, P += lambda h F_f (the kicks of
 *   adjacent steps merged), each drift being n_gauge Omelyan steps of the
 *   gauge force and U <- exp(i e P) U; the fermion force F_f is bms_force's Lie
 *   force of the force rational with its solves at tol_md;
 *   H1 and dH = H1 - H0.
 * U (in/out) and P (in/out, momenta drawn by the caller as P^a ~ N(0, 1)) are
 * device arrays in the layouts above; eta is the device Gaussian block
 * [cb][color][n] complex128 (NULL when n = 0). The caller keeps a copy of U
 * and accepts with probability min(1, exp(-dH)). The library's own copy of
 * the links follows U (bms_set_gauge is called on every new U).
 * Errors: BMS_EINVAL for bad parameters; a failing solve's status (r holds
 * what was computed up to it); BMS_ENAN for a non-finite energy.
 */
int bms_rhmc_trajectory(bms_ctx* ctx, const bms_rhmc_params* p, void* U, void* P,
                        const void* eta, bms_rhmc_result* r);

/*
 * Per-kernel GPU timing. While enabled, bms_solve records HIP events on the
 * library stream around every kernel of each block iteration and accumulates,
 * per kernel class, the summed event time, the number of launches that did
 * work, and their algorithmic HBM bytes (each block vector, link and solution
 * read or written once per launch; small n x n data not counted):
 *   BMS_KERNEL_HOP      half hop, links + in + out (+ aux for the D_eo hop)
 *   BMS_KERNEL_GRAM     the iteration's four Grams: P, Q, W read
 *   BMS_KERNEL_CHOLQR   Cholesky-QR Gram: Q, W read
 *   BMS_KERNEL_UPDATE   fused update: Q, W read, Q written, and per shift
 *                       whose update window it applies P^(s), X^(s) read and
 *                       written plus, once, the earlier Q blocks the longest
 *                       such window spans (every active shift every iteration
 *                       for variants 0..3 and 6)
 *   BMS_KERNEL_SMALL    the n x n kernels (no block data)
 *   BMS_KERNEL_FORCE    the whole bms_force call (for variant 0 its D_oe hops
 *                       included): every solution read once, the 4V FP64
 *                       links once, the output written once
 * bms_timing_enable(ctx, 1) also clears the
 * accumulators; bms_timing_read returns them (host pointers, any may be NULL).
 * bms_timing_flops returns the matrix-core work of the same launches for
 * BMS_KERNEL_UPDATE (the real products of the Q step and of the applied
 * windows, 2 flops per multiply-add: per complex product 3 rows n^2 for
 * n = 16, rows (2n)^2 for n = 8), split into FP64 and FP32 arithmetic; 0 for
 * the other classes and for the vector kernels.
 * bms_timing_floor returns in *seconds the least time the recorded launches
 * of a class need at the given peaks (bytes/s, FP64 and FP32 flops/s, each
 * > 0): for BMS_KERNEL_UPDATE the sum over its launches of
 * max(bytes / hbm, flops_f64 / f64 + flops_f32 / f32), each launch bound by
 * whichever roof is higher for it; for the other classes bytes / hbm.
 * BMS_EINVAL for a bad kernel, a NULL output or a peak that is not positive.
 */
#define BMS_KERNEL_HOP 0
#define BMS_KERNEL_GRAM 1
#define BMS_KERNEL_CHOLQR 2
#define BMS_KERNEL_UPDATE 3
#define BMS_KERNEL_SMALL 4
#define BMS_KERNEL_FORCE 5
#define BMS_NKERNELS 6

int bms_timing_enable(bms_ctx* ctx, int enable);

/*
 * Kernel variant selection. For BMS_KERNEL_UPDATE: 4 and 5 = the
 * matrix-core (MFMA) kernel at n = 8 and 16 (FP32 or FP64 blocks, the Q step
 * in FP64) with one or two 16-row tiles per wave, where the shifts other
 * than the smallest are updated once per window of iterations (4 in FP64,
 * 8 in FP32: X^(s) and P^(s) of the whole window from the window's start and
 * the Q blocks it spans, 4 block vectors per shift per window instead of per
 * iteration; Algorithm 1's updates composed over the window);
 * 6 = the same kernel updating every shift every iteration, one tile per
 * wave; 0..3 = the vector kernels
 * (0 = four row chunks per work-group with both coefficient columns in
 * registers, 1 = two chunks, one column at a time, 2 = four chunks, one
 * column at a time, 3 = two chunks, both columns); -1 restores the built-in
 * default (4 where it applies, else 2). For BMS_KERNEL_GRAM (n = 8 and 16,
 * FP32 or FP64 inputs, FP64 accumulation): 1 and 2 = the matrix-core kernel
 * with every wave streaming its own rows, 4 or 8 row steps in flight; 3, 4,
 * 5 = the matrix-core kernel with rows staged through LDS, 1, 2 or 4 chunks
 * in flight per work-group; 0 = the vector kernel; -1 = the default (2).
 * For BMS_KERNEL_HOP: 1 = four threads per site sharing the site's links
 * (n = 4, 8, 16, 32), 0 = one thread per site and column group, 2 and 3 = 0
 * and 1 in a tiled traversal (8 x 8 x 4 tiles in y, z, t of whole x-rows,
 * each (y, z) pencil on one XCD; lattices the tiles do not fit run in the
 * natural order), 4 = at n = 16 persistent waves that keep the next hops'
 * columns and links in flight through a ring in LDS (direct-to-LDS loads;
 * for lattices with V/2 a multiple of 128 and a ring that fits one
 * work-group's LDS, else variant 1; the hop configuration's tiles apply and
 * its cap is the ring depth, 2 or 4), -1 = the default (1 where it applies,
 * tiled in FP64 at n >= 16). For BMS_KERNEL_FORCE: 1 and 2 = the fused kernel (y = D_oe x
 * formed on chip for all n * n_shifts columns, each link loaded once and
 * written once; links in registers, or in LDS with the loads two columns
 * ahead), 0 = D_oe hops per shift into a buffer, then one lane group per
 * link; -1 = the default (2). Other kernels are rejected with BMS_EINVAL;
 * other widths and precisions ignore the setting. Results do not depend on the variant beyond rounding
 * order.
 */
int bms_set_variant(bms_ctx* ctx, int kernel, int variant);

/*
 * Traversal of the half hop for one precision (BMS_PREC_F64 or BMS_PREC_F32
 * blocks): cfg = {ty, tz, tt, cap, nt}.
 *   ty, tz, tt  tiles of whole x-rows, ty x tz x tt sites in y, z, t; the
 *               (y, z) pencils of tiles go to the 8 XCDs in turn and each XCD
 *               walks its pencils tile after tile along t (lattices the tiles do
 *               not divide run in the natural order); ty = 0: natural order
 *   cap         at most cap resident work-groups per compute unit (0: no cap;
 *               -1: the built-in choice by block width)
 *   nt          1: link loads with the non-temporal hint
 * cfg = NULL or cfg[0] = -1 restores the built-in choice. Applies to the
 * quad and per-group hop kernels alike (bms_set_variant picks the kernel);
 * results do not depend on it. bms_get_hop_config returns the setting.
 * Errors: BMS_EINVAL for a bad precision, extent, cap or nt.
 */
int bms_set_hop_config(bms_ctx* ctx, int precision, const int cfg[5]);
int bms_get_hop_config(const bms_ctx* ctx, int precision, int cfg[5]);

/*
 * Cache file of bms_autotune (a text file of JSON lines, one per tuned
 * problem shape; NULL or "" = no cache). With a cache set, bms_autotune
 * first looks for the key (device architecture, lattice, n, n_shifts,
 * precision, links per site and link rows read) and applies the stored choice without timing anything; on a
 * miss it times the candidates and appends the result.
 */
int bms_set_tune_cache(bms_ctx* ctx, const char* path);

/* The variant currently set for a kernel class (BMS_KERNEL_HOP, _GRAM, _UPDATE). */
int bms_get_variant(const bms_ctx* ctx, int kernel, int* variant);

/*
 * Pick the fastest variant of the hop, Gram and update kernels for this
 * context's lattice, block width n, shifts and precision (BMS_PREC_F64 or
 * BMS_PREC_MIXED): one kernel class after another, every candidate is timed
 * (HIP events on the library stream) over `iters` block iterations of a
 * real solve of B, and the fastest is kept (see bms_set_variant). B as for
 * bms_solve; X is a caller array of the bms_solve shape used as scratch (its
 * contents are undefined afterwards). Results of later solves do not depend
 * on the choice beyond rounding order. Errors: BMS_EINVAL for bad arguments
 * (as bms_solve, plus iters outside [1, 4096]); the status of a failing solve
 * otherwise.
 */
int bms_autotune(bms_ctx* ctx, double mass, int n, int n_shifts, const double* shifts,
                 int precision, int iters, const void* B, void* X);

/*
 * A batch of independent solves, e.g. an uneven batch of gauge fields on
 * different lattices: problem i is bms_solve(ctxs[i], mass[i], n[i],
 * n_shifts[i], shifts[i], tol[i], max_iter[i], opts ? &opts[i] : NULL, B[i],
 * X[i], stats ? &stats[i] : NULL), each on its own context (distinct
 * contexts; each with its own library stream), all run at the same time from
 * host threads so that the GPU overlaps them. status[i] receives problem i's
 * status. Returns BMS_OK when every problem did, else the first failing
 * problem's status; BMS_EINVAL (nothing run) for nprob outside [1, 64], a
 * NULL array or context, or a context given twice. Blocks until all are done.
 */
int bms_solve_batch(int nprob, bms_ctx* const* ctxs, const double* mass, const int* n,
                    const int* n_shifts, const double* const* shifts, const double* tol,
                    const int* max_iter, const bms_opts* opts, const void* const* B,
                    void* const* X, bms_stats* stats, int* status);
int bms_timing_read(const bms_ctx* ctx, int kernel, double* ms, long long* launches,
                    double* bytes);
int bms_timing_flops(const bms_ctx* ctx, int kernel, double* flops_f64, double* flops_f32);
int bms_timing_floor(const bms_ctx* ctx, int kernel, double hbm_bytes_per_s,
                     double f64_flops_per_s, double f32_flops_per_s, double* seconds);

#ifdef __cplusplus
}
#endif

#endif /* BMS_H */
