"""Thin Python binding of the bms C ABI (include/bms.h).

Argument marshalling only: every step runs in libbms.so. Functions carry the
C names; tensors are torch CUDA tensors (complex128 unless noted), contiguous,
in the layouts of bms.h:

  gauge U[mu][idx][3][3], block B[cb][3][n], solutions X[shift][cb][3][n],
  gradient G[mu][idx][3][3] (or F[mu][idx][8] float64 for BMS_FORCE_LIE).

Raises BmsError (a RuntimeError) on any non-zero status. The library must be
built (paper_1808_01829_amd/build.py); importing fails loudly otherwise.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbms.so")

BMS_OK = 0
BMS_EINVAL = -1
BMS_ENOMEM = -2
BMS_EHIP = -3
BMS_EBREAKDOWN = -4
BMS_ENOCONV = -5
BMS_ENAN = -6
BMS_ESTATE = -7
BMS_PREC_F64 = 0
BMS_PREC_F32 = 1
BMS_PREC_MIXED = 2
BMS_MAX_RHS = 32
BMS_MAX_SHIFTS = 64
BMS_FORCE_RAW = 0
BMS_FORCE_LIE = 1

BMS_KERNEL_HOP = 0
BMS_KERNEL_GRAM = 1
BMS_KERNEL_CHOLQR = 2
BMS_KERNEL_UPDATE = 3
BMS_KERNEL_SMALL = 4
BMS_KERNEL_FORCE = 5
KERNEL_NAMES = ["hop", "gram", "cholqr_gram", "update", "small", "force"]

EXPORTS = ["bms_default_opts", "bms_error_string", "bms_last_error", "bms_create", "bms_destroy",
           "bms_set_gauge", "bms_apply_hop", "bms_apply_mdagm", "bms_solve", "bms_action",
           "bms_force", "bms_timing_enable", "bms_timing_read", "bms_set_variant",
           "bms_get_variant", "bms_autotune", "bms_solve_batch", "bms_action_noalloc",
           "bms_rational_apply", "bms_set_hop_config", "bms_get_hop_config",
           "bms_set_tune_cache", "bms_set_gauge_improved", "bms_gauge_action",
           "bms_gauge_force", "bms_gauge_update", "bms_kinetic_energy",
           "bms_default_rhmc_params", "bms_rhmc_trajectory", "bms_timing_flops",
           "bms_timing_floor", "bms_set_link_rows", "bms_get_link_rows"]


class bms_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("reliable_interval", ctypes.c_int),
                ("freeze_tol", ctypes.c_double), ("check_interval", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("qr_passes", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("mixed_switch", ctypes.c_double)]


class bms_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("multishift_iterations", ctypes.c_int),
                ("refine_iterations", ctypes.c_int), ("iterations_f64", ctypes.c_int),
                ("iterations_f32", ctypes.c_int), ("hop_calls", ctypes.c_int),
                ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("max_true_residual", ctypes.c_double),
                ("true_residual", ctypes.POINTER(ctypes.c_double))]


_STAT_INTS = ("iterations", "multishift_iterations", "refine_iterations", "iterations_f64",
              "iterations_f32", "hop_calls", "reliable_updates")


def _stats_dict(st):
    d = {k: getattr(st, k) for k in _STAT_INTS}
    d["converged"] = bool(st.converged)
    d["max_true_residual"] = st.max_true_residual
    return d


_dp = ctypes.POINTER(ctypes.c_double)


class bms_rhmc_params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("mass", ctypes.c_double), ("n", ctypes.c_int),
                ("tau", ctypes.c_double), ("n_steps", ctypes.c_int), ("n_gauge", ctypes.c_int),
                ("lambda_", ctypes.c_double),
                ("ns_hb", ctypes.c_int), ("a0_hb", ctypes.c_double), ("alpha_hb", _dp),
                ("beta_hb", _dp),
                ("ns_acc", ctypes.c_int), ("a0_acc", ctypes.c_double), ("alpha_acc", _dp),
                ("beta_acc", _dp),
                ("ns_md", ctypes.c_int), ("alpha_md", _dp), ("beta_md", _dp),
                ("tol_hb", ctypes.c_double), ("tol_md", ctypes.c_double),
                ("precision_md", ctypes.c_int), ("max_iter", ctypes.c_int)]


class bms_rhmc_result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("H0", "H1", "dH", "K0", "K1", "Sg0", "Sg1", "Sf0",
                                                "Sf1", "max_residual_hb")] + \
               [("iterations", ctypes.c_longlong), ("force_evals", ctypes.c_int)]


class BmsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_lib().bms_error_string(code).decode(), msg))
        self.code = code


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libbms.so is not built (run paper_1808_01829_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        vp, ip, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(
            ctypes.c_double), ctypes.c_int, ctypes.c_double
        L.bms_default_opts.argtypes = [ctypes.POINTER(bms_opts)]
        L.bms_default_opts.restype = None
        L.bms_error_string.argtypes = [i]
        L.bms_error_string.restype = ctypes.c_char_p
        L.bms_last_error.argtypes = [vp]
        L.bms_last_error.restype = ctypes.c_char_p
        L.bms_create.argtypes = [ctypes.POINTER(vp), ip, ip, vp]
        L.bms_destroy.argtypes = [vp]
        L.bms_set_gauge.argtypes = [vp, vp]
        L.bms_set_gauge_improved.argtypes = [vp, vp, vp]
        L.bms_gauge_action.argtypes = [vp, d, vp, dp]
        L.bms_gauge_force.argtypes = [vp, d, vp, vp, d]
        L.bms_gauge_update.argtypes = [vp, d, vp, vp]
        L.bms_kinetic_energy.argtypes = [vp, vp, dp]
        L.bms_default_rhmc_params.argtypes = [ctypes.POINTER(bms_rhmc_params)]
        L.bms_default_rhmc_params.restype = None
        L.bms_rhmc_trajectory.argtypes = [vp, ctypes.POINTER(bms_rhmc_params), vp, vp, vp,
                                          ctypes.POINTER(bms_rhmc_result)]
        L.bms_apply_hop.argtypes = [vp, i, i, vp, vp, i]
        L.bms_apply_mdagm.argtypes = [vp, d, d, i, vp, vp, i]
        L.bms_solve.argtypes = [vp, d, i, i, dp, d, i, ctypes.POINTER(bms_opts), vp, vp,
                                ctypes.POINTER(bms_stats)]
        L.bms_action.argtypes = [vp, i, i, d, dp, vp, vp, dp]
        L.bms_rational_apply.argtypes = [vp, d, i, i, d, dp, dp, d, i, ctypes.POINTER(bms_opts),
                                         vp, vp, vp, ctypes.POINTER(bms_stats)]
        L.bms_action_noalloc.argtypes = [vp, i, i, d, dp, vp, vp, dp]
        L.bms_force.argtypes = [vp, i, i, dp, vp, vp, i]
        L.bms_timing_enable.argtypes = [vp, i]
        L.bms_set_variant.argtypes = [vp, i, i]
        L.bms_timing_read.argtypes = [vp, i, dp, ctypes.POINTER(ctypes.c_longlong), dp]
        L.bms_timing_flops.argtypes = [vp, i, dp, dp]
        L.bms_timing_floor.argtypes = [vp, i, d, d, d, dp]
        L.bms_set_link_rows.argtypes = [vp, i]
        L.bms_get_link_rows.argtypes = [vp, ip, dp]
        L.bms_get_variant.argtypes = [vp, i, ip]
        L.bms_set_hop_config.argtypes = [vp, i, ip]
        L.bms_get_hop_config.argtypes = [vp, i, ip]
        L.bms_set_tune_cache.argtypes = [vp, ctypes.c_char_p]
        L.bms_autotune.argtypes = [vp, d, i, i, dp, i, i, vp, vp]
        L.bms_solve_batch.argtypes = [i, ctypes.POINTER(vp), dp, ip, ip,
                                      ctypes.POINTER(dp), dp, ip, ctypes.POINTER(bms_opts),
                                      ctypes.POINTER(vp), ctypes.POINTER(vp),
                                      ctypes.POINTER(bms_stats), ip]
        for f in EXPORTS:
            if f not in ("bms_default_opts", "bms_error_string", "bms_last_error",
                         "bms_default_rhmc_params"):
                getattr(L, f).restype = ctypes.c_int
        _L = L
    return _L


def lib():
    """The loaded libbms.so (ctypes.CDLL)."""
    return _lib()


def _check(ctx, rc):
    if rc != 0:
        msg = _lib().bms_last_error(ctx).decode() if ctx else ""
        raise BmsError(rc, msg)


def _ptr(t):
    """Device pointer of a contiguous CUDA tensor, or an int address."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _doubles(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def bms_default_opts():
    o = bms_opts()
    _lib().bms_default_opts(ctypes.byref(o))
    return o


def bms_error_string(code):
    return _lib().bms_error_string(int(code)).decode()


def bms_create(dims, bc=(1, 1, 1, -1), stream=None):
    """Returns an opaque context handle (ctypes.c_void_p)."""
    h = ctypes.c_void_p()
    d = (ctypes.c_int * 4)(*[int(x) for x in dims])
    b = (ctypes.c_int * 4)(*[int(x) for x in bc])
    if stream is None:
        stream = 0
    rc = _lib().bms_create(ctypes.byref(h), d, b, ctypes.c_void_p(int(stream)))
    _check(None, rc)
    return h


def bms_destroy(ctx):
    _check(None, _lib().bms_destroy(ctx))


def bms_set_gauge(ctx, U):
    _check(ctx, _lib().bms_set_gauge(ctx, _ptr(U)))


def bms_set_gauge_improved(ctx, V, W):
    _check(ctx, _lib().bms_set_gauge_improved(ctx, _ptr(V), _ptr(W)))


def bms_apply_hop(ctx, parity_out, n, inp, out, precision=BMS_PREC_F64):
    _check(ctx, _lib().bms_apply_hop(ctx, int(parity_out), int(n), _ptr(inp), _ptr(out),
                                     int(precision)))


def bms_apply_mdagm(ctx, mass, sigma, n, inp, out, precision=BMS_PREC_F64):
    _check(ctx, _lib().bms_apply_mdagm(ctx, float(mass), float(sigma), int(n), _ptr(inp),
                                       _ptr(out), int(precision)))


def bms_solve(ctx, mass, n, shifts, tol, max_iter, opts, B, X, want_residuals=True,
              raise_on_error=True):
    """Returns (status, stats dict). X is written in place."""
    ns = len(shifts)
    st = bms_stats()
    res = (ctypes.c_double * (ns * n))() if want_residuals else None
    if res is not None:
        st.true_residual = ctypes.cast(res, ctypes.POINTER(ctypes.c_double))
    rc = _lib().bms_solve(ctx, float(mass), int(n), ns, _doubles(shifts), float(tol),
                          int(max_iter), ctypes.byref(opts) if opts is not None else None,
                          _ptr(B), _ptr(X), ctypes.byref(st))
    stats = _stats_dict(st)
    stats["status"] = rc
    if res is not None:
        stats["true_residual"] = [[res[s * n + i] for i in range(n)] for s in range(ns)]
    if raise_on_error:
        _check(ctx, rc)
    return rc, stats


def bms_rational_apply(ctx, mass, n, a0, alpha, shifts, tol, max_iter, opts, B, X, out,
                       raise_on_error=True):
    """out = a0 B + sum_j alpha_j (A + shifts_j)^-1 B; X receives the solutions.
    Returns (status, stats dict)."""
    ns = len(shifts)
    st = bms_stats()
    res = (ctypes.c_double * (ns * n))()
    st.true_residual = ctypes.cast(res, ctypes.POINTER(ctypes.c_double))
    rc = _lib().bms_rational_apply(ctx, float(mass), int(n), ns, float(a0), _doubles(alpha),
                                   _doubles(shifts), float(tol), int(max_iter),
                                   ctypes.byref(opts) if opts is not None else None, _ptr(B),
                                   _ptr(X), _ptr(out), ctypes.byref(st))
    stats = _stats_dict(st)
    stats["status"] = rc
    stats["true_residual"] = [[res[s * n + i] for i in range(n)] for s in range(ns)]
    if raise_on_error:
        _check(ctx, rc)
    return rc, stats


def bms_action(ctx, n, a0, alpha, B, X):
    S = (ctypes.c_double * n)()
    ns = len(alpha)
    _check(ctx, _lib().bms_action(ctx, int(n), ns, float(a0), _doubles(alpha), _ptr(B), _ptr(X),
                                  S))
    return [S[i] for i in range(n)]


def bms_action_noalloc(ctx, n, a0, alpha, B, X):
    S = (ctypes.c_double * n)()
    ns = len(alpha)
    _check(ctx, _lib().bms_action_noalloc(ctx, int(n), ns, float(a0), _doubles(alpha), _ptr(B),
                                          _ptr(X), S))
    return [S[i] for i in range(n)]


def bms_force(ctx, n, alpha, X, out, flags=BMS_FORCE_RAW):
    _check(ctx, _lib().bms_force(ctx, int(n), len(alpha), _doubles(alpha), _ptr(X), _ptr(out),
                                 int(flags)))


def bms_timing_enable(ctx, enable=True):
    _check(ctx, _lib().bms_timing_enable(ctx, 1 if enable else 0))


def bms_set_variant(ctx, kernel, variant):
    _check(ctx, _lib().bms_set_variant(ctx, int(kernel), int(variant)))


def bms_get_variant(ctx, kernel):
    v = ctypes.c_int()
    _check(ctx, _lib().bms_get_variant(ctx, int(kernel), ctypes.byref(v)))
    return v.value


def bms_set_hop_config(ctx, precision, cfg):
    """cfg = (ty, tz, tt, cap, nt), or None for the built-in choice."""
    arr = (ctypes.c_int * 5)(*(cfg if cfg is not None else (-1, 0, 0, 0, 0)))
    _check(ctx, _lib().bms_set_hop_config(ctx, int(precision), arr))


def bms_get_hop_config(ctx, precision):
    arr = (ctypes.c_int * 5)()
    _check(ctx, _lib().bms_get_hop_config(ctx, int(precision), arr))
    return tuple(arr)


def bms_set_tune_cache(ctx, path):
    _check(ctx, _lib().bms_set_tune_cache(ctx, path.encode() if path else None))


def bms_autotune(ctx, mass, n, shifts, precision, iters, B, X):
    _check(ctx, _lib().bms_autotune(ctx, float(mass), int(n), len(shifts), _doubles(shifts),
                                    int(precision), int(iters), _ptr(B), _ptr(X)))


def bms_solve_batch(ctxs, masses, ns, shifts, tols, max_iters, opts, Bs, Xs, raise_on_error=True):
    """Independent solves run concurrently, problem i on context ctxs[i].
    Returns (status, [per-problem status], [per-problem stats dict])."""
    k = len(ctxs)
    vp = ctypes.c_void_p
    sh = [_doubles(s) for s in shifts]
    st = (bms_stats * k)()
    res = [(ctypes.c_double * (len(shifts[i]) * ns[i]))() for i in range(k)]
    for i in range(k):
        st[i].true_residual = ctypes.cast(res[i], ctypes.POINTER(ctypes.c_double))
    op = (bms_opts * k)()
    for i in range(k):
        op[i] = opts[i] if opts is not None else bms_default_opts()
    status = (ctypes.c_int * k)()
    rc = _lib().bms_solve_batch(
        k, (vp * k)(*[c.value for c in ctxs]), (ctypes.c_double * k)(*map(float, masses)),
        (ctypes.c_int * k)(*ns), (ctypes.c_int * k)(*[len(s) for s in shifts]),
        (ctypes.POINTER(ctypes.c_double) * k)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
                                                for a in sh]),
        (ctypes.c_double * k)(*map(float, tols)), (ctypes.c_int * k)(*max_iters), op,
        (vp * k)(*[_ptr(b).value for b in Bs]), (vp * k)(*[_ptr(x).value for x in Xs]), st, status)
    stats = []
    for i in range(k):
        nsh, n = len(shifts[i]), ns[i]
        d = _stats_dict(st[i])
        d["status"] = status[i]
        d["true_residual"] = [[res[i][s * n + j] for j in range(n)] for s in range(nsh)]
        stats.append(d)
    if raise_on_error and rc != 0:
        bad = next(i for i in range(k) if status[i] != 0)
        _check(ctxs[bad], status[bad])
    return rc, list(status), stats


def bms_timing_read(ctx, kernel):
    """Returns (milliseconds, launches, algorithmic bytes) accumulated for a kernel class."""
    ms, nl, by = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    _check(ctx, _lib().bms_timing_read(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(nl),
                                       ctypes.byref(by)))
    return ms.value, nl.value, by.value


def bms_timing_flops(ctx, kernel):
    """Returns (FP64 flops, FP32 flops) of matrix-core work accumulated for a kernel class."""
    f64, f32 = ctypes.c_double(), ctypes.c_double()
    _check(ctx, _lib().bms_timing_flops(ctx, int(kernel), ctypes.byref(f64), ctypes.byref(f32)))
    return f64.value, f32.value


def bms_timing_floor(ctx, kernel, hbm_bytes_per_s, f64_flops_per_s, f32_flops_per_s):
    """Least time (s) the recorded launches of a kernel class need at the given peaks."""
    t = ctypes.c_double()
    _check(ctx, _lib().bms_timing_floor(ctx, int(kernel), float(hbm_bytes_per_s),
                                        float(f64_flops_per_s), float(f32_flops_per_s),
                                        ctypes.byref(t)))
    return t.value


class Context:
    """Owns a bms_ctx; torch-tensor convenience wrappers over the C calls."""

    def __init__(self, dims, bc=(1, 1, 1, -1), stream=None):
        import torch
        self.dims = tuple(int(d) for d in dims)
        self.bc = tuple(int(b) for b in bc)
        self.vol = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.vh = self.vol // 2
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.h = bms_create(self.dims, self.bc, stream)

    def close(self):
        if self.h is not None:
            bms_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_gauge(self, U):
        import torch
        assert U.dtype == torch.complex128 and tuple(U.shape) == (4, self.vol, 3, 3)
        bms_set_gauge(self.h, U)

    def set_link_rows(self, rows):
        """2: the hop reads SU(3) links as two rows when the field allows (default); 3: all nine
        entries. Takes effect at the next set_gauge."""
        _check(self.h, _lib().bms_set_link_rows(self.h, int(rows)))

    def link_rows(self, with_deviation=False):
        """Rows per link the current links are read in (2 or 3); with_deviation: also the
        largest third-row deviation from SU(3) the last check found (-1: none ran)."""
        r, d = ctypes.c_int(), ctypes.c_double()
        _check(self.h, _lib().bms_get_link_rows(self.h, ctypes.byref(r), ctypes.byref(d)))
        return (r.value, d.value) if with_deviation else r.value

    def gauge_action(self, beta, U):
        S = ctypes.c_double()
        _check(self.h, _lib().bms_gauge_action(self.h, float(beta), _ptr(U), ctypes.byref(S)))
        return S.value

    def gauge_force(self, beta, U, P, scale=1.0):
        """P += scale * F (Wilson gauge force, su(3) components)."""
        _check(self.h, _lib().bms_gauge_force(self.h, float(beta), _ptr(U), _ptr(P), float(scale)))

    def gauge_update(self, eps, P, U):
        """U <- exp(i eps P^a T^a) U in place."""
        _check(self.h, _lib().bms_gauge_update(self.h, float(eps), _ptr(P), _ptr(U)))

    def kinetic_energy(self, P):
        K = ctypes.c_double()
        _check(self.h, _lib().bms_kinetic_energy(self.h, _ptr(P), ctypes.byref(K)))
        return K.value

    def set_gauge_improved(self, V, W):
        """One-hop links V and three-hop links W of the improved operator
        (coefficients folded in), both shaped like U."""
        import torch
        for F in (V, W):
            assert F.dtype == torch.complex128 and tuple(F.shape) == (4, self.vol, 3, 3)
        bms_set_gauge_improved(self.h, V, W)

    def _block(self, v, dtype):
        assert v.dtype == dtype and v.dim() == 3 and v.shape[0] == self.vh and v.shape[1] == 3, \
            "block must be [Vh][3][n] of %s" % dtype
        return v.shape[2]

    def apply_hop(self, parity_out, v, precision=BMS_PREC_F64):
        import torch
        dt = torch.complex128 if precision == BMS_PREC_F64 else torch.complex64
        n = self._block(v, dt)
        out = torch.empty_like(v)
        bms_apply_hop(self.h, parity_out, n, v, out, precision)
        return out

    def apply_mdagm(self, mass, sigma, v, precision=BMS_PREC_F64):
        import torch
        dt = torch.complex128 if precision == BMS_PREC_F64 else torch.complex64
        n = self._block(v, dt)
        out = torch.empty_like(v)
        bms_apply_mdagm(self.h, mass, sigma, n, v, out, precision)
        return out

    def solve(self, mass, shifts, B, tol=1e-10, max_iter=10000, opts=None, raise_on_error=True,
              **kw):
        import torch
        n = self._block(B, torch.complex128)
        if opts is None:
            opts = bms_default_opts()
        for k, v in kw.items():
            setattr(opts, k, v)
        X = torch.empty((len(shifts),) + tuple(B.shape), dtype=torch.complex128, device=B.device)
        rc, stats = bms_solve(self.h, mass, n, list(shifts), tol, max_iter, opts, B, X,
                              raise_on_error=raise_on_error)
        return X, stats

    def rational_apply(self, mass, r, B, tol=1e-10, max_iter=10000, opts=None,
                       raise_on_error=True, **kw):
        """r(A) B for a rational approximation r (a0, alpha, beta); returns
        (out, X, stats) with X the shifted solutions."""
        import torch
        n = self._block(B, torch.complex128)
        if opts is None:
            opts = bms_default_opts()
        for k, v in kw.items():
            setattr(opts, k, v)
        X = torch.empty((len(r.beta),) + tuple(B.shape), dtype=torch.complex128, device=B.device)
        out = torch.empty_like(B)
        _, stats = bms_rational_apply(self.h, mass, n, r.a0, list(r.alpha), list(r.beta), tol,
                                      max_iter, opts, B, X, out, raise_on_error=raise_on_error)
        return out, X, stats

    def action(self, a0, alpha, B, X):
        n = B.shape[2]
        return bms_action(self.h, n, a0, list(alpha), B, X)

    def set_variant(self, kernel, variant):
        bms_set_variant(self.h, kernel, variant)

    def get_variant(self, kernel):
        return bms_get_variant(self.h, kernel)

    def autotune(self, mass, shifts, B, precision=BMS_PREC_F64, iters=16):
        """Time the kernel variants on this problem and keep the fastest;
        returns {kernel name: chosen variant}."""
        import torch
        n = self._block(B, torch.complex128)
        X = torch.empty((len(shifts),) + tuple(B.shape), dtype=torch.complex128, device=B.device)
        bms_autotune(self.h, mass, n, list(shifts), precision, iters, B, X)
        out = {KERNEL_NAMES[k]: self.get_variant(k)
               for k in (BMS_KERNEL_HOP, BMS_KERNEL_GRAM, BMS_KERNEL_UPDATE)}
        out["hop_f64"] = bms_get_hop_config(self.h, BMS_PREC_F64)
        out["hop_f32"] = bms_get_hop_config(self.h, BMS_PREC_F32)
        return out

    def set_hop_config(self, precision, cfg):
        bms_set_hop_config(self.h, precision, cfg)

    def get_hop_config(self, precision):
        return bms_get_hop_config(self.h, precision)

    def set_tune_cache(self, path):
        bms_set_tune_cache(self.h, path)

    def timing(self, enable=True):
        bms_timing_enable(self.h, enable)

    def timing_read(self):
        return {KERNEL_NAMES[k]: bms_timing_read(self.h, k) for k in range(len(KERNEL_NAMES))}

    def timing_flops(self):
        return {KERNEL_NAMES[k]: bms_timing_flops(self.h, k) for k in range(len(KERNEL_NAMES))}

    def timing_floor(self, kernel, hbm_bytes_per_s, f64_flops_per_s, f32_flops_per_s):
        k = KERNEL_NAMES.index(kernel) if isinstance(kernel, str) else int(kernel)
        return bms_timing_floor(self.h, k, hbm_bytes_per_s, f64_flops_per_s, f32_flops_per_s)

    def force(self, alpha, X, flags=BMS_FORCE_RAW):
        import torch
        n = X.shape[3]
        if flags == BMS_FORCE_RAW:
            out = torch.empty((4, self.vol, 3, 3), dtype=torch.complex128, device=X.device)
        else:
            out = torch.empty((4, self.vol, 8), dtype=torch.float64, device=X.device)
        bms_force(self.h, n, list(alpha), X, out, flags)
        return out


def rhmc_trajectory(ctx, U, P, eta, beta, mass, r_hb=None, r_acc=None, r_md=None, tau=1.0,
                    n_steps=10, n_gauge=3, lam=1.0 / 6.0, tol_hb=1e-14, tol_md=1e-7,
                    precision_md=BMS_PREC_F64, max_iter=100000):
    """bms_rhmc_trajectory on a Context: U (links, in/out) and P (momenta,
    in/out) device tensors, eta the Gaussian block (None for pure gauge HMC);
    r_* the heatbath, action and force rational approximations. Returns the
    result as a dict."""
    p = bms_rhmc_params()
    _lib().bms_default_rhmc_params(ctypes.byref(p))
    p.beta, p.mass, p.tau = float(beta), float(mass), float(tau)
    p.n_steps, p.n_gauge, p.lambda_ = int(n_steps), int(n_gauge), float(lam)
    p.tol_hb, p.tol_md, p.precision_md, p.max_iter = float(tol_hb), float(tol_md), \
        int(precision_md), int(max_iter)
    keep = []
    if eta is None:
        p.n = 0
    else:
        p.n = int(eta.shape[2])
        for tag, r in (("hb", r_hb), ("acc", r_acc), ("md", r_md)):
            al, be = _doubles(r.alpha), _doubles(r.beta)
            keep += [al, be]
            setattr(p, "ns_" + tag, len(r.beta))
            setattr(p, "alpha_" + tag, ctypes.cast(al, _dp))
            setattr(p, "beta_" + tag, ctypes.cast(be, _dp))
            if tag != "md":
                setattr(p, "a0_" + tag, float(r.a0))
    res = bms_rhmc_result()
    rc = _lib().bms_rhmc_trajectory(ctx.h, ctypes.byref(p), _ptr(U), _ptr(P),
                                    _ptr(eta) if eta is not None else None, ctypes.byref(res))
    _check(ctx.h, rc)
    return {k: getattr(res, k) for k, _ in bms_rhmc_result._fields_}


def solve_batch(contexts, masses, shifts, Bs, tol=1e-10, max_iter=10000, opts=None,
                raise_on_error=True):
    """bms_solve_batch over Context objects: problem i solves
    (A_i + shifts[i][s]) X = Bs[i] on contexts[i]; all run concurrently.
    Returns ([X_i], [stats_i])."""
    import torch
    k = len(contexts)
    ns = [c._block(B, torch.complex128) for c, B in zip(contexts, Bs)]
    Xs = [torch.empty((len(shifts[i]),) + tuple(Bs[i].shape), dtype=torch.complex128,
                      device=Bs[i].device) for i in range(k)]
    tols = tol if isinstance(tol, (list, tuple)) else [tol] * k
    mits = max_iter if isinstance(max_iter, (list, tuple)) else [max_iter] * k
    ops = opts if (opts is None or isinstance(opts, (list, tuple))) else [opts] * k
    _, _, stats = bms_solve_batch([c.h for c in contexts], masses, ns, shifts, tols, mits, ops, Bs,
                                  Xs, raise_on_error=raise_on_error)
    return Xs, stats
