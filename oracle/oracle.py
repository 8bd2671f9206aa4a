"""Test infrastructure only: Python side of the plain FP64 CPU oracle.

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module. It wraps the C oracle (staggered.c: the staggered operator, CG,
multi-shift CG, force) and adds numpy routines:

  * solve_block     X^(s) = (A + s)^-1 B for every shift and column, by the
                    C multi-shift CG per column (the plain definition of what
                    the block solver must return).
  * sbcgrq          Algorithm 1 (SBCGrQ) in numpy, in the paper's order and
                    notation, using the C operator; used for iteration counts
                    and for the recurrences' invariants.
  * rational_apply  r(A) B = a0 B + sum_j a_j (A + b_j)^-1 B by plain CG per
                    shift and column (heatbath and accept-step solves).
  * action          S = sum_i phi_i^dag (a0 phi_i + sum_j a_j X_ij), eq. RA.
  * force           dS/dU from the C oracle (derivation in staggered.c).
  * dense_operator  the explicit matrix of A + sigma on a small lattice.

Block layout everywhere: B[cb][color][rhs] (complex128), X[shift][cb][color][rhs].
It shares no code with the HIP library; the seeded inputs come from
paper_1808_01829_amd.inputs, which holds no solver arithmetic.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        src = os.path.join(HERE, "staggered.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.c_void_p
        L.ora_dslash_half.argtypes = [ip, ip, dp, ctypes.c_int, dp, dp]
        L.ora_mdagm.argtypes = [ip, ip, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.ora_cg.argtypes = [ip, ip, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                             ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.ora_cg.restype = ctypes.c_int
        L.ora_mscg.argtypes = [ip, ip, dp, ctypes.c_double, ctypes.c_int, dp, dp, dp,
                               ctypes.c_double, ctypes.c_int, dp]
        L.ora_mscg.restype = ctypes.c_int
        L.ora_force.argtypes = [ip, ip, dp, ctypes.c_int, dp, dp, dp]
        L.ora_dslash_half_imp.argtypes = [ip, ip, dp, dp, ctypes.c_int, dp, dp]
        L.ora_mdagm_imp.argtypes = [ip, ip, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp]
        L.ora_cg_imp.argtypes = [ip, ip, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp,
                                 ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
        L.ora_cg_imp.restype = ctypes.c_int
        L.ora_mscg_imp.argtypes = [ip, ip, dp, dp, ctypes.c_double, ctypes.c_int, dp, dp, dp,
                                   ctypes.c_double, ctypes.c_int, dp]
        L.ora_mscg_imp.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _i4(a):
    return (ctypes.c_int * 4)(*[int(v) for v in a])


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def vol(dims):
    return int(np.prod(dims))


# ---- operator --------------------------------------------------------------

def dslash_half(dims, bc, U, par_out, v, W=None):
    """(D v) on sites of parity par_out; v is a half vector [Vh][3]. With W
    (three-hop links [mu][idx][3][3]) the improved operator, U then being the
    one-hop links."""
    U = _c(U)
    v = _c(v)
    out = np.empty_like(v)
    if W is None:
        lib().ora_dslash_half(_i4(dims), _i4(bc), _ptr(U), int(par_out), _ptr(v), _ptr(out))
    else:
        W = _c(W)
        lib().ora_dslash_half_imp(_i4(dims), _i4(bc), _ptr(U), _ptr(W), int(par_out), _ptr(v),
                                  _ptr(out))
    return out


def mdagm(dims, bc, U, mass, sigma, v, W=None):
    """(A + sigma) v, A = m^2 - D_eo D_oe; v is [Vh][3] or a block [Vh][3][n]."""
    U = _c(U)
    v = _c(v)
    if v.ndim == 3:
        return np.stack([mdagm(dims, bc, U, mass, sigma, v[..., j], W)
                         for j in range(v.shape[2])], axis=-1)
    out = np.empty_like(v)
    if W is None:
        lib().ora_mdagm(_i4(dims), _i4(bc), _ptr(U), float(mass), float(sigma), _ptr(v),
                        _ptr(out))
    else:
        W = _c(W)
        lib().ora_mdagm_imp(_i4(dims), _i4(bc), _ptr(U), _ptr(W), float(mass), float(sigma),
                            _ptr(v), _ptr(out))
    return out


def dense_operator(dims, bc, U, mass, sigma, W=None):
    """Explicit matrix of (A + sigma) on the 3*Vh-dimensional even-site space."""
    n = vol(dims) // 2 * 3
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        A[:, k] = mdagm(dims, bc, U, mass, sigma, e.reshape(-1, 3), W).reshape(-1)
    return A


# ---- solvers ---------------------------------------------------------------

def cg(dims, bc, U, mass, sigma, b, tol=1e-13, maxiter=100000, W=None):
    """Plain CG for one half vector. Returns (x, iterations, true relative residual)."""
    U = _c(U)
    b = _c(b)
    x = np.empty_like(b)
    tr = ctypes.c_double(0)
    if W is None:
        k = lib().ora_cg(_i4(dims), _i4(bc), _ptr(U), float(mass), float(sigma), _ptr(b), _ptr(x),
                         float(tol), int(maxiter), ctypes.byref(tr))
    else:
        W = _c(W)
        k = lib().ora_cg_imp(_i4(dims), _i4(bc), _ptr(U), _ptr(W), float(mass), float(sigma),
                             _ptr(b), _ptr(x), float(tol), int(maxiter), ctypes.byref(tr))
    return x, k, tr.value


def mscg(dims, bc, U, mass, shifts, b, tol=1e-13, maxiter=100000, W=None):
    """Multi-shift CG for one half vector and ascending shifts.

    Returns (x[nshift][Vh][3], iterations, true relative residual per shift)."""
    shifts = np.ascontiguousarray(shifts, dtype=np.float64)
    if np.any(np.diff(shifts) < 0):
        raise ValueError("shifts must be ascending")
    U = _c(U)
    b = _c(b)
    x = np.empty((len(shifts),) + b.shape, dtype=np.complex128)
    tr = np.zeros(len(shifts))
    if W is None:
        k = lib().ora_mscg(_i4(dims), _i4(bc), _ptr(U), float(mass), len(shifts), _ptr(shifts),
                           _ptr(b), _ptr(x), float(tol), int(maxiter), _ptr(tr))
    else:
        W = _c(W)
        k = lib().ora_mscg_imp(_i4(dims), _i4(bc), _ptr(U), _ptr(W), float(mass), len(shifts),
                               _ptr(shifts), _ptr(b), _ptr(x), float(tol), int(maxiter),
                               _ptr(tr))
    return x, k, tr


def solve_block(dims, bc, U, mass, shifts, B, tol=1e-13, maxiter=100000, W=None):
    """X[s] = (A + shifts[s])^-1 B for a block B[Vh][3][n], any shift order.

    Returns (X[nshift][Vh][3][n], true relative residual [nshift][n])."""
    shifts = np.asarray(shifts, dtype=np.float64)
    order = np.argsort(shifts, kind="stable")
    n = B.shape[2]
    X = np.empty((len(shifts),) + B.shape, dtype=np.complex128)
    res = np.empty((len(shifts), n))
    for j in range(n):
        x, _, tr = mscg(dims, bc, U, mass, shifts[order], B[..., j], tol, maxiter, W)
        X[order, ..., j] = x
        res[order, j] = tr
    return X, res


def true_residuals(dims, bc, U, mass, shifts, B, X, W=None):
    """|b_i - (A + s) x_i| / |b_i| for every shift s and column i (FP64)."""
    res = np.empty((len(shifts), B.shape[2]))
    bn = np.linalg.norm(B.reshape(-1, B.shape[2]), axis=0)
    for s, sig in enumerate(shifts):
        r = B - mdagm(dims, bc, U, mass, sig, X[s], W)
        res[s] = np.linalg.norm(r.reshape(-1, B.shape[2]), axis=0) / np.where(bn > 0, bn, 1)
    return res


def _qr_pos(V):
    """Thin QR with a real positive diagonal of R."""
    q, r = np.linalg.qr(V)
    d = np.diag(r).copy()
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1), 1)
    return q * ph[None, :], np.conj(ph)[:, None] * r


def sbcgrq(apply_a0, B, shifts, tol, maxiter=10000, freeze_tol=None):
    """Algorithm 1 (SBCGrQ) on flattened blocks, in the paper's notation.

    apply_a0(P) must return (A + sigma_0) P for an L x n block P, with
    sigma_0 = shifts[0] the smallest shift. The loop stops when every column of
    every shift has relative residual norm |delta^(s)_k e_i| / |delta_0 e_i|
    below tol, where delta^(s)_k = rho_k alpha_k^-1 alpha^(s)_k (the shifted
    residual is Q_k delta^(s)_k). A shift stops being updated once all its
    columns are below freeze_tol (default tol).

    Returns dict(X=[N_s][L][n], iters, history) where history[k][s] holds the
    per-column residual estimates after iteration k.
    """
    freeze_tol = tol if freeze_tol is None else freeze_tol
    shifts = np.asarray(shifts, dtype=np.float64)
    ns = len(shifts)
    if np.any(np.diff(shifts) < 0):
        raise ValueError("shifts must be ascending")
    L, n = B.shape
    eye = np.eye(n, dtype=np.complex128)
    X = np.zeros((ns, L, n), dtype=np.complex128)
    Q, delta = _qr_pos(B)
    delta0 = delta.copy()
    norm0 = np.linalg.norm(delta0, axis=0)
    P = np.stack([Q.copy() for _ in range(ns)])
    rho_prev = delta.copy()
    alpha_prev = eye.copy()
    alpha_s = [eye.copy() for _ in range(ns)]
    beta_s = [eye.copy() for _ in range(ns)]
    delta_s = [delta0.copy() for _ in range(ns)]
    active = np.ones(ns, dtype=bool)
    history = []
    k = 0
    while k < maxiter:
        rel = np.array([np.linalg.norm(d, axis=0) / norm0 for d in delta_s])
        history.append(rel)
        active &= ~(rel.max(axis=1) < freeze_tol)
        if rel.max() < tol or not active.any():
            break
        k += 1
        AP = apply_a0(P[0])
        alpha = np.linalg.inv(np.conj(P[0]).T @ AP)
        Q, rho = _qr_pos(Q - AP @ alpha)
        X[0] += P[0] @ (alpha @ delta)
        P[0] = Q + P[0] @ np.conj(rho).T
        delta = rho @ delta
        delta_s[0] = delta
        ainv = np.linalg.inv(alpha)
        for s in range(1, ns):
            if not active[s]:
                continue
            t = alpha @ rho_prev @ np.linalg.inv(alpha_prev)
            beta_new = np.linalg.inv(eye + (shifts[s] - shifts[0]) * alpha
                                     + t @ (eye - beta_s[s]) @ np.conj(rho_prev).T)
            alpha_new = beta_new @ t @ alpha_s[s]
            X[s] += P[s] @ alpha_new
            P[s] = Q + P[s] @ beta_new @ np.conj(rho).T
            beta_s[s] = beta_new
            alpha_s[s] = alpha_new
            delta_s[s] = rho @ ainv @ alpha_new
        rho_prev = rho
        alpha_prev = alpha
    return dict(X=X, iters=k, history=history, Q=Q, delta_s=delta_s)


def sbcgrq_lattice(dims, bc, U, mass, shifts, B, tol, maxiter=10000, freeze_tol=None):
    """sbcgrq on a lattice block B[Vh][3][n]; returns X[shift][Vh][3][n] etc."""
    shifts = np.asarray(shifts, dtype=np.float64)
    order = np.argsort(shifts, kind="stable")
    vh, _, n = B.shape
    U = _c(U)

    def a0(P):
        return mdagm(dims, bc, U, mass, shifts[order[0]], P.reshape(vh, 3, n)).reshape(-1, n)

    out = sbcgrq(a0, B.reshape(-1, n), shifts[order], tol, maxiter, freeze_tol)
    X = np.empty((len(shifts), vh, 3, n), dtype=np.complex128)
    X[order] = out["X"].reshape(len(shifts), vh, 3, n)
    out["X"] = X
    return out


# ---- action and force ------------------------------------------------------

def rational_apply(dims, bc, U, mass, a0, alpha, beta, B, tol=1e-14, maxiter=100000):
    """r(A) B = a0 B + sum_j alpha_j (A + beta_j)^-1 B (eq. RA applied to a
    block), every (A + beta_j)^-1 b_i by its own plain CG (no multi-shift
    recurrence). Used for the pseudofermion heatbath phi = r_hb(A) eta and
    the accept-step solves (Sec. II, Sec. IV). Returns (out, X[shift])."""
    B = _c(B)
    X = np.empty((len(beta),) + B.shape, dtype=np.complex128)
    for s, sig in enumerate(beta):
        for j in range(B.shape[2]):
            x, _, _ = cg(dims, bc, U, mass, float(sig), np.ascontiguousarray(B[..., j]), tol,
                         maxiter)
            X[s, ..., j] = x
    out = a0 * B + np.tensordot(np.asarray(alpha, dtype=np.float64), X, axes=(0, 0))
    return out, X


def action(B, X, a0, alpha):
    """Per-column S_i = Re phi_i^dag (a0 phi_i + sum_j a_j X_ij) (eq. RA applied
    to the pseudofermion action of Sec. II)."""
    acc = a0 * B + np.tensordot(np.asarray(alpha, dtype=np.float64), X, axes=(0, 0))
    return np.real(np.sum(np.conj(B) * acc, axis=(0, 1)))


def force(dims, bc, U, alpha, X):
    """G[mu][idx][a][b] = dS/dRe U + i dS/dIm U for S = sum_ij alpha_j phi_i^dag
    (A + s_j)^-1 phi_i, given the solutions X[j][Vh][3][n]."""
    U = _c(U)
    ns, vh, _, n = X.shape
    xv = np.ascontiguousarray(np.transpose(X, (0, 3, 1, 2)).reshape(ns * n, vh, 3))
    coef = np.ascontiguousarray(np.repeat(np.asarray(alpha, dtype=np.float64), n))
    g = np.empty((4, vol(dims), 3, 3), dtype=np.complex128)
    lib().ora_force(_i4(dims), _i4(bc), _ptr(U), ns * n, _ptr(coef), _ptr(xv), _ptr(g))
    return g


def lie_force(U, G):
    """F^a = -dS/d omega^a for U -> exp(i omega^a T^a) U: F^a = Im Tr[T^a U M]
    with M = G^dag. Returns [mu][idx][8]."""
    M = np.conj(np.swapaxes(G, -1, -2))
    UM = U @ M
    return np.imag(np.einsum("aij,...ji->...a", su3_generators(), UM))


def su3_generators():
    """T^a = lambda_a / 2 (Gell-Mann matrices), written out here."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l / 2
