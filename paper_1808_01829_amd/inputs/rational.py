"""Rational approximation coefficients for r(x) ~ x^(-p) (inputs to the solver).

The paper replaces fractional powers of M^dag M by the partial-fraction form of
eq. RA, r(x) = a0 + sum_j a_j / (x + b_j) with a_j, b_j > 0 (Sec. II), but does
not say how the coefficients are obtained. Here they are the best type (N, N)
rational approximation in the relative-error sense on [lo, hi], found with the
classical rational Remez exchange carried out in high precision (mpmath):

  1. On 2N+2 reference points x_i solve the linear system
        p(x_i) - f_i q(x_i) - (-1)^i E f_i q_prev(x_i) = 0,  q(0) = 1,
     for the numerator p, denominator q (both degree N) and level E,
     iterating q_prev -> q until E settles.
  2. Move the reference to the 2N+2 alternating extrema of r/f - 1.
  3. Stop when the extrema all have |error| equal to within a small fraction.

Then a0 = p_N/q_N and the poles -b_j are the (real, negative) roots of q with
residues a_j = p(-b_j)/q'(-b_j). Coefficients are cached per argument set.

This is input generation only; none of the Krylov solver's arithmetic is here.
"""
import functools
import math

import mpmath as mp
import numpy as np


class RationalApprox:
    """r(x) = a0 + sum_j alpha[j] / (x + beta[j]) approximating x^(-power)."""

    def __init__(self, power, lo, hi, a0, alpha, beta, error):
        self.power = power
        self.lo = lo
        self.hi = hi
        self.a0 = float(a0)
        self.alpha = np.asarray(alpha, dtype=np.float64)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.error = float(error)

    @property
    def n_poles(self):
        return len(self.beta)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self.a0 + np.sum(self.alpha / (x[..., None] + self.beta), axis=-1)

    def rel_error(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self(x) * x ** self.power - 1.0

    def as_dict(self):
        return dict(power=self.power, lo=self.lo, hi=self.hi, a0=self.a0,
                    alpha=self.alpha.tolist(), beta=self.beta.tolist(), error=self.error)


def _polyval(c, x):
    s = mp.mpf(0)
    for ck in reversed(c):
        s = s * x + ck
    return s


def _solve_level(xs, fs, n, qprev):
    """One linear solve of the reference equations for (p, q_1..q_n, E)."""
    m = 2 * n + 2
    a = mp.matrix(m, m)
    rhs = mp.matrix(m, 1)
    for i, (x, f) in enumerate(zip(xs, fs)):
        xp = mp.mpf(1)
        for k in range(n + 1):
            a[i, k] = xp
            xp *= x
        xp = x
        for k in range(1, n + 1):
            a[i, n + k] = -f * xp
            xp *= x
        sgn = 1 if i % 2 == 0 else -1
        a[i, 2 * n + 1] = -sgn * f * _polyval(qprev, x)
        rhs[i] = f
    sol = mp.lu_solve(a, rhs)
    p = [sol[k] for k in range(n + 1)]
    q = [mp.mpf(1)] + [sol[n + k] for k in range(1, n + 1)]
    return p, q, sol[2 * n + 1]


def _err(p, q, power, x):
    return _polyval(p, x) / _polyval(q, x) * x ** power - 1


def _extrema(p, q, power, lo, hi, npts):
    """Alternating extrema of the relative error on [lo, hi] (log-spaced scan
    plus golden-section refinement of each interior extremum)."""
    lg = [mp.log(lo) + (mp.log(hi) - mp.log(lo)) * k / (npts - 1) for k in range(npts)]
    xs = [mp.e ** t for t in lg]
    xs[0], xs[-1] = lo, hi
    es = [_err(p, q, power, x) for x in xs]
    cand = [0]
    for k in range(1, npts - 1):
        if (es[k] - es[k - 1]) * (es[k + 1] - es[k]) <= 0:
            cand.append(k)
    cand.append(npts - 1)
    pts = []
    for k in cand:
        if k in (0, npts - 1):
            pts.append((xs[k], es[k]))
            continue
        sgn = 1 if es[k] > 0 else -1
        a, b = lg[k - 1], lg[k + 1]
        g = (mp.sqrt(5) - 1) / 2
        c1 = b - g * (b - a)
        c2 = a + g * (b - a)
        f1 = sgn * _err(p, q, power, mp.e ** c1)
        f2 = sgn * _err(p, q, power, mp.e ** c2)
        for _ in range(40):
            if f1 > f2:
                b, c2, f2 = c2, c1, f1
                c1 = b - g * (b - a)
                f1 = sgn * _err(p, q, power, mp.e ** c1)
            else:
                a, c1, f1 = c1, c2, f2
                c2 = a + g * (b - a)
                f2 = sgn * _err(p, q, power, mp.e ** c2)
        xm = mp.e ** ((a + b) / 2)
        pts.append((xm, _err(p, q, power, xm)))
    # merge runs of equal sign keeping the largest magnitude
    alt = []
    for x, e in pts:
        if alt and (alt[-1][1] > 0) == (e > 0):
            if abs(e) > abs(alt[-1][1]):
                alt[-1] = (x, e)
        else:
            alt.append((x, e))
    return alt


def _pick(alt, m):
    """Choose m alternating points, dropping the smaller end while too many."""
    alt = list(alt)
    while len(alt) > m:
        if abs(alt[0][1]) < abs(alt[-1][1]):
            alt.pop(0)
        else:
            alt.pop()
    return alt


@functools.lru_cache(maxsize=64)
def remez(power, lo, hi, n, dps=None, max_iter=40, rtol=1e-4):
    """Best relative-error type (n, n) approximation of x^(-power) on [lo, hi]."""
    if not (lo > 0 and hi > lo and n >= 1):
        raise ValueError("need 0 < lo < hi and n >= 1")
    ratio = hi / lo
    if dps is None:
        dps = int(40 + 2 * n * math.log10(ratio))
    with mp.workdps(dps):
        plo = mp.mpf(lo) / mp.mpf(hi)  # work on s = x/hi in [plo, 1]
        phi = mp.mpf(1)
        pw = mp.mpf(power)
        m = 2 * n + 2
        # initial reference: Chebyshev-like points in log x
        xs = [plo * (phi / plo) ** ((1 - mp.cos(mp.pi * i / (m - 1))) / 2) for i in range(m)]
        q = [mp.mpf(1)] + [mp.mpf(0)] * n
        level = None
        npts = max(400, 60 * m)
        for _ in range(max_iter):
            fs = [x ** (-pw) for x in xs]
            for _inner in range(30):
                p, q, e_new = _solve_level(xs, fs, n, q)
                if level is not None and abs(e_new - level) <= abs(e_new) * mp.mpf(10) ** (-dps // 3):
                    level = e_new
                    break
                level = e_new
            alt = _extrema(p, q, pw, plo, phi, npts)
            if len(alt) < m:
                raise RuntimeError("Remez: lost alternation (%d < %d points)" % (len(alt), m))
            alt = _pick(alt, m)
            mags = [abs(e) for _, e in alt]
            emax, emin = max(mags), min(mags)
            xs = [x for x, _ in alt]
            if emax - emin <= rtol * emax:
                break
        else:
            raise RuntimeError("Remez did not converge")
        # partial fractions on the scaled variable, then undo the scaling
        qc = list(reversed(q))  # highest degree first for polyroots
        roots = mp.polyroots(qc, maxsteps=400, extraprec=4 * dps)
        betas, alphas = [], []
        dq = [k * q[k] for k in range(1, n + 1)]
        for r in roots:
            if abs(mp.im(r)) > mp.mpf(10) ** (-dps // 4) * (1 + abs(r)):
                raise RuntimeError("Remez: complex pole")
            r = mp.re(r)
            betas.append(-r)
            alphas.append(_polyval(p, r) / _polyval(dq, r))
        a0 = p[n] / q[n]
        scale = mp.mpf(hi) ** (-pw)
        order = sorted(range(n), key=lambda j: betas[j])
        beta = [float(betas[j] * hi) for j in order]
        alpha = [float(alphas[j] * hi * scale) for j in order]
        return RationalApprox(power, lo, hi, float(a0 * scale), alpha, beta, float(emax))


def zolotarev_inv_sqrt(lo, hi, n):
    """Zolotarev's optimal relative-error approximation of x^(-1/2) on [lo, hi]
    as a product form, returned as a callable and its max relative error.

    With k' = sqrt(1 - lo/hi), K = K(k'^2) and c_l = sn^2/cn^2 (l K/(2n+1); k'^2)
    the function  x -> prod_l (x/lo + c_{2l}) / (x/lo + c_{2l-1})  (times a
    constant) equioscillates in relative error on [lo, hi]; the constant is
    fixed here so that the error is centred. Used only as an independent check
    of the Remez routine.
    """
    from scipy.special import ellipj, ellipk

    m = 1.0 - lo / hi
    kk = ellipk(m)
    cs = []
    for l in range(1, 2 * n + 1):
        sn, cn, _, _ = ellipj(l * kk / (2 * n + 1), m)
        cs.append(sn * sn / (cn * cn))

    def base(x):
        t = np.asarray(x, dtype=np.float64) / lo
        r = np.ones_like(t)
        for l in range(n):
            r = r * (t + cs[2 * l + 1]) / (t + cs[2 * l])
        return r

    xs = np.exp(np.linspace(np.log(lo), np.log(hi), 200001))
    g = base(xs) * np.sqrt(xs)
    gmin, gmax = g.min(), g.max()
    d = 2.0 / (gmin + gmax)
    err = (gmax - gmin) / (gmax + gmin)
    return (lambda x: d * base(x)), err
