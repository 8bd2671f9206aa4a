"""Pins of the oracle's improved (less local) staggered operator: one-hop
links V and three-hop links W (the paper's outlook, Sec. V, expects such an
operator to gain more from reading each link once per block). CPU only.

* the free spectrum m^2 + sum (c1 sin p + c3 sin 3p)^2 at V = c1, W = c3
  (Naik coefficients 9/8 and -1/24), dense, both boundary conditions,
  lattices with extents 4 (where three hops wrap onto one) and 6;
* W = 0 is the unimproved operator; D_eo = -D_oe^dag; A >= m^2;
* gauge covariance with V_mu(x) -> g(x) V g(x+mu)^dag and
  W_mu(x) -> g(x) W g(x+3mu)^dag;
* the oracle's CG on the improved operator against the FFT exact solve;
* a three-hop boundary factor taken from the first step only (a plausible
  mistake) is caught by the antiperiodic free spectrum.
"""
import os
import subprocess
import importlib.util

import numpy as np
import pytest

from oracle import freefield as F
from oracle import oracle as O
from paper_1808_01829_amd.inputs import gaussian_block, random_gauge, unit_gauge

C1, C3 = 9.0 / 8.0, -1.0 / 24.0
BCS = [(1, 1, 1, 1), (1, 1, 1, -1)]


def naik_free(dims):
    U = unit_gauge(dims)
    return C1 * U, C3 * U


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 4, 6)])
@pytest.mark.parametrize("bc", BCS)
def test_improved_free_spectrum(dims, bc):
    m = 0.1
    V, W = naik_free(dims)
    ev = np.sort(np.linalg.eigvalsh(O.dense_operator(dims, bc, V, m, 0.0, W)))
    ref = F.spectrum(dims, bc, m, C1, C3)
    assert np.abs(ev - ref).max() < 1e-12
    # and not the unimproved spectrum
    assert np.abs(ev - F.spectrum(dims, bc, m)).max() > 1e-3


def test_improved_reduces_and_is_antihermitian():
    dims, bc = (4, 4, 2, 6), (1, 1, 1, -1)
    V, W = random_gauge(dims, 0.7, 11), random_gauge(dims, 0.7, 12)
    b = gaussian_block(dims, 1, 13)[..., 0]
    assert np.array_equal(O.mdagm(dims, bc, V, 0.1, 0.0, b, np.zeros_like(W)),
                          O.mdagm(dims, bc, V, 0.1, 0.0, b))
    vh = int(np.prod(dims)) // 2
    n = 3 * vh
    Doe = np.empty((n, n), dtype=complex)
    Deo = np.empty((n, n), dtype=complex)
    e = np.zeros(n, dtype=complex)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        Doe[:, k] = O.dslash_half(dims, bc, V, 1, e.reshape(-1, 3), W).reshape(-1)
        Deo[:, k] = O.dslash_half(dims, bc, V, 0, e.reshape(-1, 3), W).reshape(-1)
    assert np.abs(Deo + Doe.conj().T).max() < 1e-14
    A = O.dense_operator(dims, bc, V, 0.2, 0.0, W)
    assert np.abs(A - A.conj().T).max() < 1e-13
    assert np.linalg.eigvalsh(A).min() >= 0.04 - 1e-12


def _gauge_transform(dims, U, g, hops):
    """U_mu(x) -> g(x) U_mu(x) g(x + hops mu)^dag, lexicographic sites."""
    L = dims
    out = np.empty_like(U)
    V = int(np.prod(dims))
    for idx in range(V):
        c = [idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2],
             idx // (L[0] * L[1] * L[2])]
        for mu in range(4):
            cn = list(c)
            cn[mu] = (cn[mu] + hops) % L[mu]
            jn = cn[0] + L[0] * (cn[1] + L[1] * (cn[2] + L[2] * cn[3]))
            out[mu, idx] = g[idx] @ U[mu, idx] @ g[jn].conj().T
    return out


def test_improved_gauge_covariance():
    dims, bc = (4, 4, 4, 6), (1, 1, 1, -1)
    V, W = random_gauge(dims, 0.7, 21), random_gauge(dims, 0.7, 22)
    g = random_gauge(dims, 1.0, 23)[0]  # one SU(3) matrix per site
    Vg, Wg = _gauge_transform(dims, V, g, 1), _gauge_transform(dims, W, g, 3)
    b = gaussian_block(dims, 1, 24)[..., 0]
    # g on even sites in checkerboard order
    idx_even = [i for i in range(int(np.prod(dims)))
                if (i % dims[0] + (i // dims[0]) % dims[1] + (i // (dims[0] * dims[1])) % dims[2]
                    + i // (dims[0] * dims[1] * dims[2])) % 2 == 0]
    ge = g[idx_even]
    lhs = O.mdagm(dims, bc, Vg, 0.1, 0.3, np.einsum("sab,sb->sa", ge, b), Wg)
    rhs = np.einsum("sab,sb->sa", ge, O.mdagm(dims, bc, V, 0.1, 0.3, b, W))
    assert np.abs(lhs - rhs).max() < 1e-13


@pytest.mark.parametrize("bc", BCS)
def test_improved_cg_equals_fft_solve(bc):
    dims = (8, 8, 4, 8)
    V, W = naik_free(dims)
    b = gaussian_block(dims, 2, 31)
    for sig in (0.0, 0.5):
        x = np.stack([O.cg(dims, bc, V, 0.05, sig, b[..., j], 1e-13, W=W)[0] for j in range(2)],
                     axis=-1)
        xf = F.solve(dims, bc, 0.05, sig, b, C1, C3)
        assert np.linalg.norm(x - xf) <= 1e-10 * np.linalg.norm(xf)
    # multi-shift CG on the improved operator agrees with its plain CG
    xs, _, _ = O.mscg(dims, bc, V, 0.05, [0.0, 0.5], b[..., 0], 1e-13, W=W)
    assert np.linalg.norm(xs[1] - F.solve(dims, bc, 0.05, 0.5, b[..., 0], C1, C3)) <= \
        1e-10 * np.linalg.norm(xs[1])


def test_planted_three_hop_boundary_factor_is_caught(tmp_path):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, "oracle", "staggered.c")).read()
    old = "acc[a] = c_add(acc[a], c_scale(t, e * b3));"
    assert src.count(old) == 1
    d = tmp_path / "mut"
    d.mkdir()
    # the forward three-hop takes the boundary factor of a single hop instead
    (d / "staggered.c").write_text(src.replace(
        old, "acc[a] = c_add(acc[a], c_scale(t, e * (c[mu] == dims[mu] - 1 ? bc[mu] : 1)));"))
    so = d / "liboracle.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-o",
                           str(so), str(d / "staggered.c"), "-lm"])
    spec = importlib.util.spec_from_file_location("oracle_mut_imp",
                                                  os.path.join(root, "oracle", "oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.HERE = str(d)
    dims, bc = (4, 4, 4, 6), (1, 1, 1, -1)
    V, W = naik_free(dims)
    ev = np.sort(np.linalg.eigvalsh(mod.dense_operator(dims, bc, V, 0.1, 0.0, W)))
    assert np.abs(ev - F.spectrum(dims, bc, 0.1, C1, C3)).max() > 1e-6
