"""Pins of the oracle's solvers (no GPU): CG and multi-shift CG against dense
numpy solves, Algorithm 1 (SBCGrQ) against the same, n_pf = 1 block CG equal
to multi-shift CG, the shifted-residual identity, covariance, and the exact
free-field solution."""
import numpy as np
import pytest

from oracle import freefield as F
from oracle import oracle as O
from paper_1808_01829_amd.inputs import (configs, gaussian_block, random_gauge,
                                         random_gauge_transform, unit_gauge)

from test_oracle_operator import _gauge_transform_links, _parity_sites

BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def small():
    dims = (4, 4, 4, 4)
    r = configs.workload_coefficients("c2")
    U = random_gauge(dims, 0.5, 2000)
    B = gaussian_block(dims, 4, 2001)
    return dims, U, B, 0.05, r


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_cg_matches_dense(dims):
    U = random_gauge(dims, 0.9, 9)
    b = gaussian_block(dims, 1, 10)[..., 0]
    for sigma in (0.0, 0.5):
        A = O.dense_operator(dims, BC, U, 0.1, sigma)
        xd = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
        x, k, tr = O.cg(dims, BC, U, 0.1, sigma, b, 1e-14)
        assert tr < 1e-13
        assert np.abs(x - xd).max() < 1e-12 * np.abs(xd).max()


def test_mscg_matches_dense_and_cg(small):
    dims, U, B, m, r = small
    X, res = O.solve_block(dims, BC, U, m, r.beta, B, 1e-13)
    assert res.max() < 1e-12
    for s in (0, len(r.beta) // 2, len(r.beta) - 1):
        A = O.dense_operator(dims, BC, U, m, r.beta[s])
        xd = np.linalg.solve(A, B.reshape(-1, B.shape[2])).reshape(B.shape)
        assert np.abs(X[s] - xd).max() < 1e-11 * np.abs(xd).max()
        x, _, _ = O.cg(dims, BC, U, m, r.beta[s], B[..., 1], 1e-13)
        assert np.abs(X[s][..., 1] - x).max() < 1e-11 * np.abs(x).max()


def test_mscg_unsorted_shift_order(small):
    dims, U, B, m, r = small
    perm = np.random.default_rng(0).permutation(len(r.beta))
    X1, _ = O.solve_block(dims, BC, U, m, r.beta, B[..., :1], 1e-13)
    X2, _ = O.solve_block(dims, BC, U, m, r.beta[perm], B[..., :1], 1e-13)
    assert np.abs(X1[perm] - X2).max() < 1e-13 * np.abs(X1).max()


def test_sbcgrq_matches_definition(small):
    dims, U, B, m, r = small
    out = O.sbcgrq_lattice(dims, BC, U, m, r.beta, B, 1e-12)
    tr = O.true_residuals(dims, BC, U, m, r.beta, B, out["X"])
    assert tr.max() < 5e-12
    for s in (0, len(r.beta) - 1):
        A = O.dense_operator(dims, BC, U, m, r.beta[s])
        xd = np.linalg.solve(A, B.reshape(-1, B.shape[2])).reshape(B.shape)
        assert np.abs(out["X"][s] - xd).max() < 1e-9 * np.abs(xd).max()


def test_sbcgrq_shifted_residual_identity(small):
    # the residual of shift s after k steps is Q_k delta^(s)_k
    dims, U, B, m, r = small
    out = O.sbcgrq_lattice(dims, BC, U, m, r.beta, B, 1e-6, freeze_tol=0.0)
    Q = out["Q"].reshape(B.shape)
    for s in range(len(r.beta)):
        R = B - O.mdagm(dims, BC, U, m, r.beta[s], out["X"][s])
        Rq = np.einsum("vcj,ji->vci", Q, out["delta_s"][s])
        assert np.abs(R - Rq).max() < 1e-10 * np.abs(B).max()


def test_sbcgrq_npf1_equals_multishift_cg(small):
    # Sec. III: block CG reduces to CG (and SBCGrQ to multi-shift CG) at n_pf = 1
    dims, U, B, m, r = small
    b = B[..., :1]
    o1 = O.sbcgrq_lattice(dims, BC, U, m, r.beta, b, 1e-10)
    x1, k1, _ = O.mscg(dims, BC, U, m, r.beta, b[..., 0], 1e-10)
    assert o1["iters"] == k1
    assert np.abs(o1["X"][..., 0] - x1).max() < 1e-10 * np.abs(x1).max()


def test_sbcgrq_single_shift_is_bcgrq(small):
    dims, U, B, m, r = small
    o = O.sbcgrq_lattice(dims, BC, U, m, r.beta[:1], B, 1e-11)
    A = O.dense_operator(dims, BC, U, m, r.beta[0])
    xd = np.linalg.solve(A, B.reshape(-1, 4)).reshape(B.shape)
    assert np.abs(o["X"][0] - xd).max() < 1e-8 * np.abs(xd).max()


def test_block_iterations_fall_with_npf(small):
    # eq. convergence_bound: the rate is set by lambda_{n_pf}, so more columns, fewer steps
    dims, U, B, m, r = small
    its = [O.sbcgrq_lattice(dims, BC, U, m, r.beta, B[..., :n], 1e-10)["iters"] for n in (1, 2, 4)]
    assert its[0] > its[1] > its[2]


def test_duplicate_shift_reproduces_unshifted(small):
    dims, U, B, m, r = small
    sh = np.concatenate([r.beta[:1], r.beta[:1], r.beta[1:3]])
    o = O.sbcgrq_lattice(dims, BC, U, m, sh, B, 1e-11)
    assert np.abs(o["X"][0] - o["X"][1]).max() < 1e-9 * np.abs(o["X"][0]).max()


def test_solution_covariance():
    dims = (4, 4, 2, 4)
    U = random_gauge(dims, 0.7, 31)
    g = random_gauge_transform(dims, 32)
    Ug = _gauge_transform_links(dims, U, g)
    ge = g[_parity_sites(dims, 0)]
    B = gaussian_block(dims, 2, 33)
    gB = np.einsum("sab,sbj->saj", ge, B)
    sh = [0.01, 0.3]
    X, _ = O.solve_block(dims, BC, U, 0.1, sh, B, 1e-13)
    Xg, _ = O.solve_block(dims, BC, Ug, 0.1, sh, gB, 1e-13)
    assert np.abs(Xg - np.einsum("sab,ksbj->ksaj", ge, X)).max() < 1e-11 * np.abs(X).max()


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (1, 1, 1, -1)])
def test_free_field_block_solve(bc):
    dims = (4, 4, 4, 6)
    B = gaussian_block(dims, 3, 41)
    sh = [0.001, 0.2, 3.0]
    o = O.sbcgrq_lattice(dims, bc, unit_gauge(dims), 0.1, sh, B, 1e-12)
    for s, sig in enumerate(sh):
        xf = F.solve(dims, bc, 0.1, sig, B)
        assert np.abs(o["X"][s] - xf).max() < 1e-9 * np.abs(xf).max()


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_action_equals_spectral_rational(name):
    """S_i = phi_i^dag r(A) phi_i (eq. RA in the action of Sec. II) from the
    eigendecomposition of the dense A on 2^4, and r(A) phi close to A^-p phi
    within the fit's relative error: pins action() and the coefficients
    without the oracle's own solvers."""
    dims = (2, 2, 2, 2)
    w = configs.WORKLOADS[name]
    r = configs.workload_coefficients(name)
    m = w["mass"]
    U = random_gauge(dims, w["eps"], 77)
    B = gaussian_block(dims, 3, 78)
    A = O.dense_operator(dims, BC, U, m, 0.0)
    lam, V = np.linalg.eigh(A)
    assert lam.min() > m * m * (1 - 1e-12) and lam.max() < 16 + m * m
    rl = r.a0 + sum(a / (lam + b) for a, b in zip(r.alpha, r.beta))
    Bf = B.reshape(-1, B.shape[-1])
    C = np.conj(V).T @ Bf
    S_spec = np.real(np.sum(np.conj(C) * (rl[:, None] * C), axis=0))
    X, _ = O.solve_block(dims, BC, U, m, r.beta, B, 1e-14)
    S = O.action(B, X, r.a0, r.alpha)
    assert np.allclose(S, S_spec, rtol=1e-11, atol=0)
    # the rational function approximates x^-p to its stated relative error
    exact = lam ** (-w["power"])
    assert np.max(np.abs(rl / exact - 1)) <= 1.01 * r.error
    S_exact = np.real(np.sum(np.conj(C) * (exact[:, None] * C), axis=0))
    assert np.all(np.abs(S / S_exact - 1) <= 1.01 * r.error)
