"""Pins of the oracle force (no GPU): central finite differences of the action
in random complex link directions and in su(3) directions, gauge covariance of
the gradient and gauge invariance of the action."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oracle as O
from paper_1808_01829_amd.inputs import (configs, gaussian_block, random_gauge,
                                         random_gauge_transform)

from test_oracle_operator import _gauge_transform_links, _parity_sites

BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def setup():
    dims = (4, 4, 2, 4)
    r = configs.workload_coefficients("c1")
    U = random_gauge(dims, 0.5, 7)
    B = gaussian_block(dims, 2, 8)
    m = 0.1

    def S(Uv):
        X, _ = O.solve_block(dims, BC, Uv, m, r.beta, B, 1e-14)
        return O.action(B, X, r.a0, r.alpha).sum()

    X, _ = O.solve_block(dims, BC, U, m, r.beta, B, 1e-14)
    G = O.force(dims, BC, U, r.alpha, X)
    return dims, r, U, B, m, S, G, X


def test_force_finite_differences_complex(setup):
    dims, r, U, B, m, S, G, X = setup
    rng = np.random.default_rng(1)
    eps = 1e-5
    for _ in range(24):
        mu, idx = rng.integers(4), rng.integers(int(np.prod(dims)))
        dU = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Up, Um = U.copy(), U.copy()
        Up[mu, idx] += eps * dU
        Um[mu, idx] -= eps * dU
        fd = (S(Up) - S(Um)) / (2 * eps)
        an = np.real(np.sum(dU * np.conj(G[mu, idx])))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_force_finite_differences_lie(setup):
    dims, r, U, B, m, S, G, X = setup
    F = O.lie_force(U, G)
    T = O.su3_generators()
    rng = np.random.default_rng(2)
    eps = 1e-5
    for _ in range(16):
        mu, idx, a = rng.integers(4), rng.integers(int(np.prod(dims))), rng.integers(8)
        Up, Um = U.copy(), U.copy()
        Up[mu, idx] = expm(1j * eps * T[a]) @ U[mu, idx]
        Um[mu, idx] = expm(-1j * eps * T[a]) @ U[mu, idx]
        fd = (S(Up) - S(Um)) / (2 * eps)
        # F^a = -dS/d omega^a
        assert abs(fd + F[mu, idx, a]) <= 1e-6 * max(1.0, abs(fd))


def test_force_gauge_covariance(setup):
    dims, r, U, B, m, S, G, X = setup
    g = random_gauge_transform(dims, 99)
    Ug = _gauge_transform_links(dims, U, g)
    ge = g[_parity_sites(dims, 0)]
    gB = np.einsum("sab,sbj->saj", ge, B)
    Xg, _ = O.solve_block(dims, BC, Ug, m, r.beta, gB, 1e-14)
    Gg = O.force(dims, BC, Ug, r.alpha, Xg)
    # G transforms like the link: G^g_mu(x) = g(x) G_mu(x) g(x+mu)^dag
    expect = _gauge_transform_links(dims, G, g)
    assert np.abs(Gg - expect).max() < 1e-10 * np.abs(G).max()
    # and the action is invariant
    assert abs(O.action(gB, Xg, r.a0, r.alpha).sum() - O.action(B, X, r.a0, r.alpha).sum()) < 1e-10 * abs(
        O.action(B, X, r.a0, r.alpha).sum())
