"""The solver studies (Figs. 1 and 2 of Sec. III) on a small lattice, with
oracle spot checks:

* the per-column counts are the multi-shift CG iteration counts of the
  oracle (the block solver at n = 1 is multi-shift CG) within +-2;
* the eigenvalue estimate by inverse subspace iteration equals the lowest
  eigenvalues of the dense operator;
* the block solve never needs more Dirac calls than the per-column solves;
* after a fixed number of iterations the shifted residuals fall with the
  shift (eq. convergence_bound_shifts), and every reported residual is the
  oracle's true residual.
"""
import numpy as np
import pytest

from gpu_common import torch_gpu
from oracle import oracle as O
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


def test_eigenvalues_match_dense(torch):
    from paper_1808_01829_amd import studies
    dims = (4, 4, 4, 4)
    ctx = studies._ctx(dims, 0.5, 77)
    lam, change = studies.low_eigenvalues(ctx, k=8, extra=8, sweeps=14)
    A = O.dense_operator(dims, BC, random_gauge(dims, 0.5, 77), 0.0, 0.0)
    ref = np.linalg.eigvalsh(A)[:8]
    print("eigenvalues of K: %s (dense %s), last change %.1e" % (lam, ref, change))
    assert np.allclose(lam, ref, rtol=1e-5)


def test_fig1_counts_and_oracle_spot_check(torch):
    from paper_1808_01829_amd import studies
    dims, eps, seed = (6, 4, 4, 6), 0.5, 91
    rows = studies.fig1(dims, eps, seed, masses=(0.1,), npfs=(1, 2, 4), poles=8, tol=1e-10)
    assert [r["n_pf"] for r in rows] == [1, 2, 4]
    for r in rows:
        assert r["block_dirac_calls"] <= r["scg_dirac_calls"] + 2 * r["n_pf"]
        assert r["max_true_residual"] <= 1e-10
        assert 0 < r["sqrt_l1_over_lnpf"] <= 1
    # n_pf = 1: the block solve is the per-column solve
    assert rows[0]["block_iterations"] == rows[0]["scg_iterations"][0]
    # the oracle's multi-shift CG on the same column takes as many iterations
    m = 0.1
    rc = configs.coefficients(0.5, m * m, 16.0 + m * m, 8)
    U = random_gauge(dims, eps, seed)
    B = gaussian_block(dims, 4, seed + 1)
    for j in range(2):
        _, k, _ = O.mscg(dims, BC, U, m, np.sort(rc.beta), np.ascontiguousarray(B[..., j]), 0.5e-10)
        assert abs(k - rows[-1]["scg_iterations"][j]) <= 2, (k, rows[-1]["scg_iterations"][j])


def test_fig2_residuals_against_oracle(torch):
    from paper_1808_01829_amd import bms, studies
    dims, eps, seed, m = (6, 4, 4, 6), 0.5, 93, 0.05
    shifts = [1e-4, 1e-2, 0.3, 3.0]
    rows = studies.fig2(dims, eps, seed, mass=m, npfs=(1, 4), k_fixed=30, r_fixed=1e-6,
                        shifts=shifts)
    for r in rows:
        rk = np.asarray(r["residual_at_k"])
        assert np.all(np.diff(rk) <= 0), rk  # larger shifts have converged further
        assert r["iterations_at_r"] > 0
    # the reported residuals are true residuals (recomputed with the oracle)
    ctx = studies._ctx(dims, eps, seed)
    B = studies._block(dims, 4, seed + 1)
    o = bms.bms_default_opts()
    o.max_refine = 0
    X, _ = ctx.solve(m, shifts, B, tol=1e-30, max_iter=30, opts=o, raise_on_error=False)
    tr = O.true_residuals(dims, BC, random_gauge(dims, eps, seed), m, shifts, B.cpu().numpy(),
                          X.cpu().numpy())
    assert np.allclose(tr.max(axis=1), rows[1]["residual_at_k"], rtol=1e-6)
