"""The matrix-core (MFMA) FP64 block update against the oracle's Algorithm 1.

After k block iterations (max_iter = k, no refinement) the solutions X^(s)_k
of the HIP solver, with the MFMA update (the default for FP64 at n = 8, 16)
and with the vector update (variant 2), are compared with the oracle's
sbcgrq run for the same k iterations. Row counts 3*Vh that are not a multiple
of the 16-row tile exercise the ragged last tile.
"""
import numpy as np
import pytest

from gpu_common import to_dev, to_np, torch_gpu
from oracle import oracle as O
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


CASES = [
    ((4, 4, 4, 4), 16, 5),   # rows 384: 24 full tiles
    ((2, 2, 2, 6), 8, 4),    # rows 72: ragged last tile
    ((2, 2, 2, 6), 16, 3),   # ragged, Krylov space 48 of 72
    ((4, 4, 2, 6), 8, 11),   # rows 288, iterations span two host chunks
    ((6, 4, 4, 2), 16, 9),   # rows 288: 18 tiles, odd tile count per wave pair
]


@pytest.mark.parametrize("dims,n,k", CASES)
def test_mfma_update_matches_oracle_iterates(torch, dims, n, k):
    from paper_1808_01829_amd import bms
    r = configs.workload_coefficients("c2")
    mass = 0.05
    U = random_gauge(dims, 0.5, 17 + n)
    B = gaussian_block(dims, n, 23 + k)
    oo = O.sbcgrq_lattice(dims, BC, U, mass, r.beta, B, 1e-30, maxiter=k)
    assert oo["iters"] == k
    Xo = oo["X"]
    ctx = bms.Context(dims, BC)
    ctx.set_gauge(to_dev(torch, U))
    out = {}
    for variant in (-1, 2):
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, variant)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-15, max_iter=k, max_refine=0,
                          raise_on_error=False)
        assert st["status"] == bms.BMS_ENOCONV and st["iterations"] == k
        out[variant] = to_np(X)
    for s in range(len(r.beta)):
        ref = np.linalg.norm(Xo[s])
        for variant, X in out.items():
            err = np.linalg.norm(X[s] - Xo[s]) / ref
            assert err <= 1e-11, (variant, s, err)
        # the two kernels differ only in rounding order
        assert np.linalg.norm(out[-1][s] - out[2][s]) / ref <= 1e-12


@pytest.mark.parametrize("n", [8, 16])
def test_mfma_full_solve_converges(torch, n):
    from paper_1808_01829_amd import bms
    dims = (4, 4, 4, 6)
    r = configs.workload_coefficients("c2")
    mass = 0.05
    U = random_gauge(dims, 0.5, 5)
    B = gaussian_block(dims, n, 6)
    ctx = bms.Context(dims, BC)
    ctx.set_gauge(to_dev(torch, U))
    res = {}
    for variant in (4, 2):
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, variant)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-10)
        tr = O.true_residuals(dims, BC, U, mass, r.beta, B, to_np(X))
        assert tr.max() <= 1e-10
        res[variant] = st["iterations"]
    assert abs(res[4] - res[2]) <= 1
