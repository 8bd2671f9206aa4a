"""The matrix-core (MFMA) kernels against the oracle's Algorithm 1.

After k block iterations (max_iter = k, no refinement) the solutions X^(s)_k
of the HIP solver are compared with the oracle's sbcgrq run for the same k
iterations, for each pairing of update kernel (MFMA = the default at n = 8, 16, with
the shifted solutions updated every second iteration, variants 4 and 5;
MFMA updating every shift every iteration = variant 6; vector = variant 2) and Gram kernel (MFMA with 8 or 4 row steps in
flight = the default and variant 1; vector = variant 0). Row counts 3*Vh that
are not a multiple of the 16-row tile, and blocks whose row range is not a
multiple of the 4-row Gram step, exercise the ragged edges.
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


# (update variant, Gram variant)
KERNELS = [(-1, -1), (2, 0), (4, 1), (2, 2), (5, 0), (2, 3), (5, 3), (4, 0), (4, 4), (5, 5),
           (6, -1), (6, 1)]


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
    for upd, gram in KERNELS:
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, upd)
        ctx.set_variant(bms.BMS_KERNEL_GRAM, gram)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-15, max_iter=k, max_refine=0,
                          raise_on_error=False)
        assert st["status"] == bms.BMS_ENOCONV and st["iterations"] == k
        out[(upd, gram)] = to_np(X)
    for s in range(len(r.beta)):
        ref = np.linalg.norm(Xo[s])
        for key, X in out.items():
            err = np.linalg.norm(X[s] - Xo[s]) / ref
            assert err <= 1e-11, (key, s, err)
        # the kernels differ only in rounding order
        for key, X in out.items():
            assert np.linalg.norm(X[s] - out[KERNELS[0]][s]) / ref <= 1e-12, (key, s)


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
    for variant in (4, 6, 2):
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, variant)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-10)
        tr = O.true_residuals(dims, BC, U, mass, r.beta, B, to_np(X))
        assert tr.max() <= 1e-10
        res[variant] = st["iterations"]
    assert abs(res[4] - res[2]) <= 1 and abs(res[6] - res[2]) <= 1


@pytest.mark.parametrize("n,max_iter", [(8, 10000), (16, 10000), (16, 23), (8, 24)])
def test_two_iteration_update_matches_every_iteration(torch, n, max_iter):
    """Shifts freeze at different iterations, after either half of the
    two-iteration cycle, and the solve may stop at max_iter with increments
    pending: the solutions equal those of the every-iteration update (variant
    6) up to the order of the additions into X, and the residual estimates
    of the two forms are the same."""
    from paper_1808_01829_amd import bms
    dims = (6, 4, 4, 6)
    r = configs.workload_coefficients("c2")
    U = random_gauge(dims, 0.5, 41 + n)
    B = gaussian_block(dims, n, 43 + n)
    ctx = bms.Context(dims, BC)
    ctx.set_gauge(to_dev(torch, U))
    out = {}
    for upd in (6, 4, 5):
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, upd)
        X, st = ctx.solve(0.05, r.beta, to_dev(torch, B), tol=1e-10, max_iter=max_iter,
                          max_refine=0, raise_on_error=False)
        out[upd] = (to_np(X), st)
    X6, st6 = out[6]
    for upd in (4, 5):
        X, st = out[upd]
        assert st["iterations"] == st6["iterations"] and st["status"] == st6["status"]
        for s in range(len(r.beta)):
            ref = np.linalg.norm(X6[s])
            assert np.linalg.norm(X[s] - X6[s]) / ref <= 1e-12, (upd, s)


@pytest.mark.parametrize("n", [8, 16])
def test_mfma_gram_mixed_precision_solve(torch, n):
    """FP32 blocks in the MFMA Gram (FP32 matrix-core products over rounds of 4D rows, FP64
    totals) against the vector Gram (FP64 accumulation) in the mixed solver: every shift
    converges and the iteration counts agree."""
    from paper_1808_01829_amd import bms
    dims = (6, 4, 4, 6)
    r = configs.workload_coefficients("c2")
    mass = 0.05
    U = random_gauge(dims, 0.5, 15)
    B = gaussian_block(dims, n, 16)
    ctx = bms.Context(dims, BC)
    ctx.set_gauge(to_dev(torch, U))
    its = {}
    for gram in (-1, 0):
        ctx.set_variant(bms.BMS_KERNEL_GRAM, gram)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-10,
                          precision=bms.BMS_PREC_MIXED, reliable_interval=20)
        tr = O.true_residuals(dims, BC, U, mass, r.beta, B, to_np(X))
        assert tr.max() <= 1e-10
        its[gram] = st["multishift_iterations"]
    assert abs(its[-1] - its[0]) <= 3


@pytest.mark.parametrize("dims,n,k", [((6, 4, 4, 6), 16, 1), ((6, 4, 4, 6), 16, 6),
                                      ((6, 4, 4, 6), 8, 6), ((2, 2, 2, 6), 16, 3)])
def test_mfma_update_f32_matches_vector(torch, dims, n, k):
    """The FP32 matrix-core update of the mixed solver against the FP32 vector
    update, k iterations, no reliable update inside, no refinement."""
    from paper_1808_01829_amd import bms
    r = configs.workload_coefficients("c2")
    mass = 0.05
    U = random_gauge(dims, 0.5, 31 + n)
    B = gaussian_block(dims, n, 37 + k)
    ctx = bms.Context(dims, BC)
    ctx.set_gauge(to_dev(torch, U))
    out = {}
    for upd in (-1, 2):
        ctx.set_variant(bms.BMS_KERNEL_UPDATE, upd)
        X, st = ctx.solve(mass, r.beta, to_dev(torch, B), tol=1e-15, max_iter=k, max_refine=0,
                          precision=bms.BMS_PREC_MIXED, reliable_interval=1000,
                          raise_on_error=False)
        assert st["multishift_iterations"] == k
        out[upd] = to_np(X)
    for s in range(len(r.beta)):
        ref = np.linalg.norm(out[2][s])
        assert np.isfinite(out[-1][s]).all(), s
        assert np.linalg.norm(out[-1][s] - out[2][s]) / ref <= 5e-5, (s, np.linalg.norm(out[-1][s] - out[2][s]) / ref)
