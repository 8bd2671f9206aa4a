"""Mixed precision (FP32 operator and block updates, FP64 small matrices,
FP64 reliable updates and defect correction) against the FP64 oracle.

P1 is the hard criterion: every column of every shift has true FP64 relative
residual <= tol, recomputed here with the oracle's operator."""
import numpy as np
import pytest

from gpu_common import rel, to_dev, to_np, torch_gpu
from oracle import oracle as O
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


def _ctx(torch, dims, U):
    from paper_1808_01829_amd import bms
    c = bms.Context(dims, BC)
    c.set_gauge(to_dev(torch, U))
    return c


# mixed_switch 3e-4 (the default): FP64 multi-shift phase to 3e-4, then one
# FP32 multi-shift phase on the remaining residual; 1e-7: a short FP32 phase;
# 0: FP32 from the start with per-shift defect correction
@pytest.mark.parametrize("switch", [3e-4, 1e-7, 0.0])
def test_mixed_parity_8x8x8x8(torch, switch):
    from paper_1808_01829_amd import bms
    w = configs.WORKLOADS["c2"]
    r = configs.workload_coefficients("c2")
    dims, n, m = w["dims"], w["n"], w["mass"]
    U = random_gauge(dims, w["eps"], 2000)
    B = gaussian_block(dims, n, 2001)
    c = _ctx(torch, dims, U)
    X, st = c.solve(m, r.beta, to_dev(torch, B), tol=1e-11, precision=bms.BMS_PREC_MIXED,
                    reliable_interval=50, mixed_switch=switch)
    X = to_np(X)
    tr = O.true_residuals(dims, BC, U, m, r.beta, B, X)
    assert tr.max() <= 1e-11
    if switch == 0.0:
        assert st["reliable_updates"] > 0
    else:
        assert st["refine_iterations"] > 0  # the FP32 phase ran
    Xo, _ = O.solve_block(dims, BC, U, m, r.beta, B, 1e-13)
    kap = (16 + m * m + r.beta) / (m * m + r.beta)
    for s in range(len(r.beta)):
        assert np.linalg.norm(X[s] - Xo[s]) <= max(1e-9, 5 * kap[s] * 1e-11) * np.linalg.norm(Xo[s])


def test_mixed_16x16x16x16_workload(torch):
    from paper_1808_01829_amd import bms
    w = configs.WORKLOADS["c3"]
    r = configs.workload_coefficients("c3")
    dims, n, m = w["dims"], w["n"], w["mass"]
    U = random_gauge(dims, w["eps"], 3000)
    B = gaussian_block(dims, n, 3001)
    c = _ctx(torch, dims, U)
    X, st = c.solve(m, r.beta, to_dev(torch, B), tol=w["tol"], precision=bms.BMS_PREC_MIXED,
                    reliable_interval=w["reliable"])
    print("mixed 16^4: iterations %d, reliable %d, refine iterations %d, max residual %.2e" % (
        st["iterations"], st["reliable_updates"], st["refine_iterations"],
        st["max_true_residual"]))
    tr = O.true_residuals(dims, BC, U, m, r.beta, B, to_np(X))
    assert tr.max() <= w["tol"]
    # the library's own FP64 residual check agrees with the oracle's
    assert np.allclose(np.asarray(st["true_residual"]), tr, rtol=1e-3, atol=1e-14)


def test_mixed_32x32x32x32_benchmark_solve_sampled(torch):
    """The benchmarked solve at full size (32^4, n_pf = 16, 20 poles, mixed,
    default kernels, the benchmark's seeds): columns 0, 7 and 15 of every shift
    have true FP64 residual <= tol recomputed with the oracle's operator, and
    the library's own residual check agrees with it."""
    from paper_1808_01829_amd import bms
    w = configs.WORKLOADS["c5"]
    r = configs.workload_coefficients("c5")
    dims, n, m = w["dims"], w["n"], w["mass"]
    U = random_gauge(dims, w["eps"], 1000 * w["id"])
    B = gaussian_block(dims, n, 1000 * w["id"] + 1)
    c = _ctx(torch, dims, U)
    X, st = c.solve(m, r.beta, to_dev(torch, B), tol=w["tol"], precision=bms.BMS_PREC_MIXED,
                    reliable_interval=w["reliable"])
    assert st["converged"]
    cols = [0, 7, 15]
    Xs = np.ascontiguousarray(to_np(X[..., cols]))
    del X
    tr = O.true_residuals(dims, BC, U, m, r.beta, np.ascontiguousarray(B[..., cols]), Xs)
    assert tr.max() <= w["tol"]
    lib = np.asarray(st["true_residual"])[:, cols]
    assert np.allclose(lib, tr, rtol=1e-3, atol=1e-14)
