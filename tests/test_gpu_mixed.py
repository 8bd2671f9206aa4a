"""Mixed precision (FP32 operator and block updates, FP64 small matrices,
FP64 reliable updates and defect correction) against the FP64 oracle.

P1 is the hard criterion: every column of every shift has true FP64 relative
residual <= tol, recomputed here with the oracle's operator. P2: the
solutions within relative 1e-9 of the oracle's FP64 multi-shift CG at 1e-14,
per shift, flat (each shift's value printed)."""
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


def _p2(X, Xo, label, cols=None):
    e = np.array([np.linalg.norm(X[s] - Xo[s]) / np.linalg.norm(Xo[s]) for s in range(len(X))])
    print("P2 %s: max %.2e; per shift %s" % (label, e.max(), " ".join("%.1e" % v for v in e)))
    return e


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
    assert st["iterations"] == st["multishift_iterations"] + st["refine_iterations"]
    assert st["iterations"] == st["iterations_f64"] + st["iterations_f32"]
    assert st["iterations_f32"] > 0
    Xo, _ = O.solve_block(dims, BC, U, m, r.beta, B, 1e-14)
    e = _p2(X, Xo, "mixed 8^4 switch %g tol 1e-11" % switch)
    assert e.max() <= 1e-9


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
    Xh = to_np(X)
    tr = O.true_residuals(dims, BC, U, m, r.beta, B, Xh)
    assert tr.max() <= w["tol"]
    # the library's own FP64 residual check agrees with the oracle's
    assert np.allclose(np.asarray(st["true_residual"]), tr, rtol=1e-3, atol=1e-14)
    # P2 on two columns against the oracle's multi-shift CG at 1e-14
    cols = [0, 5]
    Xo, _ = O.solve_block(dims, BC, U, m, r.beta, np.ascontiguousarray(B[..., cols]), 1e-14)
    e = _p2(np.ascontiguousarray(Xh[..., cols]), Xo, "mixed 16^4 columns %s" % cols)
    assert e.max() <= 1e-9


def test_mixed_32x32x32x32_benchmark_solve_all_columns(torch):
    """The benchmarked solve at full size (32^4, n_pf = 16, 20 poles, mixed,
    default kernels, the benchmark's seeds): all 16 columns of all 20 shifts
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
    print("mixed 32^4: iterations %d (multi-shift FP64 %d, after it %d; FP64 %d, FP32 %d), "
          "hop calls %d, reliable updates %d" % (
              st["iterations"], st["multishift_iterations"], st["refine_iterations"],
              st["iterations_f64"], st["iterations_f32"], st["hop_calls"],
              st["reliable_updates"]), flush=True)
    assert st["iterations"] == st["iterations_f64"] + st["iterations_f32"]
    lib = np.asarray(st["true_residual"])
    worst = 0.0
    for s in range(len(r.beta)):
        Xs = to_np(X[s])
        tr = O.true_residuals(dims, BC, U, m, [r.beta[s]], B, Xs[None])[0]
        assert tr.max() <= w["tol"], (s, tr.max())
        assert np.allclose(lib[s], tr, rtol=1e-3, atol=1e-14)
        worst = max(worst, tr.max())
    print("mixed 32^4: all %d columns x %d shifts, max true residual %.2e" % (
        n, len(r.beta), worst))
