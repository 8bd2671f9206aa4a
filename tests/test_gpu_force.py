"""Force (eq. force) and autograd on the GPU.

* parity of the raw gradient and the su(3) force with the oracle, computed
  from the oracle's own solutions, on small lattices;
* on the 16^3x32 workload (n_pf = 8, 16 poles): the su(3) force against
  central finite differences of the action along 64 random single-link su(3)
  directions, the action difference taken as sum_j alpha_j Re phi^dag (X+ - X-)
  so that no large sums cancel;
* torch.autograd.gradcheck of the autograd.Function on a 2^4 lattice.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from gpu_common import rel, to_dev, to_np, torch_gpu
from oracle import oracle as O
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


# block widths 2 ... 16 (the workloads' widths 8 and 16 with the 16 poles of
# the 16^3 x 32 force workload), odd widths, and a lattice with extent 2
@pytest.mark.parametrize("dims,n,name", [((4, 4, 2, 4), 2, "c1"), ((4, 4, 4, 6), 3, "c2"),
                                         ((8, 8, 8, 8), 4, "c2"), ((4, 4, 4, 6), 8, "c4"),
                                         ((4, 6, 4, 4), 16, "c4"), ((6, 4, 2, 4), 5, "c4"),
                                         ((4, 4, 4, 4), 12, "c2")])
def test_force_parity(torch, dims, n, name):
    from paper_1808_01829_amd import bms
    r = configs.workload_coefficients(name)
    U = random_gauge(dims, 0.5, 31)
    B = gaussian_block(dims, n, 32)
    m = 0.05
    Xo, res = O.solve_block(dims, BC, U, m, r.beta, B, 1e-13)
    Go = O.force(dims, BC, U, r.alpha, Xo)
    Fo = O.lie_force(U, Go)
    c = bms.Context(dims, BC)
    c.set_gauge(to_dev(torch, U))
    Xd = to_dev(torch, Xo)  # the oracle's solutions as the kernel's input
    # the fused kernel (default) and the hops + per-link kernel (variant 0)
    for v in (-1, 0):
        c.set_variant(bms.BMS_KERNEL_FORCE, v)
        G = to_np(c.force(r.alpha, Xd, bms.BMS_FORCE_RAW))
        F = to_np(c.force(r.alpha, Xd, bms.BMS_FORCE_LIE))
        print("force n=%d %s variant %d: raw %.1e, Lie %.1e" % (
            n, "x".join(map(str, dims)), v, rel(G, Go), rel(F, Fo)))
        assert rel(G, Go) < 1e-12
        assert rel(F, Fo) < 1e-12
    c.set_variant(bms.BMS_KERNEL_FORCE, -1)
    # the full GPU path (solve + force) agrees to the solver's accuracy
    X, st = c.solve(m, r.beta, to_dev(torch, B), tol=1e-12)
    F2 = to_np(c.force(r.alpha, X, bms.BMS_FORCE_LIE))
    assert rel(F2, Fo) < 1e-7


def test_force_finite_differences_16c32(torch):
    from paper_1808_01829_amd import bms
    w = configs.WORKLOADS["c4"]
    r = configs.workload_coefficients("c4")
    dims, n, m = w["dims"], w["n"], w["mass"]
    U = random_gauge(dims, w["eps"], 4000)
    B = gaussian_block(dims, n, 4001)
    Bd = to_dev(torch, B)
    c = bms.Context(dims, BC)
    c.set_gauge(to_dev(torch, U))
    X, st = c.solve(m, r.beta, Bd, tol=1e-12, max_iter=20000)
    F = to_np(c.force(r.alpha, X, bms.BMS_FORCE_LIE))
    T = O.su3_generators()
    al = torch.tensor(r.alpha, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(44)
    eps = 1e-4
    Ug = to_dev(torch, U)
    errs = []
    for _ in range(64):
        mu, idx, a = int(rng.integers(4)), int(rng.integers(int(np.prod(dims)))), int(rng.integers(8))
        Xs = []
        for sgn in (1, -1):
            Up = Ug.clone()
            Up[mu, idx] = to_dev(torch, expm(1j * sgn * eps * T[a]) @ U[mu, idx])
            c.set_gauge(Up)
            Xp, _ = c.solve(m, r.beta, Bd, tol=1e-12, max_iter=20000)
            Xs.append(Xp)
        D = Xs[0] - Xs[1]
        dS = torch.einsum("s,s->", al, torch.real(torch.einsum("vci,svci->s", Bd.conj(), D)))
        fd = float(dS) / (2 * eps)
        errs.append(abs(fd + F[mu, idx, a]) / max(1e-3, abs(F[mu, idx, a])))
    assert max(errs) < 1e-4, errs


def test_autograd_gradcheck(torch):
    from paper_1808_01829_amd import bms
    from paper_1808_01829_amd.autograd import pseudofermion_action
    dims = (2, 2, 2, 2)
    r = configs.workload_coefficients("c1")
    U = random_gauge(dims, 0.5, 51)
    B = gaussian_block(dims, 2, 52)
    c = bms.Context(dims, BC)
    Ut = to_dev(torch, U).requires_grad_(True)
    Bd = to_dev(torch, B)

    def f(u):
        return pseudofermion_action(u, Bd, c, 0.1, r, tol=1e-13)

    assert torch.autograd.gradcheck(f, (Ut,), eps=1e-6, atol=1e-7, rtol=1e-5, fast_mode=True)
    # backward equals the oracle gradient
    S = f(Ut)
    S.backward()
    Xo, _ = O.solve_block(dims, BC, U, 0.1, r.beta, B, 1e-14)
    assert rel(to_np(Ut.grad), O.force(dims, BC, U, r.alpha, Xo)) < 1e-9
    assert abs(float(S) - O.action(B, Xo, r.a0, r.alpha).sum()) < 1e-10 * abs(float(S))
