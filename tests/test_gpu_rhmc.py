"""RHMC trajectory on the GPU (Sec. II; the settings of Sec. IV) against the
oracle's numpy trajectory.

* the gauge-field steps: Wilson action, staple force (added into momenta),
  link exponential and kinetic energy, element by element;
* a pure gauge HMC trajectory and an RHMC trajectory with two pseudofermions
  (heatbath, accept action, two-level Omelyan integration) with every solve
  at 1e-12: final links, momenta and every energy equal the oracle's;
* at the paper's settings (force solves at 1e-7, heatbath and action at
  1e-14) on the 8^4 workload: S_f(phi) = eta^dag eta after the heatbath,
  and dH falls about 4x when the step halves (second order).
"""
import numpy as np
import pytest

from gpu_common import rel, to_dev, to_np, torch_gpu
from oracle import rhmc as R
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge

pytestmark = pytest.mark.gpu
BC = (1, 1, 1, -1)


@pytest.fixture(scope="module")
def torch():
    return torch_gpu()


def _mom(dims, seed):
    return np.random.default_rng(seed).standard_normal((4, int(np.prod(dims)), 8))


def _fits(name="c2"):
    return dict(r_hb=configs.heatbath_coefficients(name), r_acc=configs.accept_coefficients(name),
                r_md=configs.workload_coefficients(name))


def test_gauge_steps_match_oracle(torch):
    from paper_1808_01829_amd import bms
    dims, beta = (4, 4, 2, 6), 5.12
    U = random_gauge(dims, 0.6, 201)
    P = _mom(dims, 202)
    c = bms.Context(dims, BC)
    Ud, Pd = to_dev(torch, U), to_dev(torch, P)
    assert abs(c.gauge_action(beta, Ud) - R.wilson_action(dims, U, beta)) <= 1e-12 * \
        R.wilson_action(dims, U, beta)
    assert abs(c.kinetic_energy(Pd) - R.kinetic(P)) <= 1e-13 * R.kinetic(P)
    c.gauge_force(beta, Ud, Pd, 0.37)
    ref = P + 0.37 * R.gauge_force(dims, U, beta)
    assert rel(to_np(Pd), ref) < 1e-13
    c.gauge_update(0.11, to_dev(torch, P), Ud)
    assert rel(to_np(Ud), R.link_update(U, P, 0.11)) < 1e-13


def _traj_gpu(torch, dims, U, P, eta, p):
    from paper_1808_01829_amd import bms
    c = bms.Context(dims, BC)
    Ud, Pd = to_dev(torch, U), to_dev(torch, P)
    kw = {k: p[k] for k in ("r_hb", "r_acc", "r_md") if k in p}
    res = bms.rhmc_trajectory(c, Ud, Pd, to_dev(torch, eta) if eta is not None else None,
                              p["beta"], p["mass"], tau=p["tau"], n_steps=p["n_steps"],
                              n_gauge=p["n_gauge"], lam=p["lambda"], tol_hb=p.get("tol_hb", 1e-14),
                              tol_md=p.get("tol_md", 1e-7), **kw)
    return to_np(Ud), to_np(Pd), res


def _params(**kw):
    p = dict(beta=5.12, mass=0.05, tau=0.3, n_steps=3, n_gauge=3)
    p["lambda"] = 1.0 / 6.0
    p.update(kw)
    return p


def test_pure_gauge_trajectory_matches_oracle(torch):
    dims = (4, 4, 4, 4)
    U = random_gauge(dims, 0.3, 211)
    P = _mom(dims, 212)
    p = _params()
    U1, P1, res = _traj_gpu(torch, dims, U, P, None, p)
    o = R.trajectory(dims, BC, U, P, None, p)
    print("pure gauge: dH %.3e (oracle %.3e)" % (res["dH"], o["dH"]))
    assert np.abs(U1 - o["U"]).max() < 1e-12
    assert np.abs(P1 - o["P"]).max() < 1e-11
    assert abs(res["dH"] - o["dH"]) < 1e-9
    assert abs(res["H0"] - o["H0"]) < 1e-9 * abs(o["H0"])


def test_rhmc_trajectory_matches_oracle(torch):
    dims = (4, 4, 4, 4)
    U = random_gauge(dims, 0.3, 221)
    P = _mom(dims, 222)
    eta = gaussian_block(dims, 2, 223)
    p = _params(tau=0.2, n_steps=2, n_gauge=2, tol_hb=1e-12, tol_md=1e-12, **_fits())
    U1, P1, res = _traj_gpu(torch, dims, U, P, eta, p)
    o = R.trajectory(dims, BC, U, P, eta, p)
    print("rhmc 4^4 n=2: dH %.6e (oracle %.6e), Sf0 %.10e (eta^2 %.10e), %d force evaluations, "
          "%d iterations" % (res["dH"], o["dH"], res["Sf0"], np.sum(np.abs(eta) ** 2),
                             res["force_evals"], res["iterations"]))
    assert res["force_evals"] == 2 * p["n_steps"] + 1
    assert np.abs(U1 - o["U"]).max() < 1e-9
    assert np.abs(P1 - o["P"]).max() < 1e-8
    for k in ("K0", "Sg0", "Sf0", "K1", "Sg1", "Sf1"):
        assert abs(res[k] - o[k]) <= 1e-9 * max(1.0, abs(o[k])), k
    assert abs(res["dH"] - o["dH"]) < 1e-7


def test_rhmc_paper_settings_8x8x8x8(torch):
    w = configs.WORKLOADS["c2"]
    dims, n = w["dims"], w["n"]
    U = random_gauge(dims, 0.3, 231)
    P = _mom(dims, 232)
    eta = gaussian_block(dims, n, 233)
    dh = []
    for k in (4, 8):
        p = _params(mass=w["mass"], tau=0.5, n_steps=k, n_gauge=3, tol_hb=1e-14, tol_md=1e-7,
                    **_fits())
        _, _, res = _traj_gpu(torch, dims, U, P, eta, p)
        e2 = float(np.sum(np.abs(eta) ** 2))
        print("rhmc 8^4 n_pf=4, %d steps: dH %.3e, Sf0/eta^2 - 1 = %.1e, heatbath/action "
              "residual %.1e, %d force evaluations, %d iterations" % (
                  k, res["dH"], res["Sf0"] / e2 - 1, res["max_residual_hb"], res["force_evals"],
                  res["iterations"]))
        assert abs(res["Sf0"] / e2 - 1) < 1e-11
        assert res["max_residual_hb"] <= 1e-14
        dh.append(abs(res["dH"]))
    assert 2.5 < dh[0] / dh[1] < 6.0, dh
