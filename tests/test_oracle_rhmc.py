"""Pins of the oracle's RHMC trajectory pieces (CPU only).

* Wilson action: zero at U = 1, gauge invariant, and its link derivative
  (the staple force) against central finite differences along random su(3)
  directions;
* link update: stays in SU(3) and composes, exp(i e P) exp(i e P) = exp(2 i e P);
* two-level OMF2: reversible (P -> -P retraces the trajectory) and second
  order (halving the step divides dH by about 4), for pure gauge and with
  pseudofermions;
* heatbath: the initial pseudofermion action equals eta^dag eta.
"""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import oracle as O
from oracle import rhmc as R
from paper_1808_01829_amd.inputs import configs, gaussian_block, random_gauge, unit_gauge

BC = (1, 1, 1, -1)
DIMS = (4, 4, 4, 4)


def _mom(dims, seed):
    return np.random.default_rng(seed).standard_normal((4, int(np.prod(dims)), 8))


def test_wilson_action_zero_and_invariant():
    assert abs(R.wilson_action(DIMS, unit_gauge(DIMS), 5.12)) < 1e-12
    U = random_gauge(DIMS, 0.5, 1)
    g = random_gauge(DIMS, 1.0, 2)[0]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[mu] = g @ U[mu] @ np.conj(np.swapaxes(R._shift(DIMS, g, mu, 1), -1, -2))
    assert abs(R.wilson_action(DIMS, Ug, 5.12) - R.wilson_action(DIMS, U, 5.12)) < 1e-10


def test_gauge_force_finite_differences():
    beta, eps = 5.12, 1e-5
    U = random_gauge((4, 4, 2, 4), 0.6, 3)
    dims = (4, 4, 2, 4)
    F = R.gauge_force(dims, U, beta)
    T = O.su3_generators()
    rng = np.random.default_rng(4)
    for _ in range(12):
        mu, idx, a = int(rng.integers(4)), int(rng.integers(np.prod(dims))), int(rng.integers(8))
        s = []
        for sg in (1, -1):
            Up = U.copy()
            Up[mu, idx] = expm(1j * sg * eps * T[a]) @ U[mu, idx]
            s.append(R.wilson_action(dims, Up, beta))
        fd = (s[0] - s[1]) / (2 * eps)
        assert abs(fd + F[mu, idx, a]) <= 1e-7 * max(1.0, abs(fd)), (mu, idx, a, fd, F[mu, idx, a])


def test_link_update_stays_su3_and_composes():
    U = random_gauge(DIMS, 0.5, 5)
    P = _mom(DIMS, 6)
    U1 = R.link_update(U, P, 0.1)
    I = np.eye(3)
    assert np.abs(U1 @ np.conj(np.swapaxes(U1, -1, -2)) - I).max() < 1e-13
    assert np.abs(np.linalg.det(U1) - 1).max() < 1e-13
    assert np.abs(R.link_update(R.link_update(U, P, 0.1), P, 0.1) - R.link_update(U, P, 0.2)).max() < 1e-13


def _params(**kw):
    p = dict(beta=5.12, mass=0.05, tau=0.3, n_steps=3, n_gauge=3, lam=1.0 / 6.0)
    p.update(kw)
    p["lambda"] = p.pop("lam")
    return p


def test_pure_gauge_omf2_reversible_and_second_order():
    U = random_gauge(DIMS, 0.3, 7)
    P = _mom(DIMS, 8)
    p = _params()
    t = R.trajectory(DIMS, BC, U, P, None, p)
    back = R.trajectory(DIMS, BC, t["U"], -t["P"], None, p)
    assert np.abs(back["U"] - U).max() < 1e-11
    assert np.abs(back["P"] + P).max() < 1e-10
    dh = [abs(R.trajectory(DIMS, BC, U, P, None, _params(n_steps=k, n_gauge=1))["dH"])
          for k in (4, 8)]
    assert 3.0 < dh[0] / dh[1] < 5.0, dh


@pytest.fixture(scope="module")
def fits():
    return dict(r_hb=configs.heatbath_coefficients("c2"), r_acc=configs.accept_coefficients("c2"),
                r_md=configs.workload_coefficients("c2"))


def test_rhmc_trajectory_heatbath_reversibility_second_order(fits):
    dims = (4, 4, 4, 4)
    U = random_gauge(dims, 0.3, 9)
    P = _mom(dims, 10)
    eta = gaussian_block(dims, 2, 11)
    p = _params(tau=0.2, n_steps=2, n_gauge=2, **fits)
    p.update(tol_hb=1e-13, tol_md=1e-13)
    t = R.trajectory(dims, BC, U, P, eta, p)
    # heatbath: S_f(phi) = eta^dag eta (the fits' product is 1 to 1e-15)
    assert abs(t["Sf0"] - np.sum(np.abs(eta) ** 2)) <= 1e-11 * t["Sf0"]
    # reversibility with the same pseudofermions
    p2 = dict(p)
    p2["h"] = p["tau"] / p["n_steps"]
    U2, P2 = R.md(dims, BC, t["U"], -t["P"], t["phi"], p2)
    assert np.abs(U2 - U).max() < 1e-9
    assert np.abs(P2 + P).max() < 1e-8
    # second order: dH falls about 4x when the step halves
    dh = []
    for k in (2, 4):
        pk = dict(p)
        pk["n_steps"] = k
        dh.append(abs(R.trajectory(dims, BC, U, P, eta, pk)["dH"]))
    assert 2.5 < dh[0] / dh[1] < 6.0, dh
