"""Pins of the input generators (no GPU): SU(3) links, Gaussian sources, and the
rational coefficients (Zolotarev's closed form for x^-1/2, equioscillation,
positivity of residues and poles as eq. RA requires)."""
import numpy as np
import pytest

from paper_1808_01829_amd.inputs import (configs, gaussian_block, random_gauge, remez,
                                         zolotarev_inv_sqrt)


def test_gauge_is_su3_and_seeded():
    U = random_gauge((2, 2, 2, 4), 0.8, 12)
    I = np.eye(3)
    assert np.abs(U @ np.conj(np.swapaxes(U, -1, -2)) - I).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    assert np.array_equal(U, random_gauge((2, 2, 2, 4), 0.8, 12))
    assert not np.array_equal(U, random_gauge((2, 2, 2, 4), 0.8, 13))
    # chunking does not change the draw
    assert np.array_equal(U, random_gauge((2, 2, 2, 4), 0.8, 12, chunk=7))


def test_gaussian_block_moments():
    B = gaussian_block((8, 8, 8, 8), 4, 3)
    assert B.shape == (2048, 3, 4)
    assert abs(np.mean(np.abs(B) ** 2) - 1) < 0.02
    assert abs(np.mean(B.real)) < 0.02 and abs(np.mean(B.imag)) < 0.02


def test_remez_equals_zolotarev_inv_sqrt():
    r = remez(0.5, 0.01, 16.01, 8)
    _, ez = zolotarev_inv_sqrt(0.01, 16.01, 8)
    assert abs(r.error - ez) < 1e-6 * ez


@pytest.mark.parametrize("name", ["c1", "c2", "c3", "c5"])
def test_cached_coefficients_equioscillate(name):
    r = configs.workload_coefficients(name)
    w = configs.WORKLOADS[name]
    assert r.n_poles == w["poles"]
    assert np.all(r.alpha > 0) and np.all(r.beta > 0) and r.a0 > 0
    xs = np.exp(np.linspace(np.log(r.lo), np.log(r.hi), 400001))
    e = r.rel_error(xs)
    assert np.abs(e).max() <= r.error * (1 + 1e-3) + 1e-15
    if r.error > 1e-11:  # resolvable in double precision
        # 2N+2 alternating extrema of (nearly) equal magnitude
        big = np.abs(e) > 0.5 * r.error  # ignore rounding noise near the zeros
        eb = e[big]
        s = np.sign(eb)
        runs = np.split(np.abs(eb), np.nonzero(np.diff(s))[0] + 1)
        peaks = np.array([x.max() for x in runs])
        assert len(peaks) == 2 * r.n_poles + 2
        assert peaks.min() > 0.99 * r.error


def test_cache_matches_fresh_fit():
    r = configs.workload_coefficients("c1")
    f = remez(0.5, 0.01, 16.01, 8)
    assert np.allclose(r.beta, f.beta, rtol=1e-9) and np.allclose(r.alpha, f.alpha, rtol=1e-9)
