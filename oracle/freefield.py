"""Test infrastructure only: exact free-field (U = 1) solves by FFT.

With U = 1 the staggered phases cancel in D^2 (eta_nu(x+mu) = -eta_nu(x) for
mu < nu, so the cross terms of D^2 cancel pairwise) and

    -D^2 = sum_mu (2 - T_{2mu} - T_{-2mu}) / 4,

a translation-invariant operator that keeps parity, with eigenvalues
sum_mu sin^2 p_mu. Hence on even sites

    (A + sigma) = m^2 + sigma + sum_mu sin^2 p_mu      in momentum space,

with p_mu = 2 pi k / L_mu (periodic) or (2k+1) pi / L_mu (antiperiodic). A
source on even sites, zero-extended to the whole lattice, is solved exactly by
dividing its Fourier transform by that symbol. This is independent of the CG
and of the operator code, and pins both at U = 1 at any lattice size.

The improved operator with one-hop links c1 and three-hop links c3 (both
times the unit matrix) is diagonalised the same way: its symbol is
m^2 + sigma + sum_mu (c1 sin p_mu + c3 sin 3 p_mu)^2 (the three-hop also
flips the staggered phases of later directions, so the cross terms cancel
as before).
"""
import numpy as np


def _site_arrays(dims):
    Lx, Ly, Lz, Lt = dims
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                             indexing="ij")
    return x, y, z, t  # arrays shaped [t][z][y][x] = lexicographic order


def _twists(dims, bc):
    return [0.0 if b > 0 else np.pi / L for L, b in zip(dims, bc)]


def symbol(dims, bc, mass, sigma, c1=1.0, c3=0.0):
    """m^2 + sigma + sum (c1 sin p + c3 sin 3p)^2 over the FFT grid, shaped [t][z][y][x]."""
    th = _twists(dims, bc)
    ks = []
    for mu, L in enumerate(dims):
        ks.append(2 * np.pi * np.fft.fftfreq(L) + th[mu])
    pt, pz, py, px = np.meshgrid(ks[3], ks[2], ks[1], ks[0], indexing="ij")

    def f(p):
        return (c1 * np.sin(p) + c3 * np.sin(3 * p)) ** 2

    return mass ** 2 + sigma + f(px) + f(py) + f(pz) + f(pt)


def _even_mask(dims):
    x, y, z, t = _site_arrays(dims)
    return ((x + y + z + t) % 2) == 0


def solve(dims, bc, mass, sigma, b, c1=1.0, c3=0.0):
    """Exact x = (A + sigma)^-1 b at U = 1 for a half vector b[Vh][3] or a
    block b[Vh][3][n] (even sites)."""
    dims = [int(d) for d in dims]
    Lx, Ly, Lz, Lt = dims
    vh = Lx * Ly * Lz * Lt // 2
    b = np.asarray(b, dtype=np.complex128)
    tail = b.shape[1:]
    even = _even_mask(dims).reshape(-1)
    idx_even = np.nonzero(even)[0]           # ascending lexicographic = cb order
    assert len(idx_even) == vh and np.all((idx_even >> 1) == np.arange(vh))
    full = np.zeros((Lx * Ly * Lz * Lt,) + tail, dtype=np.complex128)
    full[idx_even] = b
    full = full.reshape((Lt, Lz, Ly, Lx) + tail)
    x, y, z, t = _site_arrays(dims)
    th = _twists(dims, bc)
    phase = np.exp(1j * (th[0] * x + th[1] * y + th[2] * z + th[3] * t))
    ph = phase.reshape(phase.shape + (1,) * len(tail))
    f = np.fft.fftn(full / ph, axes=(0, 1, 2, 3))
    sym = symbol(dims, bc, mass, sigma, c1, c3).reshape((Lt, Lz, Ly, Lx) + (1,) * len(tail))
    sol = np.fft.ifftn(f / sym, axes=(0, 1, 2, 3)) * ph
    return sol.reshape((-1,) + tail)[idx_even]


def spectrum(dims, bc, mass, c1=1.0, c3=0.0):
    """Eigenvalues of A on the even-site space at U = 1 (each momentum of the
    full lattice carries one even-site mode per colour after halving)."""
    s = symbol(dims, bc, mass, 0.0, c1, c3).reshape(-1)
    # the full-lattice operator -D^2 is block diagonal in parity with equal
    # spectra on both parities, so the even-site spectrum is every value once
    # per colour, halved in multiplicity
    vals = np.sort(np.repeat(s, 3))
    return vals[::2]
