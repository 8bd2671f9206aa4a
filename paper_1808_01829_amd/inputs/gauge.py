"""Seeded synthetic inputs: SU(3) gauge fields and complex-Gaussian pseudofermions.

These generators are shared by the HIP path and the oracle. They contain none of
the solver's arithmetic: they only draw random numbers and build unitary links.

Layouts (public, identical to the C-ABI):
  gauge   U[mu][idx][a][b], complex128, idx = x + Lx*(y + Ly*(z + Lz*t))
  block   B[cb][color][rhs], complex128 (site-major, right-hand side fastest)

The paper simulates thermalised beta=5.12 ensembles (Sec. IV); those are not
available, so fields are drawn as U = exp(i eps H) with H = sum_a h_a lambda_a/2,
h_a ~ N(0,1). Pseudofermion sources follow the Gaussian p(eta) ~ exp(-eta^dag eta)
used for the heatbath in Sec. II: Re and Im are N(0, 1/2).
"""
import numpy as np

# Gell-Mann matrices lambda_1..lambda_8
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1] = -1j
_GM[1][1, 0] = 1j
_GM[2][0, 0] = 1
_GM[2][1, 1] = -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2] = -1j
_GM[4][2, 0] = 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2] = -1j
_GM[6][2, 1] = 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)

GELL_MANN = _GM
# su(3) generators T^a = lambda_a / 2
GENERATORS = _GM / 2


def volume(dims):
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def check_dims(dims):
    dims = [int(d) for d in dims]
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError("lattice extents must be four even numbers >= 2, got %r" % (dims,))
    return dims


def _reunitarise(u):
    """Project 3x3 matrices back onto SU(3): Gram-Schmidt on rows 0,1 and
    row2 = conj(row0 x row1)."""
    r0 = u[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = u[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def su3_exp(h, eps):
    """exp(i eps H) for Hermitian H, by eigendecomposition, then re-unitarised."""
    w, v = np.linalg.eigh(h)
    ph = np.exp(1j * eps * w)
    u = np.einsum("...ij,...j,...kj->...ik", v, ph, np.conj(v))
    return _reunitarise(u)


def random_gauge(dims, eps, seed, chunk=1 << 18):
    """U[mu][idx] = exp(i eps H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1).

    Draws are made from numpy's PCG64 with the given seed in the fixed order
    (mu, idx, a), in chunks, so the field does not depend on chunk size.
    """
    dims = check_dims(dims)
    n = 4 * volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        h = rng.standard_normal((e - s, 8))
        hm = np.einsum("la,aij->lij", h, GENERATORS)
        out[s:e] = su3_exp(hm, eps)
    return out.reshape(4, volume(dims), 3, 3)


def unit_gauge(dims):
    """The free field U = 1."""
    dims = check_dims(dims)
    u = np.zeros((4, volume(dims), 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def gaussian_block(dims, n, seed):
    """B[cb][color][rhs] with Re, Im ~ N(0, 1/2) (so E|z|^2 = 1)."""
    dims = check_dims(dims)
    vh = volume(dims) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((vh, 3, n, 2)) * np.sqrt(0.5)
    return z[..., 0] + 1j * z[..., 1]


def random_gauge_transform(dims, seed):
    """Random SU(3) matrix per site g[idx] (for covariance checks)."""
    dims = check_dims(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = np.einsum("la,aij->lij", rng.standard_normal((volume(dims), 8)), GENERATORS)
    return su3_exp(h, 1.0)
