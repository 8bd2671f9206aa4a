"""Test infrastructure only: a plain numpy RHMC trajectory (Sec. II and the
run settings of Sec. IV) for checking the library's trajectory.

Only tests may import this module. It uses the C oracle's operator, plain
CG per shift and column, force and Lie force (oracle.py) and adds:

  wilson_action   S_g = beta sum_{x, mu<nu} (1 - Re Tr U_mu nu(x) / 3),
                  U_mu nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                  (the gauge part of the HMC; periodic links)
  gauge_force     F^a = -dS_g/d omega^a for U_mu(x) -> exp(i omega^a T^a) U_mu(x):
                  with the staple sum A_mu(x) of the six plaquettes through the
                  link, Re Tr(U A) changes by -omega^a Im Tr(T^a U A), so
                  F^a = -(beta/3) Im Tr(T^a U A)
  link_update     U <- exp(i eps P^a T^a) U (eigendecomposition of the
                  Hermitian exponent)
  trajectory      heatbath phi = r_hb(A) eta, H = 1/2 sum (P^a)^2 + S_g + S_f,
                  two-level second-order Omelyan (OMF2) molecular dynamics
                  (outer level: fermion force; each outer drift of the links
                  integrated by n_gauge inner OMF2 steps of the gauge force),
                  final H, dH.
Layouts as in oracle.py: U[mu][idx][3][3], P[mu][idx][8], eta/phi [Vh][3][n].
"""
import numpy as np

from . import oracle as O


def _shift(dims, F, mu, k):
    """G[..., x, ...] = F[..., x + k mu, ...] for fields shaped [V][...] in
    lexicographic order (periodic)."""
    Lx, Ly, Lz, Lt = dims
    f = F.reshape((Lt, Lz, Ly, Lx) + F.shape[1:])
    axis = 3 - mu
    return np.roll(f, -k, axis=axis).reshape(F.shape)


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def plaquettes(dims, U):
    """Re Tr U_mu nu(x) / 3 for every site and mu < nu: [6][V]."""
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            P = U[mu] @ _shift(dims, U[nu], mu, 1) @ _dag(_shift(dims, U[mu], nu, 1)) @ _dag(U[nu])
            out.append(np.real(np.trace(P, axis1=-2, axis2=-1)) / 3.0)
    return np.array(out)


def wilson_action(dims, U, beta):
    return float(beta * np.sum(1.0 - plaquettes(dims, U)))


def staples(dims, U, mu):
    """A_mu(x) = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
                               + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)],
    so that the plaquettes through U_mu(x) sum to Re Tr(U_mu(x) A_mu(x))."""
    A = np.zeros_like(U[mu])
    for nu in range(4):
        if nu == mu:
            continue
        up = _shift(dims, U[nu], mu, 1) @ _dag(_shift(dims, U[mu], nu, 1)) @ _dag(U[nu])
        Unu_m = _shift(dims, U[nu], nu, -1)                  # U_nu(x - nu)
        down = _dag(_shift(dims, Unu_m, mu, 1)) @ _dag(_shift(dims, U[mu], nu, -1)) @ Unu_m
        A += up + down
    return A


def gauge_force(dims, U, beta):
    """F^a = -(beta/3) Im Tr(T^a U A), [mu][V][8]."""
    T = O.su3_generators()
    F = np.empty(U.shape[:2] + (8,))
    for mu in range(4):
        W = U[mu] @ staples(dims, U, mu)
        F[mu] = -(beta / 3.0) * np.imag(np.einsum("aij,...ji->...a", T, W))
    return F


def link_update(U, P, eps):
    """U <- exp(i eps P^a T^a) U."""
    T = O.su3_generators()
    X = eps * np.einsum("...a,aij->...ij", P, T)
    w, V = np.linalg.eigh(X)
    E = V @ (np.exp(1j * w)[..., None] * _dag(V))
    return E @ U


def kinetic(P):
    return float(0.5 * np.sum(P * P))


def _solve(dims, bc, U, mass, shifts, B, tol):
    X, _ = O.solve_block(dims, bc, U, mass, shifts, B, tol)
    return X


def fermion_action(dims, bc, U, mass, r, phi, tol):
    X = _solve(dims, bc, U, mass, r.beta, phi, tol)
    return float(np.sum(O.action(phi, X, r.a0, r.alpha)))


def fermion_force(dims, bc, U, mass, r, phi, tol):
    X = _solve(dims, bc, U, mass, r.beta, phi, tol)
    return O.lie_force(U, O.force(dims, bc, U, r.alpha, X))


def omf2(P, U, h, n, lam, kick, drift):
    """n second-order Omelyan steps of size h for H = T(P) + S(U):
    P += lam h F; U drift h/2; P += (1 - 2 lam) h F; U drift h/2; P += lam h F,
    the last kick of a step merged with the first of the next."""
    P = kick(P, U, lam * h)
    for k in range(n):
        U = drift(P, U, 0.5 * h)
        P = kick(P, U, (1.0 - 2.0 * lam) * h)
        U = drift(P, U, 0.5 * h)
        P = kick(P, U, (2.0 if k < n - 1 else 1.0) * lam * h)
    return P, U


def md(dims, bc, U, P, phi, p):
    """Two-level OMF2: the fermion force on the outer level, each outer drift
    integrated by p['n_gauge'] inner OMF2 steps of the gauge force."""
    lam = p["lambda"]

    def gauge_kick(P, U, e):
        return P + e * gauge_force(dims, U, p["beta"])

    def link_drift(P, U, e):
        return link_update(U, P, e)

    def outer_drift(P, U, t):
        return omf2(P, U, t / p["n_gauge"], p["n_gauge"], lam, gauge_kick, link_drift)

    def fermion_kick(P, U, e):
        if phi is None:
            return P
        return P + e * fermion_force(dims, bc, U, p["mass"], p["r_md"], phi, p["tol_md"])

    # the outer drift returns (P, U): inner gauge kicks change P as well
    P = fermion_kick(P, U, lam * p["h"])
    for k in range(p["n_steps"]):
        P, U = outer_drift(P, U, 0.5 * p["h"])
        P = fermion_kick(P, U, (1.0 - 2.0 * lam) * p["h"])
        P, U = outer_drift(P, U, 0.5 * p["h"])
        P = fermion_kick(P, U, (2.0 if k < p["n_steps"] - 1 else 1.0) * lam * p["h"])
    return U, P


def trajectory(dims, bc, U, P, eta, p):
    """One RHMC trajectory. p: beta, mass, tau, n_steps, n_gauge, lambda,
    r_hb, r_acc, r_md (RationalApprox), tol_hb, tol_md. eta = None runs pure
    gauge HMC. Returns dict(U, P, H0, H1, dH, ...)."""
    p = dict(p)
    p["h"] = p["tau"] / p["n_steps"]
    if eta is not None:
        phi, _ = O.rational_apply(dims, bc, U, p["mass"], p["r_hb"].a0, p["r_hb"].alpha,
                                  p["r_hb"].beta, eta, tol=p["tol_hb"])
        Sf0 = fermion_action(dims, bc, U, p["mass"], p["r_acc"], phi, p["tol_hb"])
    else:
        phi, Sf0 = None, 0.0
    K0, Sg0 = kinetic(P), wilson_action(dims, U, p["beta"])
    U1, P1 = md(dims, bc, U, P, phi, p)
    K1, Sg1 = kinetic(P1), wilson_action(dims, U1, p["beta"])
    Sf1 = fermion_action(dims, bc, U1, p["mass"], p["r_acc"], phi, p["tol_hb"]) \
        if phi is not None else 0.0
    H0, H1 = K0 + Sg0 + Sf0, K1 + Sg1 + Sf1
    return dict(U=U1, P=P1, phi=phi, H0=H0, H1=H1, dH=H1 - H0, K0=K0, K1=K1, Sg0=Sg0,
                Sg1=Sg1, Sf0=Sf0, Sf1=Sf1)
