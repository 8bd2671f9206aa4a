"""The five synthetic workloads (lattice, field, mass, n_pf, poles, precision).

Each workload names: lattice extents (x,y,z,t), the disorder eps of the seeded
field U = exp(i eps H), the staggered mass m, the number n_pf of pseudofermions
(block width), the exponent p of r(x) ~ x^(-p) and the number of poles of its
partial-fraction form, fitted on [m^2, 16 + m^2] (the spectrum of A = M^dag M
on even sites lies there since |D| <= 4), the solver tolerance and precision.

The paper's own run (Sec. IV) is Nf=4 staggered on 8^4 at am=0.002 with
thermalised fields; these workloads use heavier masses and seeded fields.
Boundary conditions: periodic in x, y, z and antiperiodic in t.

Seeds: gauge field seed = 1000*id, pseudofermion block seed = 1000*id + 1,
batch member k gauge/block seeds = 1000*id + 10*(k+1) (+1).
"""
import json
import os

from . import rational

BC_DEFAULT = (1, 1, 1, -1)

WORKLOADS = {
    "c1": dict(id=1, dims=(4, 4, 4, 4), eps=0.3, mass=0.1, n=1, power=0.5, poles=8,
               tol=1e-10, precision="f64"),
    "c2": dict(id=2, dims=(8, 8, 8, 8), eps=0.5, mass=0.05, n=4, power=1.0 / 8, poles=12,
               tol=1e-10, precision="f64"),
    "c3": dict(id=3, dims=(16, 16, 16, 16), eps=0.7, mass=0.02, n=8, power=1.0 / 16, poles=16,
               tol=1e-10, precision="mixed", reliable=50),
    "c4": dict(id=4, dims=(16, 16, 16, 32), eps=0.7, mass=0.02, n=8, power=1.0 / 16, poles=16,
               tol=1e-10, precision="f64"),
    "c5": dict(id=5, dims=(32, 32, 32, 32), eps=0.8, mass=0.01, n=16, power=1.0 / 32, poles=20,
               tol=1e-10, precision="mixed", reliable=50,
               batch=[(8, 8, 8, 8), (16, 16, 16, 16), (24, 24, 24, 24)]),
}

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coefficients.json")


def _key(power, lo, hi, n):
    return "%.17g|%.17g|%.17g|%d" % (power, lo, hi, n)


def coefficients(power, lo, hi, n):
    """Rational coefficients, read from the committed cache when present."""
    if os.path.exists(_CACHE):
        with open(_CACHE) as f:
            tab = json.load(f)
        d = tab.get(_key(power, lo, hi, n))
        if d is not None:
            return rational.RationalApprox(d["power"], d["lo"], d["hi"], d["a0"], d["alpha"],
                                           d["beta"], d["error"])
    return rational.remez(power, lo, hi, n)


def workload_coefficients(name):
    w = WORKLOADS[name]
    m2 = w["mass"] ** 2
    return coefficients(w["power"], m2, 16.0 + m2, w["poles"])


# Heatbath and accept-step fits (Sec. II: the pseudofermions are drawn as
# phi = [M^dag M]^(+p/2) eta from Gaussian eta, so that the action
# phi^dag [M^dag M]^(-p) phi equals eta^dag eta; Sec. IV runs these solves at
# residual 1e-14 with rational approximations of relative error below 1e-15).
# The pole counts reach that error on the workload's spectrum interval.
HMC_FITS = {
    "c2": dict(heatbath_poles=20, accept_poles=21),
}


def heatbath_coefficients(name):
    """r_hb(x) ~ x^(+p/2) for the workload's action exponent p."""
    w = WORKLOADS[name]
    m2 = w["mass"] ** 2
    return coefficients(-0.5 * w["power"], m2, 16.0 + m2, HMC_FITS[name]["heatbath_poles"])


def accept_coefficients(name):
    """r(x) ~ x^(-p) at the accept-step accuracy."""
    w = WORKLOADS[name]
    m2 = w["mass"] ** 2
    return coefficients(w["power"], m2, 16.0 + m2, HMC_FITS[name]["accept_poles"])


def _fits():
    """(label, power, lo, hi, poles) of every stored fit."""
    out = []
    for name, w in WORKLOADS.items():
        m2 = w["mass"] ** 2
        out.append((name, w["power"], m2, 16.0 + m2, w["poles"]))
    for name, h in HMC_FITS.items():
        w = WORKLOADS[name]
        m2 = w["mass"] ** 2
        out.append((name + " heatbath", -0.5 * w["power"], m2, 16.0 + m2, h["heatbath_poles"]))
        out.append((name + " accept", w["power"], m2, 16.0 + m2, h["accept_poles"]))
    return out


def write_cache(only_missing=True):
    """Fit the coefficients and store them (run as a script). Entries already
    in the cache are kept unless only_missing is False."""
    tab = {}
    if only_missing and os.path.exists(_CACHE):
        with open(_CACHE) as f:
            tab = json.load(f)
    for label, power, lo, hi, poles in _fits():
        key = _key(power, lo, hi, poles)
        if key in tab:
            continue
        r = rational.remez(power, lo, hi, poles)
        tab[key] = r.as_dict()
        print(label, "poles", poles, "relative error %.3e" % r.error, flush=True)
    with open(_CACHE, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    import sys
    write_cache(only_missing="--all" not in sys.argv)
