"""Writes free_field_4444.txt: the spectrum of the even-site staggered
operator A = m^2 - D_eo D_oe at U = 1 on a 4^4 lattice, from its closed form.

At U = 1 the staggered operator is diagonalised by plane waves; every
momentum p (p_mu = 2 pi k / 4, shifted by pi / 4 in t for an antiperiodic
boundary) gives A = m^2 + sum_mu sin^2 p_mu. The even-site restriction keeps
half of the 3 * 256 colour-site states, so each momentum's eigenvalue counts
3 / 2 times. This enumerates the momenta (no lattice code, no oracle) and
stores eigenvalue - m^2 with its multiplicity, per boundary condition.
Run from the repository root: python tests/golden/make_free_field.py
"""
import itertools
import math
import os
from collections import Counter

L = 4


def spectrum(antiperiodic_t):
    c = Counter()
    for k in itertools.product(range(L), repeat=4):
        p = [2 * math.pi * k[mu] / L for mu in range(4)]
        if antiperiodic_t:
            p[3] += math.pi / L
        c[round(sum(math.sin(x) ** 2 for x in p), 12)] += 3
    return {lam: mult // 2 for lam, mult in sorted(c.items())}


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_field_4444.txt")
    lines = ["# Even-site staggered operator A = m^2 - D_eo D_oe at U = 1 on a 4^4 lattice:",
             "# eigenvalue minus m^2, and its multiplicity (384 states per boundary condition).",
             "# Closed form A(p) = m^2 + sum_mu sin^2 p_mu of the free staggered operator (the",
             "# operator the paper's RHMC acts with); written by make_free_field.py.",
             "# bc shift multiplicity"]
    for name, anti in (("periodic", False), ("antiperiodic_t", True)):
        for lam, mult in spectrum(anti).items():
            lines.append("%s %.12g %d" % (name, lam, mult))
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
