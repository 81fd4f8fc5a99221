"""Oracle lattice constants: generator for ``oracle/lattice_constants.h``.

TEST INFRASTRUCTURE ONLY.  This script belongs to the CPU oracle; the HIP
library derives its own constants with code of its own and never reads the
header written here.

What it computes (Sec. 5 and Appendix A, Table "Model Parameters D2Q37"):

* D2Q9 (not in the paper; the textbook degree-5 Gauss-Hermite rule):
  theta = 1/3, weights 4/9, 1/9, 1/36.
* D2Q37: the velocity abscissae of the appendix table, in lattice units
  (v_i / c integer, c = 1 so theta = 1/c^2).  The table prints the weights
  to about 15-16 significant digits, which is not enough for a long-double
  oracle.  The eight orbit weights and theta are therefore re-derived as the
  exact solution of the nine symmetric Gauss-Hermite moment conditions of
  degree 0..8 (Sec. 5: a rule of degree d integrates the Gaussian moments
  exactly), starting Newton's method from the printed table.  The solution
  agrees with every printed weight to better than 6e-16; the tests check
  this against the printed values stored in tests/golden.

Canonical velocity order (shared by every interface that exchanges
populations): orbits in the appendix-table order, and inside an orbit the
members sorted by their polar angle in [0, 2*pi).

Run:  python oracle/gen_constants.py   (rewrites oracle/lattice_constants.h)
"""
import math
import os

import mpmath as mp

mp.mp.dps = 60

# Appendix table: orbit representatives (v/c) and printed weights.
D2Q37_ORBITS = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 2), (3, 0), (1, 2), (1, 3)]
D2Q37_PRINTED_W = [
    "0.233150669132352000", "0.107306091542219000", "0.057667859888794800",
    "0.014208216158450700", "0.001011937592673570", "0.000245301027757717",
    "0.005353049000513770", "0.000283414252994198",
]
# Footnote of the table: lattice speed c = 1.19697977039307 sqrt(theta).
D2Q37_PRINTED_C = "1.19697977039307"

D2Q9_ORBITS = [(0, 0), (1, 0), (1, 1)]


def orbit_members(a, b):
    """All images of (a, b) under the square's symmetry group, by angle."""
    pts = set()
    for p, q in ((a, b), (b, a)):
        for sx in (1, -1):
            for sy in (1, -1):
                pts.add((sx * p, sy * q))
    return sorted(pts, key=lambda v: math.atan2(v[1], v[0]) % (2 * math.pi))


def double_factorial(n):
    r = 1
    while n > 1:
        r *= n
        n -= 2
    return r


def solve_d2q37():
    """Orbit weights and theta from the degree 0..8 moment conditions."""
    members = [orbit_members(*o) for o in D2Q37_ORBITS]
    # Independent even moments of a square-symmetric rule up to degree 8.
    powers = [(0, 0), (2, 0), (4, 0), (2, 2), (6, 0), (4, 2), (8, 0), (6, 2), (4, 4)]

    def residual(*x):
        w, th = x[:8], x[8]
        out = []
        for p, q in powers:
            s = mp.mpf(0)
            for k in range(8):
                s += w[k] * sum(mp.mpf(vx) ** p * mp.mpf(vy) ** q for vx, vy in members[k])
            exact = double_factorial(p - 1) * double_factorial(q - 1) * th ** ((p + q) // 2)
            out.append(s - exact)
        return out

    c = mp.mpf(D2Q37_PRINTED_C)
    x0 = [mp.mpf(v) for v in D2Q37_PRINTED_W] + [1 / c ** 2]
    sol = mp.findroot(residual, x0, tol=mp.mpf(10) ** -55)
    return [sol[k] for k in range(8)], sol[8], members


def lattice_tables():
    """Return {Q: (velocities, weights(mpf), theta(mpf))} in canonical order."""
    out = {}
    third = mp.mpf(1) / 3
    w9 = [mp.mpf(4) / 9, mp.mpf(1) / 9, mp.mpf(1) / 36]
    vel, wt = [], []
    for k, o in enumerate(D2Q9_ORBITS):
        for m in orbit_members(*o):
            vel.append(m)
            wt.append(w9[k])
    out[9] = (vel, wt, third)
    w37, th37, members = solve_d2q37()
    vel, wt = [], []
    for k in range(8):
        for m in members[k]:
            vel.append(m)
            wt.append(w37[k])
    out[37] = (vel, wt, th37)
    return out


def _lit(x):
    return mp.nstr(x, 30, strip_zeros=False, min_fixed=-5, max_fixed=5) + "L"


def write_header(path):
    tabs = lattice_tables()
    lines = [
        "/* Oracle lattice constants, written by oracle/gen_constants.py (do not edit).",
        " * TEST INFRASTRUCTURE ONLY: used by the CPU oracle, never by the HIP library.",
        " * D2Q9: textbook degree-5 rule.  D2Q37: Appendix A table, weights and theta",
        " * refined to 30 digits from the degree 0..8 Gauss-Hermite moment conditions.",
        " * Canonical order: orbits in table order, members by polar angle. */",
        "#ifndef ORACLE_LATTICE_CONSTANTS_H",
        "#define ORACLE_LATTICE_CONSTANTS_H",
    ]
    for q in (9, 37):
        vel, wt, th = tabs[q]
        lines.append(f"static const int ORC_Q{q}_V[{q}][2] = {{")
        lines.append("  " + ", ".join(f"{{{vx}, {vy}}}" for vx, vy in vel))
        lines.append("};")
        lines.append(f"static const long double ORC_Q{q}_W[{q}] = {{")
        for w in wt:
            lines.append(f"  {_lit(w)},")
        lines.append("};")
        lines.append(f"static const long double ORC_Q{q}_THETA = {_lit(th)};")
    lines.append("#endif")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    write_header(os.path.join(here, "lattice_constants.h"))
    tabs = lattice_tables()
    print("theta37 =", mp.nstr(tabs[37][2], 25), " c =", mp.nstr(1 / mp.sqrt(tabs[37][2]), 25))
