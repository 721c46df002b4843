"""Writes aharoni_prism.txt: Aharoni's closed-form prism demagnetizing factor
(J. Appl. Phys. 83, 3432 (1998), Eq. 1), an expression independent of Newell's
f/g functions.  Run: python tests/golden/make_aharoni.py"""
import os

from numpy import arctan, log, pi, sqrt


def aharoni_dz(a, b, c):
    """D_z of a 2a x 2b x 2c prism (c along z)."""
    r = sqrt(a * a + b * b + c * c)
    ab, bc, ac = sqrt(a * a + b * b), sqrt(b * b + c * c), sqrt(a * a + c * c)
    s = ((b * b - c * c) / (2 * b * c) * log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * log((r - b) / (r + b))
         + b / (2 * c) * log((ab + a) / (ab - a)) + a / (2 * c) * log((ab + b) / (ab - b))
         + c / (2 * a) * log((bc - b) / (bc + b)) + c / (2 * b) * log((ac - a) / (ac + a))
         + 2 * arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) / (3 * a * b * c) * r
         + c / (a * b) * (ac + bc)
         - (ab ** 3 + bc ** 3 + ac ** 3) / (3 * a * b * c))
    return s / pi


CASES = [(1, 1, 1), (4, 4, 1), (1, 0.7, 0.4), (3, 2, 5), (50, 50, 1), (64, 64, 2), (0.5, 2, 1)]

if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "aharoni_prism.txt")
    header = [ln for ln in open(path) if ln.startswith("#")]
    with open(path, "w") as f:
        f.writelines(header)
        for a, b, c in CASES:
            f.write(f"{a!r} {b!r} {c!r} {aharoni_dz(a, b, c):.17g}\n")
