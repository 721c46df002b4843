"""Atomistic spin dynamics on a simple-cubic lattice in FP64 (oracle; test
infrastructure only).

* Spin-averaged macrocells, Eq. (9) (Sec. IV): a cubic macrocell of edge
  h = macro * a holds N_S = macro^3 spins and carries
      M = (1/h^3) sum_j S_j = mu_s mu_B / (a^3 N_S) * sum_j S^_j   (A/m);
  the demagnetizing field of Eq. (1) is evaluated on the macrocell mesh and
  applied equally to every spin of the macrocell.
* Nearest-neighbour exchange, Eq. (7): H_ex,i = J/(mu0 mu_B mu_s) sum_nn S^_j,
  open boundaries (a missing neighbour contributes nothing).
* Stochastic LLG, Eq. (10), at T = 0 (no thermal field), written for the unit
  spin S^ in Landau-Lifshitz form: dS^/dt = -gamma/(1+alpha^2) [S^ x H +
  alpha S^ x (S^ x H)].
* Heun: predictor S_p = S + dt f(S); corrector S + dt/2 (f(S) + f(S_p));
  the spin is renormalised once at the end of the step (the predictor is not).

Arrays are (3, nz, ny, nx) with x fastest.
"""

import numpy as np

from . import demag, llg

MU_B = 9.2740100783e-24  # J/T
MU0 = llg.MU0


def macro_average(S, macro, a, mu_s):
    """Eq. (9): macrocell magnetisation (3, nz/m, ny/m, nx/m) from unit spins S."""
    S = np.asarray(S, dtype=np.float64)
    _, nz, ny, nx = S.shape
    m = int(macro)
    blocks = S.reshape(3, nz // m, m, ny // m, m, nx // m, m).sum(axis=(2, 4, 6))
    return mu_s * MU_B / (a**3 * m**3) * blocks


def broadcast_macro(Hm, macro):
    """Apply each macrocell's field to every spin it holds."""
    m = int(macro)
    return np.repeat(np.repeat(np.repeat(Hm, m, axis=1), m, axis=2), m, axis=3)


def exchange_field(S, J, mu_s):
    """Eq. (7) with open boundaries."""
    S = np.asarray(S, dtype=np.float64)
    acc = np.zeros_like(S)
    for axis in (1, 2, 3):
        n = S.shape[axis]
        if n == 1:
            continue
        lo = [slice(None)] * 4
        hi = [slice(None)] * 4
        lo[axis] = slice(0, n - 1)
        hi[axis] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        acc[lo] += S[hi]
        acc[hi] += S[lo]
    return J / (MU0 * MU_B * mu_s) * acc


class Atomistic:
    """Spins n = (nx, ny, nz) on a simple-cubic lattice of constant a (m)."""

    def __init__(self, n, a, macro, J, mu_s, alpha, gamma=llg.GAMMA,
                 Hzee=(0.0, 0.0, 0.0), workers=None, kind="newell"):
        self.n = tuple(int(v) for v in n)
        self.a, self.macro = float(a), int(macro)
        self.J, self.mu_s, self.alpha, self.gamma = float(J), float(mu_s), float(alpha), float(gamma)
        self.Hzee = np.asarray(Hzee, dtype=np.float64).reshape(3, 1, 1, 1)
        nm = tuple(v // self.macro for v in self.n)
        h = self.macro * self.a
        # kind "newell": demagnetizing field of the macrocells (Eq. 9 into Eq. 1);
        # kind "dipole" with macro = 1: the lattice dipole-dipole field of Eq. (8)
        self.demag = demag.DemagFFT(nm, (h, h, h), workers, kind)

    def field(self, S):
        Hd = self.demag(macro_average(S, self.macro, self.a, self.mu_s))
        return (exchange_field(S, self.J, self.mu_s) + broadcast_macro(Hd, self.macro)
                + self.Hzee)

    def rhs(self, S):
        return llg.llg_rhs(S, self.field(S), self.alpha, self.gamma)

    def heun_step(self, S, dt):
        S = np.asarray(S, dtype=np.float64)
        f0 = self.rhs(S)
        Sp = S + dt * f0
        out = S + 0.5 * dt * (f0 + self.rhs(Sp))
        return out / np.linalg.norm(out, axis=0, keepdims=True)

    def run(self, S, dt, nsteps):
        for _ in range(nsteps):
            S = self.heun_step(S, dt)
        return S
