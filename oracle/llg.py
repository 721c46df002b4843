"""Micromagnetic exchange, LLG right-hand side and RK4 in FP64 (oracle; test
infrastructure only).

* Exchange field, Eq. (4) (Sec. III): H_ex = 2A/(mu0 Ms) * lap(m), with the
  7-point Laplacian sum_d (m[i+e_d] - 2 m[i] + m[i-e_d]) / h_d^2.  The paper
  states no boundary condition; free (Neumann) boundaries are taken: a missing
  neighbour is replaced by m[i] itself, so it contributes nothing.  Along a
  periodic axis (Sec. II, periodic boundary conditions) the neighbours wrap
  around: the first and last cells are neighbours.  An axis with a single cell
  contributes no term.
* LLG, Eq. (5), rewritten in explicit Landau-Lifshitz form:
      dm/dt = -gamma/(1+alpha^2) * [m x H + alpha m x (m x H)].
* Effective field (Sec. III): H_eff = H_d + H_ex + H_Zee (constant Zeeman).
* RK4 (Sec. III): the classic four-stage scheme; H_d is recomputed at every
  stage; m is renormalised to unit length once, at the end of each step.

gamma is a parameter; its default is mu0 * gamma_e = 2.21276e5 m/(A s)
(the paper gives no value).

Demagnetizing-field extrapolation (Sec. III): the demagnetizing field at the RK
sub-steps can be taken from a polynomial through previously computed values, a
quartic for RK4.  The scheme itself is not printed; the reading used here
(``LLGExtrapolated``): each step evaluates H_d once, at its start, from m_n; the
sub-steps at t_n + dt/2 (twice) and t_n + dt take H_d from the quartic in time
through the five most recent step-start values H_d(t_n), ..., H_d(t_{n-4}).
Until five such values exist the steps are plain RK4 (every stage evaluated);
a change of dt starts the history afresh (the nodes are dt apart).
"""

import numpy as np

from . import demag
from . import pbc as pbc_mod

MU0 = 4e-7 * np.pi
GAMMA = 2.21276e5  # mu0 * 1.76086e11, m/(A s)


def exchange_field(m, cell, A, Ms, pbc=(False, False, False)):
    """H_ex = 2A/(mu0 Ms) lap(m); m is (3, nz, ny, nx); free boundaries except
    along the axes (x, y, z) flagged in pbc, which wrap around."""
    m = np.asarray(m, dtype=np.float64)
    dx, dy, dz = cell
    lap = np.zeros_like(m)
    for axis, h, per in ((3, dx, pbc[0]), (2, dy, pbc[1]), (1, dz, pbc[2])):
        n = m.shape[axis]
        if n == 1:
            continue
        if per:
            lap += (np.roll(m, -1, axis) + np.roll(m, 1, axis) - 2.0 * m) / (h * h)
            continue
        fwd = np.zeros_like(m)  # m[i+1] - m[i], zero at the last cell
        bwd = np.zeros_like(m)  # m[i-1] - m[i], zero at the first cell
        sl_lo = [slice(None)] * 4
        sl_hi = [slice(None)] * 4
        sl_lo[axis] = slice(0, n - 1)
        sl_hi[axis] = slice(1, n)
        sl_lo, sl_hi = tuple(sl_lo), tuple(sl_hi)
        fwd[sl_lo] = m[sl_hi] - m[sl_lo]
        bwd[sl_hi] = m[sl_lo] - m[sl_hi]
        lap += (fwd + bwd) / (h * h)
    return 2.0 * A / (MU0 * Ms) * lap


def llg_rhs(m, H, alpha, gamma=GAMMA):
    """Landau-Lifshitz form of Eq. (5); m and H are (3, ...) arrays."""
    mxH = np.cross(m, H, axis=0)
    mxmxH = np.cross(m, mxH, axis=0)
    return -gamma / (1.0 + alpha * alpha) * (mxH + alpha * mxmxH)


class LLG:
    """Thin-film LLG problem: mesh n = (nx, ny, nz), cell (dx, dy, dz) in m."""

    def __init__(self, n, cell, Ms, A, alpha, gamma=GAMMA, Hzee=(0.0, 0.0, 0.0),
                 workers=None, demag_on=True, pbc=(False, False, False), images=None):
        self.n = tuple(int(v) for v in n)
        self.cell = tuple(float(c) for c in cell)
        self.Ms, self.A, self.alpha, self.gamma = float(Ms), float(A), float(alpha), float(gamma)
        self.Hzee = np.asarray(Hzee, dtype=np.float64).reshape(3, 1, 1, 1)
        self.pbc = tuple(bool(p) for p in pbc)
        if not demag_on:
            self.demag = None
        elif any(self.pbc):
            images = pbc_mod.DEFAULT_IMAGES if images is None else images
            self.demag = pbc_mod.DemagPBC(self.n, self.cell, self.pbc, images, workers)
        else:
            self.demag = demag.DemagFFT(self.n, self.cell, workers)

    def field(self, m):
        H = exchange_field(m, self.cell, self.A, self.Ms, self.pbc) + self.Hzee
        if self.demag is not None:
            H = H + self.demag(self.Ms * m)
        return H

    def rhs(self, m):
        return llg_rhs(m, self.field(m), self.alpha, self.gamma)

    def rk4_step(self, m, dt):
        m = np.asarray(m, dtype=np.float64)
        k1 = self.rhs(m)
        k2 = self.rhs(m + 0.5 * dt * k1)
        k3 = self.rhs(m + 0.5 * dt * k2)
        k4 = self.rhs(m + dt * k3)
        out = m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return out / np.linalg.norm(out, axis=0, keepdims=True)

    def run(self, m, dt, nsteps):
        for _ in range(nsteps):
            m = self.rk4_step(m, dt)
        return m

    def energy(self, m):
        """Exchange + demag + Zeeman energy (J) of the discrete system:
        E = -mu0 Ms V sum_i m_i . (H_ex/2 + H_d/2 + H_zee)."""
        V = float(np.prod(self.cell))
        Hhalf = 0.5 * exchange_field(m, self.cell, self.A, self.Ms, self.pbc)
        if self.demag is not None:
            Hhalf = Hhalf + 0.5 * self.demag(self.Ms * m)
        Hhalf = Hhalf + self.Hzee
        return float(-MU0 * self.Ms * V * np.sum(m * Hhalf))


def quartic_extrapolate(history, theta):
    """Value at t_n + theta dt of the degree-4 polynomial in t through the five
    values history = [F(t_n), F(t_n - dt), ..., F(t_n - 4 dt)] (any array shape):
    least-squares fit of a degree-4 polynomial through five points, which is
    the interpolating polynomial, evaluated at theta."""
    h = np.stack([np.asarray(v, dtype=np.float64) for v in history])
    nodes = -np.arange(5, dtype=np.float64)          # in units of dt, t_n at 0
    coef = np.polynomial.polynomial.polyfit(nodes, h.reshape(5, -1), 4)
    val = np.polynomial.polynomial.polyval(theta, coef)
    return val.reshape(h.shape[1:])


class LLGExtrapolated(LLG):
    """RK4 with one demagnetizing-field evaluation per step (quartic extrapolation
    at the sub-steps once five step-start values exist; plain RK4 before)."""

    def __init__(self, *args, **kwargs):
        super().__init__(*args, **kwargs)
        self.history = []   # H_d at the starts of the most recent steps, newest first
        self.history_dt = None

    def _field_with(self, m, Hd):
        return exchange_field(m, self.cell, self.A, self.Ms, self.pbc) + self.Hzee + Hd

    def rk4_step(self, m, dt):
        m = np.asarray(m, dtype=np.float64)
        if dt != self.history_dt:
            self.history, self.history_dt = [], dt
        Hd0 = self.demag(self.Ms * m)
        self.history = [Hd0] + self.history[:4]
        rhs = lambda mm, Hd: llg_rhs(mm, self._field_with(mm, Hd), self.alpha, self.gamma)
        k1 = rhs(m, Hd0)
        if len(self.history) == 5:
            Hhalf = quartic_extrapolate(self.history, 0.5)
            Hfull = quartic_extrapolate(self.history, 1.0)
            m2 = m + 0.5 * dt * k1
            k2 = rhs(m2, Hhalf)
            m3 = m + 0.5 * dt * k2
            k3 = rhs(m3, Hhalf)
            m4 = m + dt * k3
            k4 = rhs(m4, Hfull)
        else:
            k2 = self.rhs(m + 0.5 * dt * k1)
            k3 = self.rhs(m + 0.5 * dt * k2)
            k4 = self.rhs(m + dt * k3)
        out = m + dt / 6.0 * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        return out / np.linalg.norm(out, axis=0, keepdims=True)


def macrospin_closed_form(theta0, phi0, H, alpha, t, gamma=GAMMA):
    """Single moment in a constant field H along +z (LL form):
    tan(theta/2) = tan(theta0/2) exp(-alpha gamma H t/(1+alpha^2)),
    phi = phi0 + gamma H t/(1+alpha^2).  Returns the unit vector (3,)."""
    g = gamma * H / (1.0 + alpha * alpha)
    theta = 2.0 * np.arctan(np.tan(theta0 / 2.0) * np.exp(-alpha * g * t))
    phi = phi0 + g * t
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])
