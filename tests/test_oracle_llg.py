"""Pins for the oracle's micromagnetic step (Eqs. 4 and 5; RK4, Sec. III) and its
atomistic step (Eqs. 7, 9 and 10; Heun, Sec. IV)."""

import numpy as np
import pytest

import workloads as W
from oracle import atomistic, demag, llg

CELL = (4e-9, 4e-9, 4e-9)


def _unit(theta, phi):
    return np.array([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi), np.cos(theta)])


def test_macrospin_closed_form():
    """One cubic cell in a field along z: its demag field is -M/3 (no torque), so the
    moment follows the closed-form damped precession."""
    Hz, alpha = 5e4, 0.1
    prob = llg.LLG((1, 1, 1), CELL, W.MS, W.A_EX, alpha, Hzee=(0, 0, Hz))
    m0 = _unit(1.2, 0.3).reshape(3, 1, 1, 1)
    dt, steps = 2e-14, 500
    m = prob.run(m0, dt, steps)
    ref = llg.macrospin_closed_form(1.2, 0.3, Hz, alpha, dt * steps)
    np.testing.assert_allclose(m[:, 0, 0, 0], ref, atol=1e-10)


def test_rk4_is_fourth_order():
    prob = llg.LLG((1, 1, 1), CELL, W.MS, W.A_EX, 0.05, Hzee=(0, 0, 2e5))
    m0 = _unit(1.0, 0.0).reshape(3, 1, 1, 1)
    T = 4e-11
    ref = llg.macrospin_closed_form(1.0, 0.0, 2e5, 0.05, T)
    errs = []
    for steps in (25, 50, 100):
        m = prob.run(m0, T / steps, steps)
        errs.append(np.linalg.norm(m[:, 0, 0, 0] - ref))
    for e1, e2 in zip(errs, errs[1:]):
        assert 12.0 < e1 / e2 < 20.0, errs


def test_uniform_m_has_no_exchange_field():
    m = np.broadcast_to(_unit(0.7, 2.0).reshape(3, 1, 1, 1), (3, 3, 5, 6)).copy()
    np.testing.assert_array_equal(llg.exchange_field(m, CELL, W.A_EX, W.MS), 0.0)


def test_exchange_neumann_eigenmode():
    """cos(k (i + 1/2) h) with k = pi p/(n h) is an eigenvector of the free-boundary
    7-point Laplacian with eigenvalue -sum_d (2 - 2 cos(k_d h_d))/h_d^2."""
    n = (12, 7, 3)
    cell = (4e-9, 3e-9, 5e-9)
    p = (3, 2, 1)
    k = [np.pi * p[d] / (n[d] * cell[d]) for d in range(3)]
    zz, yy, xx = np.meshgrid(*(np.arange(v) for v in (n[2], n[1], n[0])), indexing="ij")
    mode = (np.cos(k[0] * (xx + 0.5) * cell[0]) * np.cos(k[1] * (yy + 0.5) * cell[1])
            * np.cos(k[2] * (zz + 0.5) * cell[2]))
    m = np.stack([mode, 0.5 * mode, -mode])
    lam = -sum((2 - 2 * np.cos(k[d] * cell[d])) / cell[d] ** 2 for d in range(3))
    H = llg.exchange_field(m, cell, W.A_EX, W.MS)
    np.testing.assert_allclose(H, 2 * W.A_EX / (llg.MU0 * W.MS) * lam * m, rtol=1e-10, atol=1e-3)


def test_llg_rhs_is_perpendicular_and_damps():
    rng = np.random.default_rng(0)
    m = W.unit_vectors((2, 3, 4), 5).astype(np.float64)
    H = rng.standard_normal(m.shape) * 1e5
    f = llg.llg_rhs(m, H, 0.1)
    np.testing.assert_allclose(np.sum(f * m, axis=0), 0.0, atol=1e-3)
    assert np.all(np.sum(f * H, axis=0) >= -1e-3)  # dE/dt = -mu0 Ms H.dm/dt <= 0


def test_energy_decreases_with_damping():
    n = (10, 8, 2)
    prob = llg.LLG(n, CELL, W.MS, W.A_EX, alpha=0.5)
    m = W.unit_vectors((n[2], n[1], n[0]), 4).astype(np.float64)
    E = [prob.energy(m)]
    for _ in range(15):
        m = prob.rk4_step(m, 2e-14)
        E.append(prob.energy(m))
    assert all(b <= a + 1e-12 * abs(a) for a, b in zip(E, E[1:])), E
    np.testing.assert_allclose(np.linalg.norm(m, axis=0), 1.0, atol=1e-14)


# ----------------------------------------------------------------- atomistic ----
def test_macrocell_moment_conservation():
    """Eq. (9): sum over macrocells of M h^3 equals the total moment mu_s mu_B sum S."""
    S = W.unit_vectors((8, 8, 12), 1).astype(np.float64)
    a, macro, mu_s = 0.4e-9, 4, 1.7
    Mm = atomistic.macro_average(S, macro, a, mu_s)
    h3 = (macro * a) ** 3
    np.testing.assert_allclose(Mm.reshape(3, -1).sum(axis=1) * h3,
                               mu_s * atomistic.MU_B * S.reshape(3, -1).sum(axis=1),
                               rtol=1e-12)


def test_atomistic_exchange_counts_neighbours():
    S = np.zeros((3, 3, 3, 3))
    S[2] = 1.0
    H = atomistic.exchange_field(S, 1e-21, 1.0)
    pref = 1e-21 / (atomistic.MU0 * atomistic.MU_B)
    # centre has 6 neighbours, a corner 3, an edge 4, a face centre 5
    assert np.isclose(H[2, 1, 1, 1], 6 * pref)
    assert np.isclose(H[2, 0, 0, 0], 3 * pref)
    assert np.isclose(H[2, 0, 0, 1], 4 * pref)
    assert np.isclose(H[2, 0, 1, 1], 5 * pref)
    # uniform state: exchange field parallel to the spins, no torque
    np.testing.assert_allclose(np.cross(S, H, axis=0), 0.0)


def test_atomistic_single_spin_closed_form():
    Hz, alpha = 3e5, 0.05
    prob = atomistic.Atomistic((1, 1, 1), 0.4e-9, 1, 1e-21, 1.0, alpha, Hzee=(0, 0, Hz))
    S0 = _unit(0.9, 1.0).reshape(3, 1, 1, 1)
    dt, steps = 2e-16, 400
    S = prob.run(S0, dt, steps)
    ref = llg.macrospin_closed_form(0.9, 1.0, Hz, alpha, dt * steps)
    np.testing.assert_allclose(S[:, 0, 0, 0], ref, atol=2e-7)


def test_heun_is_second_order():
    Hz, alpha = 3e5, 0.05
    prob = atomistic.Atomistic((1, 1, 1), 0.4e-9, 1, 1e-21, 1.0, alpha, Hzee=(0, 0, Hz))
    S0 = _unit(0.9, 1.0).reshape(3, 1, 1, 1)
    T = 2e-11
    ref = llg.macrospin_closed_form(0.9, 1.0, Hz, alpha, T)
    errs = [np.linalg.norm(prob.run(S0, T / s, s)[:, 0, 0, 0] - ref) for s in (50, 100, 200)]
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.2 < e1 / e2 < 4.8, errs


def test_atomistic_demag_is_macrocell_demag():
    """With J = 0 and no Zeeman, the field on every spin is the macrocell H_d."""
    n, a, macro = (8, 4, 4), 0.4e-9, 2
    S = W.unit_vectors((n[2], n[1], n[0]), 9).astype(np.float64)
    prob = atomistic.Atomistic(n, a, macro, 0.0, 2.0, 0.1)
    H = prob.field(S)
    Mm = atomistic.macro_average(S, macro, a, 2.0)
    h = macro * a
    Hm = demag.demag_direct(Mm, (h, h, h))
    np.testing.assert_allclose(H[:, ::macro, ::macro, ::macro], Hm, rtol=1e-10, atol=1e-6)
    np.testing.assert_allclose(H[:, 1::macro, 1::macro, 1::macro], Hm, rtol=1e-10, atol=1e-6)


# ---------------------------------------------------------------- H_d extrapolation
def test_quartic_extrapolation_is_exact_for_quartics_only():
    """The sub-step field is the degree-4 polynomial through five step-start values:
    exact for any polynomial of degree <= 4 in time, not for degree 5."""
    rng = np.random.default_rng(4)
    for deg in (0, 2, 3, 4):
        c = rng.standard_normal((deg + 1, 3, 2, 2))
        F = lambda s: sum(c[k] * s ** k for k in range(deg + 1))
        hist = [F(-j) for j in range(5)]
        for theta in (0.5, 1.0, 2.5):
            np.testing.assert_allclose(llg.quartic_extrapolate(hist, theta), F(theta), rtol=0, atol=1e-10)
    F5 = lambda s: s ** 5
    assert abs(float(llg.quartic_extrapolate([F5(-j) for j in range(5)], 1.0)) - 1.0) > 1.0
    # one step ahead the weights are the binomial ones 5, -10, 10, -5, 1
    e = np.eye(5)
    w = [float(llg.quartic_extrapolate(list(e[j]), 1.0)) for j in range(5)]
    np.testing.assert_allclose(w, [5, -10, 10, -5, 1], atol=1e-9)


def test_extrapolated_rk4_starts_as_plain_rk4():
    n = (8, 8, 2)
    m0 = W.unit_vectors((2, 8, 8), 3).astype(np.float64)
    a = llg.LLG(n, W.CELL_4NM, W.MS, W.A_EX, 0.02).run(m0, 1e-13, 4)
    b = llg.LLGExtrapolated(n, W.CELL_4NM, W.MS, W.A_EX, 0.02).run(m0, 1e-13, 4)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-13)


def test_extrapolated_rk4_keeps_fourth_order():
    """Against a fine-step plain RK4 reference, the error of RK4 with quartic H_d
    extrapolation falls ~16x per halving of dt and stays within 2x of plain RK4
    (the extrapolation costs no accuracy order)."""
    n = (16, 16, 2)
    m0 = W.unit_vectors((2, 16, 16), 3).astype(np.float64)
    T = 8e-12
    ref = llg.LLG(n, W.CELL_4NM, W.MS, W.A_EX, 0.02).run(m0, T / 640, 640)
    scale = np.linalg.norm(ref - m0)
    errs = []
    for dt in (4e-13, 2e-13, 1e-13):
        ns = int(round(T / dt))
        plain = llg.LLG(n, W.CELL_4NM, W.MS, W.A_EX, 0.02).run(m0, dt, ns)
        extr = llg.LLGExtrapolated(n, W.CELL_4NM, W.MS, W.A_EX, 0.02).run(m0, dt, ns)
        e_plain = np.linalg.norm(plain - ref) / scale
        e_extr = np.linalg.norm(extr - ref) / scale
        assert e_extr <= 2.0 * e_plain, (dt, e_extr, e_plain)
        errs.append(e_extr)
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs


def _num_grad(E, x, idx, eps):
    """Central difference of the scalar E at the entries idx of x (exact up to
    rounding for a quadratic E)."""
    g = []
    for i in idx:
        xp, xm = x.copy(), x.copy()
        xp[i] += eps
        xm[i] -= eps
        g.append((E(xp) - E(xm)) / (2 * eps))
    return np.array(g)


@pytest.mark.parametrize("pbc", [(False, False, False), (True, False, True)])
def test_exchange_field_is_the_energy_gradient(pbc):
    """Eq. (4) from the exchange energy it derives from: E = A int |grad m|^2 dV,
    discretised as A V sum over neighbour pairs |m_j - m_i|^2 / h^2 (each pair
    once, pairs across a periodic boundary included), so that
    H_ex = -dE/dm_i / (mu0 Ms V).  The field is differentiated numerically from
    the energy, so the prefactor 2A/(mu0 Ms) and the free-boundary rule are
    checked, not restated."""
    n = (6, 5, 4)
    cell = (4e-9, 3e-9, 2.5e-9)
    V = cell[0] * cell[1] * cell[2]
    rng = np.random.default_rng(11)
    m = rng.standard_normal((3, n[2], n[1], n[0]))

    def energy(mm):
        e = 0.0
        for axis, h, per in ((3, cell[0], pbc[0]), (2, cell[1], pbc[1]), (1, cell[2], pbc[2])):
            d = np.diff(mm, axis=axis)
            e += np.sum(d * d) / h**2
            if per:
                first = np.take(mm, [0], axis=axis)
                last = np.take(mm, [mm.shape[axis] - 1], axis=axis)
                e += np.sum((first - last) ** 2) / h**2
        return W.A_EX * V * e

    H = llg.exchange_field(m, cell, W.A_EX, W.MS, pbc=pbc)
    idx = [(c, z, y, x) for c in range(3) for (z, y, x) in
           ((0, 0, 0), (3, 4, 5), (1, 2, 3), (0, 4, 2), (2, 0, 5))]
    g = _num_grad(energy, m, idx, 1e-3)
    expect = -g / (llg.MU0 * W.MS * V)
    got = np.array([H[i] for i in idx])
    np.testing.assert_allclose(got, expect, rtol=1e-6, atol=1e-6 * np.abs(expect).max())


def test_atomistic_exchange_is_the_energy_gradient():
    """Eq. (7) from the Heisenberg energy E = -J sum over nearest-neighbour pairs
    S_i . S_j (open boundaries): H_i = -dE/dS_i / (mu0 mu_s mu_B), with mu_B the
    Bohr magneton; differentiated numerically."""
    n = (5, 4, 3)
    J, mu_s = 1e-21, 2.0
    mu_b = 9.2740100783e-24  # Bohr magneton, J/T (CODATA 2018)
    rng = np.random.default_rng(12)
    S = rng.standard_normal((3, n[2], n[1], n[0]))

    def energy(s):
        e = 0.0
        for axis in (1, 2, 3):
            a = np.take(s, range(s.shape[axis] - 1), axis=axis)
            b = np.take(s, range(1, s.shape[axis]), axis=axis)
            e += np.sum(a * b)
        return -J * e

    H = atomistic.exchange_field(S, J, mu_s)
    idx = [(c, z, y, x) for c in range(3) for (z, y, x) in ((0, 0, 0), (1, 2, 3), (2, 3, 4), (1, 0, 2))]
    g = _num_grad(energy, S, idx, 1e-3)
    expect = -g / (llg.MU0 * mu_s * mu_b)
    got = np.array([H[i] for i in idx])
    np.testing.assert_allclose(got, expect, rtol=1e-6, atol=1e-6 * np.abs(expect).max())
