"""Pins for the oracle's demagnetizing tensor (Sec. II, Eq. 1: "formulas in Ref. [23]").

Each check is fixed by something other than the oracle's own formulas: exact
values (cube 1/3), identities of the definition (trace, parity), an independent
published closed form (Aharoni's prism factor, tests/golden/aharoni_prism.txt),
and brute-force 6-D Gauss-Legendre quadrature of the defining double integral.
"""

import os

import numpy as np
import pytest

from oracle import newell

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "aharoni_prism.txt")

CELLS = [(1.0, 1.0, 1.0), (1.0, 0.7, 0.4), (4e-9, 4e-9, 4e-9), (2.0, 3.0, 1.5)]


def test_cube_self_term_is_one_third():
    N0 = newell.newell_near(0, 0, 0, (1.0, 1.0, 1.0))
    np.testing.assert_allclose(N0[:3], 1.0 / 3.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(N0[3:], 0.0, atol=1e-15)


@pytest.mark.parametrize("cell", CELLS)
def test_self_term_trace_is_one(cell):
    N0 = newell.newell_near(0, 0, 0, cell)
    assert abs(N0[:3].sum() - 1.0) < 1e-14


@pytest.mark.parametrize("cell,tol", [((1.0, 1.0, 1.0), 1e-8), ((1.0, 0.7, 0.4), 3e-7),
                                      ((4e-9, 4e-9, 4e-9), 1e-8), ((2.0, 3.0, 1.5), 2e-7)])
def test_trace_vanishes_away_from_origin(cell, tol):
    """trace N(r) = 0 for r != 0 (the dipole tensor is traceless).  The residual is
    the rounding noise of the near-field stencil, largest just inside the switch
    radius and larger for flat cells (more cancellation in the short axis)."""
    rng = np.random.default_rng(0)
    d = rng.integers(-40, 41, size=(3, 400))
    d = d[:, np.any(d != 0, axis=0)]
    N = newell.tensor(d[0], d[1], d[2], cell)
    scale = np.abs(N).max(axis=0)
    assert np.max(np.abs(N[:3].sum(axis=0)) / scale) < tol


def test_aharoni_prism_factors():
    """Newell's self term with cell = body equals Aharoni's independent closed form."""
    rows = np.loadtxt(GOLDEN, comments="#")
    for a, b, c, dz in rows:
        got = newell.body_factor((2 * a, 2 * b, 2 * c))[2]
        assert abs(got - dz) < 1e-13 * max(1.0, abs(dz)), (a, b, c, got, dz)
        # the same prism turned so that each axis in turn is the long one
        got_x = newell.body_factor((2 * c, 2 * b, 2 * a))[0]
        assert abs(got_x - dz) < 1e-13, (a, b, c, got_x, dz)


def _quadrature_tensor(r, cell, n=10):
    """N_ab(r) = (1/V) Int Int D_ab(r + x - y) dx dy by n-point Gauss-Legendre per
    dimension of the 6-D integral; D_ab = (delta_ab |u|^2 - 3 u_a u_b)/(4 pi |u|^5)."""
    cell = np.asarray(cell, dtype=float) / max(cell)
    g, w = np.polynomial.legendre.leggauss(n)
    X = np.asarray(r, dtype=float) * cell
    u, wt = [], []
    for d in range(3):
        xs, ys = np.meshgrid(g * cell[d] / 2, g * cell[d] / 2, indexing="ij")
        u.append((X[d] + xs - ys).ravel())
        wt.append(np.outer(w * cell[d] / 2, w * cell[d] / 2).ravel())
    Ux, Uy, Uz = np.meshgrid(*u, indexing="ij")
    W = np.einsum("i,j,k->ijk", *wt)
    R2 = Ux**2 + Uy**2 + Uz**2
    R5 = R2 * R2 * np.sqrt(R2)
    pairs = [(Ux, Ux), (Uy, Uy), (Uz, Uz), (Ux, Uy), (Ux, Uz), (Uy, Uz)]
    out = np.empty(6)
    for c, (a, b) in enumerate(pairs):
        delta = 1.0 if c < 3 else 0.0
        out[c] = np.sum(W * (delta * R2 - 3 * a * b) / (4 * np.pi * R5)) / np.prod(cell)
    return out


@pytest.mark.parametrize("r,cell", [
    ((3, 0, 0), (1, 1, 1)), ((2, 2, 1), (1, 1, 1)), ((3, -2, 1), (1, 1, 1)),
    ((-2, 1, 3), (1, 0.7, 0.4)), ((0, 4, -3), (1, 0.7, 0.4)), ((2, -3, 2), (2, 3, 1.5)),
])
def test_newell_matches_quadrature_of_definition(r, cell):
    q = _quadrature_tensor(r, cell)
    a = newell.newell_near(*r, cell)
    assert np.max(np.abs(q - a)) / np.max(np.abs(a)) < 1e-10


def test_far_expansion_matches_quadrature_at_moderate_distance():
    # At ~6 cells the expansion error is ~1e-6 relative; the quadrature is exact to 1e-12.
    for r in [(6, 2, 1), (-4, 5, 3)]:
        q = _quadrature_tensor(r, (1, 1, 1), n=8)
        f = newell.newell_far(*r, (1, 1, 1))
        assert np.max(np.abs(q - f)) / np.max(np.abs(q)) < 5e-6


@pytest.mark.parametrize("cell,tol", [((1, 1, 1), 2e-8), ((1, 0.7, 0.4), 3e-7)])
def test_near_far_continuity_at_switch_radius(cell, tol):
    """Both evaluations agree where the oracle switches between them."""
    rng = np.random.default_rng(1)
    h = np.asarray(cell) / max(cell)
    pts = []
    while len(pts) < 60:
        d = rng.integers(-25, 26, size=3)
        rho = np.linalg.norm(d * h)
        if newell.RC - 1.0 < rho <= newell.RC + 1.0:
            pts.append(d)
    d = np.array(pts).T
    a = newell.newell_near(d[0], d[1], d[2], cell)
    b = newell.newell_far(d[0], d[1], d[2], cell)
    err = np.max(np.abs(a - b) / np.abs(a).max(axis=0))
    assert err < tol


@pytest.mark.parametrize("cell", [(1, 1, 1), (1, 0.7, 0.4)])
def test_parity_of_grid(cell):
    n = (5, 4, 3)
    grid = newell.tensor_grid(n, cell)
    rng = np.random.default_rng(2)
    for _ in range(40):
        i, j, k = (int(rng.integers(-v + 1, v)) for v in n)
        direct = newell.tensor(i, j, k, cell)
        np.testing.assert_allclose(grid[:, k + n[2] - 1, j + n[1] - 1, i + n[0] - 1], direct,
                                   rtol=1e-10, atol=1e-14)
    # diagonal components even, N_ab odd in a and b
    d = newell.tensor(3, -2, 1, cell)
    m = newell.tensor(-3, -2, 1, cell)
    np.testing.assert_allclose(m, d * np.array([1, 1, 1, -1, -1, 1]), rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("n,cell", [
    ((4, 4, 4), (1, 1, 1)), ((8, 8, 2), (1, 1, 1)), ((5, 3, 2), (1, 0.7, 0.4)),
    ((48, 40, 3), (1, 1, 1)),  # reaches the far-field expansion
])
def test_body_average_identity(n, cell):
    """(1/N) sum_i sum_j N(i-j) equals the tensor of the whole body (a single cell
    of size n*cell): exact demagnetizing factors of a uniformly magnetised prism."""
    nx, ny, nz = n
    grid = newell.tensor_grid(n, cell)
    w = (np.einsum("k,j,i->kji", nz - np.abs(np.arange(-nz + 1, nz)),
                   ny - np.abs(np.arange(-ny + 1, ny)), nx - np.abs(np.arange(-nx + 1, nx))))
    avg = np.einsum("ckji,kji->c", grid, w) / (nx * ny * nz)
    body = newell.body_factor((nx * cell[0], ny * cell[1], nz * cell[2]))
    np.testing.assert_allclose(avg, body, rtol=0, atol=1e-9)
    assert abs(avg[:3].sum() - 1.0) < 1e-9


def test_thin_film_limit():
    """N_zz of a flat body tends to 1 as the aspect ratio grows."""
    vals = [newell.body_factor((L, L, 1.0))[2] for L in (4, 16, 64, 256, 4096, 65536)]
    assert all(b > a for a, b in zip(vals, vals[1:]))
    assert vals[-1] > 0.9998
