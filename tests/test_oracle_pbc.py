"""Pins of the periodic-boundary oracle (Sec. II: a modified kernel, no zero
padding along a periodic axis) against facts it does not compute itself."""

import numpy as np
import pytest

import workloads as W
from oracle import demag, llg, pbc

CELL = W.CELL_4NM
RECT = (5e-9, 4e-9, 3e-9)


def _uniform(n, axis):
    M = np.zeros((3, n[2], n[1], n[0]))
    M[axis] = 1.0
    return M


@pytest.mark.parametrize("n,mask,images,cell,kind", [
    ((4, 4, 2), (1, 1, 0), 2, CELL, "newell"),
    ((4, 2, 2), (1, 0, 1), 2, RECT, "newell"),
    ((2, 4, 4), (0, 1, 1), 1, RECT, "newell"),
    ((4, 2, 2), (1, 1, 1), 1, CELL, "newell"),     # periods of two cells
    ((3, 4, 2), (1, 1, 0), 2, CELL, "newell"),     # odd period: no r = n/2 entry
    ((4, 4, 2), (1, 1, 0), 2, CELL, "dipole"),
    ((4, 1, 2), (1, 1, 0), 3, CELL, "newell"),     # periodic axis of one cell
])
def test_fft_equals_direct_image_sum(n, mask, images, cell, kind):
    """The circular convolution with the image kernel equals the explicit double
    sum over source cells and their periodic images."""
    rng = np.random.default_rng(sum(n) + images)
    M = rng.standard_normal((3, n[2], n[1], n[0]))
    H = pbc.DemagPBC(n, cell, mask, images, kind=kind)(M)
    ref = pbc.demag_pbc_direct(M, cell, mask, images, kind=kind)
    assert demag.rel_l2(H, ref) < 1e-12


@pytest.mark.parametrize("n,mask,images,cell", [
    ((8, 4, 2), (1, 1, 0), 3, CELL),
    ((4, 4, 4), (1, 1, 1), 2, RECT),
    ((8, 2, 2), (1, 0, 0), 5, CELL),
    ((4, 8, 1), (0, 1, 1), 2, RECT),
])
def test_trace_is_one_in_every_cell(n, mask, images, cell):
    """Gauss: the tensor of a body (here the mesh and its images) has trace 1 at
    every point inside it, so sum_a H_a(M = e_a) = -1 in every cell."""
    D = pbc.DemagPBC(n, cell, mask, images)
    tr = sum(D(_uniform(n, a))[a] for a in range(3))
    np.testing.assert_allclose(tr, -1.0, atol=1e-10)


@pytest.mark.parametrize("images", [1, 2, 4])
def test_fully_periodic_cube_is_minus_a_third(images):
    """Three periodic axes of a cubic mesh of cubic cells: the field is uniform
    (translation invariance) and its mean is the volume-average demagnetizing
    factor of a cube, 1/3 (cubic symmetry and trace 1), at every image count."""
    n = (4, 4, 4)
    D = pbc.DemagPBC(n, CELL, (1, 1, 1), images)
    for a in range(3):
        H = D(_uniform(n, a))
        np.testing.assert_allclose(H[a], -1.0 / 3.0, atol=1e-11)
        for b in range(3):
            if b != a:
                np.testing.assert_allclose(H[b], 0.0, atol=1e-11)


def test_film_tends_to_the_infinite_slab():
    """Two periodic in-plane axes: uniform M_z sees -M_z(1 - c/P) with the
    missing far sheet falling off as 1/P; in-plane M sees no field."""
    n = (8, 8, 1)
    dev = []
    for P in (8, 16, 32):
        D = pbc.DemagPBC(n, CELL, (1, 1, 0), P)
        H = D(_uniform(n, 2))
        np.testing.assert_allclose(H[2], H[2].mean(), atol=1e-12)
        np.testing.assert_allclose(H[:2], 0.0, atol=1e-12)
        dev.append(1.0 + H[2].mean())
        Hx = D(_uniform(n, 0))
        assert np.abs(Hx[0]).max() < dev[-1]
    assert 0 < dev[-1] < 2e-3
    for a, b in zip(dev, dev[1:]):
        assert 1.85 < a / b < 2.15


def test_wire_has_no_end_charges():
    """One periodic axis along uniform M: the end charges recede with the image
    count and the axial field falls off as 1/P^2."""
    n = (8, 2, 2)
    vals = [abs(pbc.DemagPBC(n, CELL, (1, 0, 0), P)(_uniform(n, 0))[0].mean())
            for P in (4, 8, 16)]
    for a, b in zip(vals, vals[1:]):
        assert 3.4 < a / b < 4.2


@pytest.mark.parametrize("mask", [(0, 0, 1), (1, 0, 1)])
def test_single_cell_period_is_a_tiled_open_mesh(mask):
    """A periodic axis of one cell with P images is the same body as an open
    mesh of 2P + 1 copies along that axis: the periodic field equals the open
    field (independently pinned) in the middle copy."""
    P = 2
    n = (1 if mask[0] else 4, 4, 1)
    rng = np.random.default_rng(3)
    M = rng.standard_normal((3, n[2], n[1], n[0]))
    H = pbc.DemagPBC(n, RECT, mask, P)(M)
    reps = (2 * P + 1 if mask[2] else 1, 1, 2 * P + 1 if mask[0] else 1)
    big = np.tile(M, (1,) + reps)
    Hbig = demag.demag_fft(big, RECT)
    sl = (slice(None), slice(P, P + 1) if mask[2] else slice(None), slice(None),
          slice(P, P + 1) if mask[0] else slice(None))
    np.testing.assert_allclose(H, Hbig[sl], rtol=0, atol=1e-12 * np.abs(Hbig).max())


@pytest.mark.parametrize("mask", [(1, 1, 0), (1, 0, 1), (1, 1, 1)])
def test_translation_equivariance(mask):
    """Circular convolution: shifting M cyclically along a periodic axis shifts
    H the same way (open axes have no such symmetry)."""
    n = (8, 4, 4)
    rng = np.random.default_rng(9)
    M = rng.standard_normal((3, n[2], n[1], n[0]))
    D = pbc.DemagPBC(n, CELL, mask, 1)
    H = D(M)
    for axis, per in zip((3, 2, 1), mask):
        if per:
            np.testing.assert_allclose(D(np.roll(M, 3, axis)), np.roll(H, 3, axis), atol=1e-12)


def test_no_periodic_axis_is_the_open_convolution():
    n = (8, 4, 2)
    M = np.random.default_rng(1).standard_normal((3, n[2], n[1], n[0]))
    np.testing.assert_allclose(pbc.DemagPBC(n, RECT, (0, 0, 0), 5)(M), demag.demag_fft(M, RECT),
                               atol=1e-13)


def test_periodic_exchange_plane_wave():
    """A plane wave cos(2 pi p i / n) along each periodic axis is an
    eigenvector of the wrapped 7-point Laplacian, eigenvalue
    -sum_d (2 - 2 cos(2 pi p_d / n_d)) / h_d^2."""
    n = (8, 6, 4)
    cell = RECT
    p = (3, 1, 1)
    zz, yy, xx = np.meshgrid(*(np.arange(v) for v in (n[2], n[1], n[0])), indexing="ij")
    mode = (np.cos(2 * np.pi * p[0] * xx / n[0]) * np.cos(2 * np.pi * p[1] * yy / n[1] + 0.3)
            * np.cos(2 * np.pi * p[2] * zz / n[2]))
    m = np.stack([mode, -0.5 * mode, 2 * mode])
    lam = -sum((2 - 2 * np.cos(2 * np.pi * p[d] / n[d])) / cell[d] ** 2 for d in range(3))
    H = llg.exchange_field(m, cell, W.A_EX, W.MS, pbc=(True, True, True))
    np.testing.assert_allclose(H, 2 * W.A_EX / (llg.MU0 * W.MS) * lam * m, rtol=1e-10,
                               atol=1e-6 * np.abs(H).max())


def test_periodic_exchange_of_two_cells_counts_both_neighbours():
    """n_d = 2 periodic: both neighbours of a cell are the other cell."""
    m = np.zeros((3, 1, 1, 2))
    m[0, 0, 0] = [1.0, -1.0]
    H = llg.exchange_field(m, (1.0, 1.0, 1.0), 1.0, 1.0, pbc=(True, False, False))
    c = 2.0 / llg.MU0
    np.testing.assert_allclose(H[0, 0, 0], [c * (2 * -1.0 - 2 * 1.0), c * (2 * 1.0 - 2 * -1.0)])
