"""Pins for the oracle's convolution (Eq. 1; Sec. II; Fig. 1; App. A).

The zero-padded FFT evaluation is checked against the definition (direct O(N^2)
sum) and against the exact mean field of a uniformly magnetised prism.
"""

import numpy as np
import pytest

import workloads as W
from oracle import demag, newell


@pytest.mark.parametrize("n,cell", [
    ((1, 1, 1), (4e-9, 4e-9, 4e-9)),
    ((4, 3, 2), (4e-9, 4e-9, 4e-9)),
    ((5, 1, 3), (4e-9, 4e-9, 4e-9)),
    ((7, 6, 1), (4e-9, 4e-9, 4e-9)),
    ((1, 9, 1), (4e-9, 4e-9, 4e-9)),
    ((6, 5, 4), (1.0, 0.7, 0.4)),
    ((32, 8, 2), (4e-9, 4e-9, 4e-9)),   # far-field expansion enters
    ((16, 16, 16), (4e-9, 4e-9, 4e-9)),
])
def test_fft_equals_direct_sum(n, cell):
    M = W.magnetisation(n, seed=sum(n)).astype(np.float64)
    Hd = demag.demag_direct(M, cell)
    Hf = demag.demag_fft(M, cell)
    assert demag.rel_l2(Hf, Hd) <= 1e-12


@pytest.mark.parametrize("n,cell", [((8, 8, 2), (1, 1, 1)), ((6, 4, 3), (1, 0.7, 0.4)),
                                    ((5, 5, 5), (1, 1, 1))])
def test_uniform_magnetisation_mean_field(n, cell):
    """Mean H over the body = -N_body . M (uniform M), N_body = prism factors."""
    nx, ny, nz = n
    body = newell.body_factor((nx * cell[0], ny * cell[1], nz * cell[2]))
    T = np.array(demag.tensor3(body))
    for Mdir in (np.eye(3)[0], np.eye(3)[1], np.eye(3)[2], np.array([0.3, -0.5, 0.81])):
        M = np.broadcast_to(Mdir.reshape(3, 1, 1, 1), (3, nz, ny, nx)).copy()
        H = demag.demag_fft(M, cell)
        np.testing.assert_allclose(H.reshape(3, -1).mean(axis=1), -T @ Mdir, atol=1e-12)


def test_cube_uniform_field_is_minus_third():
    M = np.zeros((3, 1, 1, 1))
    M[0] = 8e5
    H = demag.demag_fft(M, (4e-9, 4e-9, 4e-9))
    np.testing.assert_allclose(H[:, 0, 0, 0], [-8e5 / 3, 0, 0], rtol=1e-14, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_demag_energy_is_positive(seed):
    """E_d = -(mu0/2) sum M.H_d >= 0 for any M."""
    M = W.magnetisation((12, 10, 3), seed).astype(np.float64)
    H = demag.demag_fft(M, (4e-9, 4e-9, 4e-9))
    assert np.sum(M * H) < 0


def test_transformed_kernel_is_real():
    """With r = +-n_d left 0, every transformed component is real (parity)."""
    op = demag.DemagFFT((6, 5, 3), (1, 0.7, 0.4))
    for K in op.Khat:
        assert np.abs(K.imag).max() <= 1e-13 * np.abs(K.real).max()


def test_padding_choice_does_not_change_result():
    """Any padded length >= 2n-1 gives the same linear convolution; compare the
    default 2n padding with an explicit 3n padding done here with numpy's FFT."""
    n, cell = (5, 4, 3), (1.0, 1.0, 1.0)
    M = W.magnetisation(n, 7).astype(np.float64)
    ref = demag.demag_fft(M, cell)
    nx, ny, nz = n
    grid = newell.tensor_grid(n, cell)
    P = (3 * nz, 3 * ny, 3 * nx)
    iz = np.arange(-nz + 1, nz) % P[0]
    iy = np.arange(-ny + 1, ny) % P[1]
    ix = np.arange(-nx + 1, nx) % P[2]
    Kh = []
    for c in range(6):
        Kp = np.zeros(P)
        Kp[np.ix_(iz, iy, ix)] = grid[c]
        Kh.append(np.fft.fftn(Kp))
    Mh = [np.fft.fftn(M[b], s=P, axes=(0, 1, 2)) for b in range(3)]
    T = demag.tensor3(Kh)
    H = np.stack([np.fft.ifftn(-(T[a][0] * Mh[0] + T[a][1] * Mh[1] + T[a][2] * Mh[2])).real
                  [:nz, :ny, :nx] for a in range(3)])
    assert demag.rel_l2(H, ref) < 1e-13


def test_demag_at_matches_full_field():
    n, cell = (9, 7, 2), (4e-9, 4e-9, 4e-9)
    M = W.magnetisation(n, 3).astype(np.float64)
    H = demag.demag_fft(M, cell)
    targets = np.array([[0, 0, 0], [8, 6, 1], [4, 3, 0]])
    got = demag.demag_at(M, cell, targets)
    for t, (x, y, z) in enumerate(targets):
        np.testing.assert_allclose(got[:, t], H[:, z, y, x], rtol=1e-12, atol=1e-6)


# ---------------------------------------------------------------- point-dipole kernel, Eq. (8)
def test_dipole_field_vanishes_at_centre_of_uniform_cubic_lattice():
    """Cubic symmetry: the lattice sum of (3 r r - r^2)/r^5 over a (2k+1)^3 cube
    centred on a site is zero, whatever the (uniform) moment direction."""
    from oracle import demag as od
    for k in (1, 2, 3):
        n = 2 * k + 1
        M = np.zeros((3, n, n, n))
        M[0], M[1], M[2] = 1.0, 0.3, -0.7
        H = od.demag_fft(M, (1e-9, 1e-9, 1e-9), kind="dipole")
        assert np.abs(H[:, k, k, k]).max() <= 1e-14 * np.abs(H).max()


def test_dipole_field_of_a_chain_is_a_zeta_sum():
    """A line of 2K+1 equal moments: at the middle site the field is
    (1/4 pi) sum_{m != 0} (3 cos^2 - 1)/|m|^3 -> 4 zeta_K(3)/(4 pi) along the line
    for moments along it, -2 zeta_K(3)/(4 pi) for moments across it (unit spacing,
    unit moment density)."""
    from oracle import demag as od
    K = 120
    n = 2 * K + 1
    zeta = sum(1.0 / m ** 3 for m in range(1, K + 1))
    M = np.zeros((3, 1, 1, n))
    M[0] = 1.0
    H = od.demag_fft(M, (1e-9, 1e-9, 1e-9), kind="dipole")
    assert H[0, 0, 0, K] == pytest.approx(4 * zeta / (4 * np.pi), rel=1e-12)
    M = np.zeros((3, 1, 1, n))
    M[1] = 1.0
    H = od.demag_fft(M, (1e-9, 1e-9, 1e-9), kind="dipole")
    assert H[1, 0, 0, K] == pytest.approx(-2 * zeta / (4 * np.pi), rel=1e-12)


def test_newell_tensor_tends_to_the_point_dipole():
    """Far from the source, the cell-averaged tensor approaches the point-dipole
    tensor: doubling the distance divides the relative difference by ~16 for
    cubic cells (the h^2 term vanishes) and by ~4 otherwise."""
    from oracle import dipole, newell

    def rel(r, cell):
        nw, dp = newell.tensor(*r, cell), dipole.tensor(*r, cell)
        return np.abs(nw - dp).max() / np.abs(dp).max()

    r1, r2 = (40, 30, 20), (80, 60, 40)
    cub = rel(r1, (1, 1, 1)) / rel(r2, (1, 1, 1))
    flat = rel(r1, (1.0, 0.7, 0.4)) / rel(r2, (1.0, 0.7, 0.4))
    assert rel(r1, (1, 1, 1)) < 1e-7
    assert 13 < cub < 19, cub
    assert 3.5 < flat < 4.5, flat


def test_dipole_fft_matches_direct_sum():
    from oracle import demag as od
    M = np.random.default_rng(2).standard_normal((3, 3, 4, 5))
    cell = (1e-9, 2e-9, 1.5e-9)
    np.testing.assert_allclose(od.demag_fft(M, cell, kind="dipole"), od.demag_direct(M, cell, kind="dipole"),
                               rtol=0, atol=1e-12 * 1)
