"""Demagnetizing field H_d = -sum_j N(i-j) M_j in FP64 (oracle; test infrastructure only).

Two evaluations of Eq. (1) (Sec. II):

* ``demag_direct``: the sum itself, O(N^2), over every cell including j = i.
  This is the definition of the result.
* ``DemagFFT`` / ``demag_fft``: the convolution theorem (Sec. II; Fig. 1;
  App. A): N and M are zero-padded to N_d = 2 n_d along each axis (N_d = 1 when
  n_d = 1, where only r_d = 0 enters), transformed, multiplied point by point
  (H^_a = -sum_b N^_ab M^_b), inverse-transformed and truncated to the mesh.
  The displacement r is stored at index r mod N_d; the entry at index n_d
  (r = +-n_d) never enters a linear convolution and is left 0.

Arrays are laid out (component, z, y, x), x fastest, SI units (A/m).
"""

import numpy as np
import scipy.fft as sfft

from . import dipole, newell


def _tensor_fn(kind):
    """Kernel of the convolution: the cell-averaged (Newell) tensor of Eq. (1),
    or the point-dipole tensor of Eq. (8) (kind "dipole")."""
    if kind == "newell":
        return newell.tensor
    if kind == "dipole":
        return dipole.tensor
    raise ValueError(kind)


def padded_size(n):
    """N_d = 2 n_d, or 1 when n_d = 1."""
    return tuple(1 if v == 1 else 2 * v for v in n)


def tensor3(Nc):
    """6 components (xx, yy, zz, xy, xz, yz) -> symmetric 3x3 nesting [a][b]."""
    xx, yy, zz, xy, xz, yz = Nc
    return ((xx, xy, xz), (xy, yy, yz), (xz, yz, zz))


def demag_direct(M, cell, kind="newell"):
    """H_i = -sum_j N(i - j) M_j by explicit summation (small meshes only).

    M: float array (3, nz, ny, nx) in A/m.  Returns H with the same shape.
    """
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    if kind == "newell":
        grid = newell.tensor_grid((nx, ny, nz), cell)  # (6, 2nz-1, 2ny-1, 2nx-1)
    else:
        kk, jj, ii = np.meshgrid(np.arange(-nz + 1, nz), np.arange(-ny + 1, ny),
                                 np.arange(-nx + 1, nx), indexing="ij")
        grid = _tensor_fn(kind)(ii, jj, kk, cell)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    src_k, src_j, src_i = kk.ravel(), jj.ravel(), ii.ravel()
    Mflat = M.reshape(3, -1)
    H = np.zeros_like(Mflat)
    for t in range(src_i.size):
        di = ii.ravel()[t] - src_i + nx - 1
        dj = jj.ravel()[t] - src_j + ny - 1
        dk = kk.ravel()[t] - src_k + nz - 1
        Nt = grid[:, dk, dj, di]  # (6, ncells): N(i - j) for all sources j
        T = tensor3(Nt)
        for a in range(3):
            H[a, t] = -sum(np.dot(T[a][b], Mflat[b]) for b in range(3))
    return H.reshape(M.shape)


def _axis_map(n, Nd):
    """For each padded index p along one axis: the displacement |r| it holds, the
    sign convention (r < 0) and whether it is used at all."""
    p = np.arange(Nd)
    r = np.where(p < n, p, p - Nd)
    used = np.abs(r) <= n - 1
    if Nd == 1:
        r = np.zeros(1, dtype=int)
        used = np.ones(1, dtype=bool)
    return np.where(used, np.abs(r), 0), r < 0, used


class DemagFFT:
    """Zero-padded FFT evaluation of Eq. (1) for one mesh and cell size.

    The transformed tensor is computed once at construction (the paper's
    initialisation stage, Sec. II).
    """

    def __init__(self, n, cell, workers=None, kind="newell", dtype=np.float64):
        """dtype: np.float64 (the oracle) or np.float32, the same steps in single
        precision (the transformed tensor rounded once from FP64), used only to
        time a like-for-like CPU figure, never as a reference."""
        self.n = tuple(int(v) for v in n)  # (nx, ny, nz)
        self.cell = tuple(float(c) for c in cell)
        self.N = padded_size(self.n)  # (Nx, Ny, Nz)
        self.workers = workers
        self.dtype = np.dtype(dtype)
        nx, ny, nz = self.n
        Nx, Ny, Nz = self.N
        kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        octant = _tensor_fn(kind)(ii, jj, kk, self.cell)  # (6, nz, ny, nx): r >= 0
        ax, sx, ux = _axis_map(nx, Nx)
        ay, sy, uy = _axis_map(ny, Ny)
        az, sz, uz = _axis_map(nz, Nz)
        used = uz[:, None, None] & uy[None, :, None] & ux[None, None, :]
        self.Khat = []
        for c, name in enumerate(newell.COMPONENTS):
            px, py, pz = newell.PARITY[name]
            sign = (np.where(sz, pz, 1)[:, None, None]
                    * np.where(sy, py, 1)[None, :, None]
                    * np.where(sx, px, 1)[None, None, :])
            Kpad = octant[c][np.ix_(az, ay, ax)] * sign * used
            Kh = sfft.rfftn(Kpad, axes=(0, 1, 2), workers=workers)
            self.Khat.append(Kh.astype(np.complex64) if self.dtype == np.float32 else Kh)
            del Kpad, Kh

    def to_float32(self):
        """The same operator computing in FP32 (tensor rounded once from FP64);
        for timing only."""
        op = object.__new__(DemagFFT)
        op.__dict__.update(self.__dict__)
        op.dtype = np.dtype(np.float32)
        op.Khat = [k.astype(np.complex64) for k in self.Khat]
        return op

    def __call__(self, M):
        M = np.asarray(M, dtype=self.dtype)
        nx, ny, nz = self.n
        Nx, Ny, Nz = self.N
        assert M.shape == (3, nz, ny, nx), M.shape
        Mhat = [sfft.rfftn(M[b], s=(Nz, Ny, Nx), axes=(0, 1, 2), workers=self.workers)
                for b in range(3)]
        T = tensor3(self.Khat)
        H = np.empty_like(M)
        for a in range(3):
            Hhat = -(T[a][0] * Mhat[0] + T[a][1] * Mhat[1] + T[a][2] * Mhat[2])
            H[a] = sfft.irfftn(Hhat, s=(Nz, Ny, Nx), axes=(0, 1, 2),
                               workers=self.workers)[:nz, :ny, :nx]
        return H


def demag_fft(M, cell, workers=None, kind="newell"):
    """One-shot H_d by the zero-padded FFT convolution."""
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    return DemagFFT((nx, ny, nz), cell, workers, kind)(M)


def demag_at(M, cell, targets):
    """H_d at a few target cells only, by the direct sum over all sources.

    targets: integer array (T, 3) of (x, y, z) cell indices.  Returns (3, T).
    Cost O(T * N); used to spot-check large meshes whose full oracle is too big.
    """
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    Mflat = M.reshape(3, -1)
    out = np.zeros((3, len(targets)))
    for t, (x, y, z) in enumerate(np.asarray(targets)):
        Nt = newell.tensor(x - ii.ravel(), y - jj.ravel(), z - kk.ravel(), cell)
        T = tensor3(Nt)
        for a in range(3):
            out[a, t] = -sum(np.dot(T[a][b], Mflat[b]) for b in range(3))
    return out


def rel_l2(H, Href):
    """Relative L2 error over all entries: ||H - Href|| / ||Href||."""
    H = np.asarray(H, dtype=np.float64)
    Href = np.asarray(Href, dtype=np.float64)
    return float(np.linalg.norm(H - Href) / np.linalg.norm(Href))


def rel_l2_per_field(H, Href):
    """Relative L2 error of each field component (H_x, H_y, H_z)."""
    return [rel_l2(H[a], Href[a]) for a in range(3)]
