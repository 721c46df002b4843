"""Periodic boundary conditions for the demagnetizing field, in FP64 (oracle; test
infrastructure only).

Sec. II: with periodic boundary conditions along an axis the convolution needs
a modified kernel and no zero padding along that axis.  The modification (the
scheme of the cited work is not printed) is read here as the sum over periodic
images of the body, truncated at `images` copies on each side:

    N_pbc(r) = sum_{m} N(r + m_x n_x h_x e_x + m_y n_y h_y e_y + m_z n_z h_z e_z),

m_d in [-images, images] along each periodic axis (0 along the others).  The
convolution along a periodic axis is circular with length n_d; the displacement
at index p is r = p for p <= n_d/2 and p - n_d beyond.  The exact (infinite)
image sum is periodic and, for the components odd in that axis, odd, hence zero
at r_d = n_d/2; that value is set to zero so that the transformed kernel stays
real, as without periodicity.

The exchange field with periodic boundaries couples the first and last cells
along a periodic axis (llg.exchange_field with pbc).
"""

import numpy as np
import scipy.fft as sfft

from . import demag, dipole, newell

DEFAULT_IMAGES = 32


def _tensor_fn(kind):
    return {"newell": newell.tensor, "dipole": dipole.tensor}[kind]


def octant_extent(n, pbc):
    """Displacements r_d = 0 .. R_d - 1 the kernel needs: n_d/2 + 1 on a periodic
    axis, n_d otherwise."""
    return tuple((v // 2 + 1) if p else v for v, p in zip(n, pbc))


def image_kernel_octant(n, cell, pbc, images=DEFAULT_IMAGES, kind="newell"):
    """N_pbc on the octant r_d in [0, R_d): array (6, Rz, Ry, Rx)."""
    nx, ny, nz = n
    Rx, Ry, Rz = octant_extent(n, pbc)
    kk, jj, ii = np.meshgrid(np.arange(Rz), np.arange(Ry), np.arange(Rx), indexing="ij")
    offs = [np.arange(-images, images + 1) if p else np.zeros(1, dtype=int) for p in pbc]
    mz, my, mx = np.meshgrid(offs[2], offs[1], offs[0], indexing="ij")
    m = np.stack([mx.ravel() * nx, my.ravel() * ny, mz.ravel() * nz], 1)   # image shifts
    fn = _tensor_fn(kind)
    out = np.zeros((6, Rz, Ry, Rx))
    batch = max(1, 2_000_000 // ii.size)
    for s in range(0, len(m), batch):
        sh = m[s:s + batch]
        out += fn(ii[None] + sh[:, 0, None, None, None], jj[None] + sh[:, 1, None, None, None],
                  kk[None] + sh[:, 2, None, None, None], cell).sum(axis=1)
    # components odd in a periodic axis vanish at r_d = n_d / 2 (exact image sum)
    for c, name in enumerate(newell.COMPONENTS):
        for axis, (v, p) in enumerate(zip(n, pbc)):
            if p and v >= 2 and v % 2 == 0 and newell.PARITY[name][axis] < 0:
                sl = [slice(None)] * 3
                sl[2 - axis] = v // 2
                out[(c,) + tuple(sl)] = 0.0
    return out


def _axis_map(n, Nd, periodic):
    """For each index p of the transform along one axis: |r|, r < 0, used."""
    if not periodic:
        return demag._axis_map(n, Nd)
    p = np.arange(Nd)
    r = np.where(p <= Nd // 2, p, p - Nd)
    return np.abs(r), r < 0, np.ones(Nd, dtype=bool)


class DemagPBC:
    """H = -sum_j N_pbc(i - j) M_j: circular along periodic axes, zero-padded along
    the others (N_d = n_d periodic, 2 n_d otherwise, 1 when n_d = 1)."""

    def __init__(self, n, cell, pbc, images=DEFAULT_IMAGES, workers=None, kind="newell"):
        self.n = tuple(int(v) for v in n)
        self.cell = tuple(float(c) for c in cell)
        self.pbc = tuple(bool(p) for p in pbc)
        self.N = tuple(v if p else (1 if v == 1 else 2 * v) for v, p in zip(self.n, self.pbc))
        self.workers = workers
        nx, ny, nz = self.n
        Nx, Ny, Nz = self.N
        octant = image_kernel_octant(self.n, self.cell, self.pbc, images, kind)
        ax, sx, ux = _axis_map(nx, Nx, self.pbc[0])
        ay, sy, uy = _axis_map(ny, Ny, self.pbc[1])
        az, sz, uz = _axis_map(nz, Nz, self.pbc[2])
        used = uz[:, None, None] & uy[None, :, None] & ux[None, None, :]
        self.Khat = []
        for c, name in enumerate(newell.COMPONENTS):
            px, py, pz = newell.PARITY[name]
            sign = (np.where(sz, pz, 1)[:, None, None]
                    * np.where(sy, py, 1)[None, :, None]
                    * np.where(sx, px, 1)[None, None, :])
            Kpad = octant[c][np.ix_(az, ay, ax)] * sign * used
            self.Khat.append(sfft.rfftn(Kpad, axes=(0, 1, 2), workers=workers))

    def __call__(self, M):
        M = np.asarray(M, dtype=np.float64)
        nx, ny, nz = self.n
        Nx, Ny, Nz = self.N
        Mhat = [sfft.rfftn(M[b], s=(Nz, Ny, Nx), axes=(0, 1, 2), workers=self.workers)
                for b in range(3)]
        T = demag.tensor3(self.Khat)
        H = np.empty_like(M)
        for a in range(3):
            Hhat = -(T[a][0] * Mhat[0] + T[a][1] * Mhat[1] + T[a][2] * Mhat[2])
            H[a] = sfft.irfftn(Hhat, s=(Nz, Ny, Nx), axes=(0, 1, 2),
                               workers=self.workers)[:nz, :ny, :nx]
        return H


def field_at(Mv, src, targets, n, cell, pbc, images=DEFAULT_IMAGES, kind="newell"):
    """Explicit double sum over the given source cells and their images at the
    given target cells: H_t = -sum_s sum_m N(t - s + m L) M_s, each periodic
    displacement folded into (-n/2, n/2] and the components odd in a periodic
    axis dropped at |r_d| = n_d/2 as in the kernel.  Mv (3, S) holds M at the
    source cells src (S, 3) = (x, y, z); targets (T, 3).  Returns (3, T)."""
    Mv = np.asarray(Mv, dtype=np.float64)
    src = np.asarray(src)
    fn = _tensor_fn(kind)
    rng = [range(-images, images + 1) if p else range(0, 1) for p in pbc]
    H = np.zeros((3, len(targets)))
    for t, tgt in enumerate(targets):
        d = np.asarray(tgt)[None, :] - src                 # (S, 3) displacements t - s
        for axis in range(3):                              # fold into (-n/2, n/2]
            if pbc[axis]:
                v = n[axis]
                d[:, axis] = np.where(d[:, axis] > v // 2, d[:, axis] - v, d[:, axis])
                d[:, axis] = np.where(d[:, axis] <= -(v - v // 2), d[:, axis] + v, d[:, axis])
        Nt = np.zeros((6, len(src)))
        for mz in rng[2]:
            for my in rng[1]:
                for mx in rng[0]:
                    Nt += fn(d[:, 0] + mx * n[0], d[:, 1] + my * n[1], d[:, 2] + mz * n[2], cell)
        for c, name in enumerate(newell.COMPONENTS):
            for axis in range(3):
                v = n[axis]
                if pbc[axis] and v >= 2 and v % 2 == 0 and newell.PARITY[name][axis] < 0:
                    Nt[c, np.abs(d[:, axis]) == v // 2] = 0.0
        T = demag.tensor3(Nt)
        for a in range(3):
            H[a, t] = -sum(np.dot(T[a][b], Mv[b]) for b in range(3))
    return H


def demag_pbc_direct(M, cell, pbc, images=DEFAULT_IMAGES, kind="newell"):
    """The field of every cell by field_at over all cells (tiny meshes only)."""
    M = np.asarray(M, dtype=np.float64)
    _, nz, ny, nx = M.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cells = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1)
    H = field_at(M.reshape(3, -1), cells, cells, (nx, ny, nz), cell, pbc, images, kind)
    return H.reshape(M.shape)
