"""Point-dipole interaction kernel, Eq. (8) (Sec. IV), in FP64 (oracle; test
infrastructure only).

Eq. (8) gives the dipole-dipole field at spin i as the sum over all other spins
j of mu_B/(4 pi) [3 (S_j . r^) r^ - S_j] / r^3, with S_j in units of the Bohr
magneton and r the vector between the two sites.  With the moment density
M_j = mu_B S_j / V (V the volume per site, a^3 on a simple-cubic lattice) this is
Eq. (1), H_i = -sum_j N(i - j) M_j, with the kernel

    N_ab(r) = V (delta_ab |r|^2 - 3 r_a r_b) / (4 pi |r|^5),   N(0) = 0,

i.e. the tensor of a point dipole (no averaging over a cell); the j = i term is
excluded by N(0) = 0.
"""

import numpy as np

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


def tensor(i, j, k, cell):
    """N at integer displacements (i, j, k) of a lattice with spacings cell."""
    dx, dy, dz = (float(c) for c in cell)
    i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
    x = i * dx
    y = j * dy
    z = k * dz
    r2 = x * x + y * y + z * z
    V = dx * dy * dz
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(r2 > 0, V / (4.0 * np.pi * r2 ** 2.5), 0.0)
    out = np.empty((6,) + i.shape)
    out[0] = c * (r2 - 3 * x * x)
    out[1] = c * (r2 - 3 * y * y)
    out[2] = c * (r2 - 3 * z * z)
    out[3] = c * (-3 * x * y)
    out[4] = c * (-3 * x * z)
    out[5] = c * (-3 * y * z)
    return out
