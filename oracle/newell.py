"""Cell-averaged demagnetizing tensor N(r) in FP64 (oracle; test infrastructure only).

What is computed
----------------
Eq. (1) of the paper (Sec. II) needs the demagnetizing tensor N between two
rectangular cells of size dx*dy*dz whose centres are r = (i*dx, j*dy, k*dz)
apart; the paper takes it from "the formulas in Ref. [23]" without printing them.
The standard cell-averaged (Newell, Williams & Dunlop 1993) definition is used:

    N_ab(r) = -1/(4 pi V) * Int_cell Int_cell d_a d_b (1/|r + x - y|) dx dy,
    V = dx*dy*dz,  H = -N M.

It is evaluated two ways, switched on the distance |r| / max(dx, dy, dz):

* near field (|r| <= RC): Newell's closed forms f (diagonal) and g (off-diagonal)
  combined by the 27-point second-difference stencil with weights
  w(0) = 2, w(+-1) = -1 per axis;
* far field (|r| > RC): the 27-point stencil loses every digit to cancellation
  a few hundred cells out, so the cell-pair average is expanded in moments of the
  separation u = x - y (triangular distribution per axis, E[u^2] = h^2/6,
  E[u^4] = h^4/15):
      N(r) ~= V * [D + sum_d h_d^2/12 d_d^2 D + sum_d h_d^4/360 d_d^4 D
                   + sum_{d<e} h_d^2 h_e^2/144 d_d^2 d_e^2 D],
      D_ab(r) = -(1/4 pi) d_a d_b (1/|r|)  (point-dipole tensor).
  The derivatives are produced symbolically by SymPy (a library primitive).

Everything is computed in units of h = max(dx, dy, dz); N is dimensionless and
invariant under a common rescaling of r and the cell.

Components are ordered (xx, yy, zz, xy, xz, yz).
Pins: tests/test_oracle_newell.py (cube self term 1/3, trace identities, 6-D
Gauss-Legendre quadrature of the definition, near/far continuity, parity,
body-average identity).
"""

import functools

import numpy as np

RC = 16.0  # near/far switch radius in units of max(dx, dy, dz)

COMPONENTS = ("xx", "yy", "zz", "xy", "xz", "yz")


# --------------------------------------------------------------------------- #
# Newell closed forms (near field)
# --------------------------------------------------------------------------- #
def _safe_div(num, den):
    out = np.zeros(np.broadcast(num, den).shape)
    nz = den != 0
    np.divide(num, den, out=out, where=nz)
    return out, nz


def newell_f(x, y, z):
    """Newell's f(x, y, z) for the diagonal component N_xx; even in every argument.

    Every term whose denominator vanishes takes its limit, which is 0.
    """
    x = np.abs(np.asarray(x, dtype=np.float64))
    y = np.abs(np.asarray(y, dtype=np.float64))
    z = np.abs(np.asarray(z, dtype=np.float64))
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    res = (2.0 * x2 - y2 - z2) * R / 6.0

    a, ok = _safe_div(y, np.sqrt(x2 + z2))
    res = res + np.where(ok, 0.5 * y * (z2 - x2) * np.arcsinh(a), 0.0)
    a, ok = _safe_div(z, np.sqrt(x2 + y2))
    res = res + np.where(ok, 0.5 * z * (y2 - x2) * np.arcsinh(a), 0.0)
    a, ok = _safe_div(y * z, x * R)
    res = res - np.where(ok, x * y * z * np.arctan(a), 0.0)
    return res


def newell_g(x, y, z):
    """Newell's g(x, y, z) for the off-diagonal component N_xy (signed arguments)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    x2, y2, z2 = x * x, y * y, z * z
    R = np.sqrt(x2 + y2 + z2)
    res = -x * y * R / 3.0

    a, ok = _safe_div(z, np.sqrt(x2 + y2))
    res = res + np.where(ok, x * y * z * np.arcsinh(a), 0.0)
    a, ok = _safe_div(x, np.sqrt(y2 + z2))
    res = res + np.where(ok, y / 6.0 * (3.0 * z2 - y2) * np.arcsinh(a), 0.0)
    a, ok = _safe_div(y, np.sqrt(x2 + z2))
    res = res + np.where(ok, x / 6.0 * (3.0 * z2 - x2) * np.arcsinh(a), 0.0)
    a, ok = _safe_div(x * y, z * R)
    res = res - np.where(ok, z2 * z / 6.0 * np.arctan(a), 0.0)
    a, ok = _safe_div(x * z, y * R)
    res = res - np.where(ok, z * y2 / 2.0 * np.arctan(a), 0.0)
    a, ok = _safe_div(y * z, x * R)
    res = res - np.where(ok, z * x2 / 2.0 * np.arctan(a), 0.0)
    return res


_W = {-1: -1.0, 0: 2.0, 1: -1.0}


def _stencil(func, X, Y, Z, hx, hy, hz):
    """sum_{p,q,s in {-1,0,1}} w_p w_q w_s func(X + p hx, Y + q hy, Z + s hz)."""
    acc = np.zeros(np.broadcast(X, Y, Z).shape)
    for p in (-1, 0, 1):
        for q in (-1, 0, 1):
            for s in (-1, 0, 1):
                acc = acc + _W[p] * _W[q] * _W[s] * func(X + p * hx, Y + q * hy, Z + s * hz)
    return acc


def newell_near(i, j, k, cell):
    """N(r) by Newell's formulas at integer displacements (i, j, k) (arrays ok).

    Returns an array of shape (6, *broadcast shape) in component order
    (xx, yy, zz, xy, xz, yz).
    """
    dx, dy, dz = (float(c) for c in cell)
    h = max(dx, dy, dz)
    dx, dy, dz = dx / h, dy / h, dz / h
    X = np.asarray(i, dtype=np.float64) * dx
    Y = np.asarray(j, dtype=np.float64) * dy
    Z = np.asarray(k, dtype=np.float64) * dz
    c = 1.0 / (4.0 * np.pi * dx * dy * dz)
    xx = c * _stencil(newell_f, X, Y, Z, dx, dy, dz)
    yy = c * _stencil(newell_f, Y, X, Z, dy, dx, dz)
    zz = c * _stencil(newell_f, Z, Y, X, dz, dy, dx)
    xy = c * _stencil(newell_g, X, Y, Z, dx, dy, dz)
    xz = c * _stencil(newell_g, X, Z, Y, dx, dz, dy)
    yz = c * _stencil(newell_g, Y, Z, X, dy, dz, dx)
    return np.stack(np.broadcast_arrays(xx, yy, zz, xy, xz, yz))


# --------------------------------------------------------------------------- #
# Moment expansion of the cell-pair average (far field), derived by SymPy
# --------------------------------------------------------------------------- #
@functools.lru_cache(maxsize=None)
def _far_field_numerators():
    """Polynomials P0, P2, P4 (per component) with

        d_a d_b phi                                                   = P0 / r^5
        sum_d hd^2/12 d_d^2 (d_a d_b phi)                             = P2 / r^9
        sum_d hd^4/360 d_d^4 (.) + sum_{d<e} hd^2 he^2/144 d_d^2 d_e^2 (.) = P4 / r^13

    for phi = 1/r, returned as numpy-callable functions of (x, y, z, hx, hy, hz).

    A derivative of 1/r of order n is a polynomial over r^(2n+1); one more
    derivative along axis d follows from the quotient rule:
        d_d [P / r^(2n+1)] = (r^2 d_d P - (2n+1) x_d P) / r^(2n+3).
    SymPy does the polynomial algebra exactly.
    """
    import sympy as sp

    x, y, z = sp.symbols("x y z", real=True)
    hx, hy, hz = sp.symbols("hx hy hz", positive=True)
    X, Hs = (x, y, z), (hx, hy, hz)
    r2 = x**2 + y**2 + z**2

    @functools.lru_cache(maxsize=None)
    def dphi(orders):
        """Numerator P of d^orders (1/r) = P / r^(2n+1), n = sum(orders)."""
        if sum(orders) == 0:
            return sp.Integer(1)
        d = next(a for a in range(3) if orders[a] > 0)
        lower = list(orders)
        lower[d] -= 1
        lower = tuple(lower)
        n = sum(lower)
        P = dphi(lower)
        return sp.expand(r2 * sp.diff(P, X[d]) - (2 * n + 1) * X[d] * P)

    def unit(*axes):
        o = [0, 0, 0]
        for a in axes:
            o[a] += 1
        return tuple(o)

    pairs = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))
    funcs = []
    for a, b in pairs:
        p0 = dphi(unit(a, b))
        p2 = sum(Hs[d] ** 2 / 12 * dphi(unit(a, b, d, d)) for d in range(3))
        p4 = sum(Hs[d] ** 4 / 360 * dphi(unit(a, b, d, d, d, d)) for d in range(3))
        for d in range(3):
            for e in range(d + 1, 3):
                p4 += Hs[d] ** 2 * Hs[e] ** 2 / 144 * dphi(unit(a, b, d, d, e, e))
        funcs.append(tuple(sp.lambdify((x, y, z, hx, hy, hz), sp.expand(p), "numpy")
                           for p in (p0, p2, p4)))
    return tuple(funcs)


def newell_far(i, j, k, cell):
    """N(r) by the moment expansion (valid for |r| >> cell); shape (6, ...)."""
    dx, dy, dz = (float(c) for c in cell)
    h = max(dx, dy, dz)
    dx, dy, dz = dx / h, dy / h, dz / h
    X = np.asarray(i, dtype=np.float64) * dx
    Y = np.asarray(j, dtype=np.float64) * dy
    Z = np.asarray(k, dtype=np.float64) * dz
    X, Y, Z = np.broadcast_arrays(X, Y, Z)
    r2 = X * X + Y * Y + Z * Z
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.sqrt(r2)
        inv5 = 1.0 / (r2 * r2 * r)
        inv9 = inv5 / (r2 * r2)
        inv13 = inv9 / (r2 * r2)
    V = dx * dy * dz
    out = np.empty((6,) + X.shape)
    for c, (p0, p2, p4) in enumerate(_far_field_numerators()):
        val = (np.broadcast_to(p0(X, Y, Z, dx, dy, dz), X.shape) * inv5
               + np.broadcast_to(p2(X, Y, Z, dx, dy, dz), X.shape) * inv9
               + np.broadcast_to(p4(X, Y, Z, dx, dy, dz), X.shape) * inv13)
        out[c] = -V / (4.0 * np.pi) * val
    return out


# --------------------------------------------------------------------------- #
# Dispatch
# --------------------------------------------------------------------------- #
def is_near(i, j, k, cell, rc=RC):
    dx, dy, dz = (float(c) for c in cell)
    h = max(dx, dy, dz)
    X = np.asarray(i, dtype=np.float64) * (dx / h)
    Y = np.asarray(j, dtype=np.float64) * (dy / h)
    Z = np.asarray(k, dtype=np.float64) * (dz / h)
    return X * X + Y * Y + Z * Z <= rc * rc


def tensor(i, j, k, cell, rc=RC):
    """N at integer displacements (i, j, k): Newell when |r| <= rc*h, expansion beyond."""
    i, j, k = np.broadcast_arrays(np.asarray(i), np.asarray(j), np.asarray(k))
    near = is_near(i, j, k, cell, rc)
    out = np.empty((6,) + i.shape)
    if near.any():
        out[:, near] = newell_near(i[near], j[near], k[near], cell)
    far = ~near
    if far.any():
        out[:, far] = newell_far(i[far], j[far], k[far], cell)
    return out


# Parity of each component under r_d -> -r_d, per axis (x, y, z):
# diagonal components are even in every axis; N_ab (a != b) is odd in a and b.
PARITY = {
    "xx": (1, 1, 1), "yy": (1, 1, 1), "zz": (1, 1, 1),
    "xy": (-1, -1, 1), "xz": (-1, 1, -1), "yz": (1, -1, -1),
}


def tensor_grid(n, cell, rc=RC):
    """N on every displacement a linear convolution over an n = (nx, ny, nz) mesh uses.

    Returns an array of shape (6, 2nz-1, 2ny-1, 2nx-1); entry [c, k+nz-1, j+ny-1,
    i+nx-1] is N_c(i, j, k).  The octant i, j, k >= 0 is evaluated and the rest
    filled by the parity of each component (pinned against direct evaluation).
    """
    nx, ny, nz = (int(v) for v in n)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    octant = tensor(ii, jj, kk, cell, rc)  # (6, nz, ny, nx)
    full = np.empty((6, 2 * nz - 1, 2 * ny - 1, 2 * nx - 1))
    for c, name in enumerate(COMPONENTS):
        px, py, pz = PARITY[name]
        o = octant[c]
        for sz in (1, -1):
            for sy in (1, -1):
                for sx in (1, -1):
                    sign = (px if sx < 0 else 1) * (py if sy < 0 else 1) * (pz if sz < 0 else 1)
                    zs = slice(nz - 1, 2 * nz - 1) if sz > 0 else slice(nz - 1, None, -1)
                    ys = slice(ny - 1, 2 * ny - 1) if sy > 0 else slice(ny - 1, None, -1)
                    xs = slice(nx - 1, 2 * nx - 1) if sx > 0 else slice(nx - 1, None, -1)
                    full[c, zs, ys, xs] = sign * o
    return full


def body_factor(body):
    """Demagnetizing factors (6 components) of a uniformly magnetised rectangular body
    of edge lengths body = (Lx, Ly, Lz): the Newell self term with the cell equal to
    the body."""
    return newell_near(0, 0, 0, body)
