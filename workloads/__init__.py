"""Seeded synthetic inputs and the named workload shapes.

This module holds random-number recipes and sizes only -- none of the method's
arithmetic -- so both the GPU path's tests/bench and the FP64 oracle can take
their inputs from it without sharing any computation.

Input recipe: magnetisation directions are drawn uniform on the unit sphere by
normalising standard-normal triples from ``numpy.random.default_rng(seed)``,
generated once on the host in FP64 and rounded to FP32; both sides consume the
same FP32 values (the oracle upcasts them), so input rounding is not counted as
error.
"""

import numpy as np

MS = 8.0e5            # saturation magnetisation, A/m
A_EX = 1.3e-11        # exchange stiffness, J/m
CELL_4NM = (4e-9, 4e-9, 4e-9)


def unit_vectors(shape_zyx, seed):
    """(3, nz, ny, nx) FP32 unit vectors, uniform on the sphere."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3,) + tuple(shape_zyx))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v.astype(np.float32)


def magnetisation(n, seed, Ms=MS):
    """M = Ms * (seeded uniform unit vectors) on an n = (nx, ny, nz) mesh, FP32."""
    nx, ny, nz = n
    return (unit_vectors((nz, ny, nx), seed) * np.float32(Ms)).astype(np.float32)


def uniform_alpha(count, seed, lo=0.01, hi=0.5):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=count)


def poisson_arrivals(count, rate, seed):
    """Arrival times (s) of a Poisson process of the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


# Named workloads (mesh in cells (nx, ny, nz), cell edge in m)
DEMAG_SMALL = dict(name="demag 32x32x4 (4 nm cubes)", n=(32, 32, 4), cell=CELL_4NM)
THIN_FILM = dict(name="thin-film LLG 512x512x16 (4 nm cubes), RK4 dt=1e-13 s",
                 n=(512, 512, 16), cell=CELL_4NM, Ms=MS, A=A_EX, alpha=0.02, dt=1e-13,
                 steps=1000)
LARGE_FILM = dict(name="large film 1024x1024x32 (4 nm cubes)", n=(1024, 1024, 32),
                  cell=CELL_4NM)
ATOMISTIC = dict(name="atomistic 1024x1024x256 spins, 4^3 macrocells", n=(1024, 1024, 256),
                 a=0.4e-9, macro=4, J=1e-21, mu_s=1.0, alpha=0.05, dt=1e-15)
SERVE_SHAPES = [(s, s, z) for s in (32, 64, 128, 256, 512) for z in (1, 2, 4, 8)]
# Switching problem of the precision study (Sec. II, Fig. 2): 2.4 um x 1.2 um x
# 10 nm, 5 nm cells, Ms = 800 kA/m; S state from saturation along [1,1,1] at
# 1 MA/m ramped to zero, then H = (-20, 1, 0) kA/m for 1 ns.  A and alpha are not
# given there: permalloy's A = 13 pJ/m and alpha = 0.02 are taken; the ramp
# (its schedule is not given) runs in ramp_steps equal field decrements of
# ramp_time each, then relax_time at zero field, all with alpha_prep.
SWITCHING = dict(name="switching 480x240x2 (5 nm cells), H = (-20, 1, 0) kA/m, 1 ns",
                 n=(480, 240, 2), cell=(5e-9, 5e-9, 5e-9), Ms=8.0e5, A=1.3e-11, alpha=0.02,
                 H_sat=1.0e6, ramp_steps=10, ramp_time=50e-12, relax_time=500e-12,
                 alpha_prep=0.5, dt_prep=2e-13, H_switch=(-2.0e4, 1.0e3, 0.0), t_switch=1e-9,
                 dt_ref=1e-14, dts=(1e-13, 2e-13, 4e-13), record_every=4e-13)


def serve_requests(count, seed):
    """Seeded request mix: (mesh n, alpha, seed for m0) drawn uniformly."""
    rng = np.random.default_rng(seed)
    shapes = [SERVE_SHAPES[i] for i in rng.integers(0, len(SERVE_SHAPES), size=count)]
    alphas = rng.uniform(0.01, 0.5, size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return list(zip(shapes, alphas.tolist(), seeds.tolist()))


def sparse_sources(n, nsrc, ntgt, seed):
    """M = MS x random unit vectors in `nsrc` distinct random cells of the mesh
    n = (nx, ny, nz), zero elsewhere, as float32 [3][nz][ny][nx]; also the
    source cells and `ntgt` random target cells, each as rows (x, y, z)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    flat = rng.choice(nx * ny * nz, size=nsrc, replace=False)
    src = np.stack([flat % nx, (flat // nx) % ny, flat // (nx * ny)], 1)
    M = np.zeros((3, nz, ny, nx), dtype=np.float32)
    M[:, src[:, 2], src[:, 1], src[:, 0]] = unit_vectors((nsrc,), seed) * np.float32(MS)
    tg = np.stack([rng.integers(0, nx, ntgt), rng.integers(0, ny, ntgt),
                   rng.integers(0, nz, ntgt)], 1)
    return M, src, tg
