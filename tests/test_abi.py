"""Host-side checks of the C ABI (no GPU needed): the shared library loads, exports
every symbol include/demag.h declares, and rejects bad arguments before any
device work."""

import ctypes
import os
import re

import pytest

import paper_2308_08447_amd as pkg

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "demag.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_]+)\s*\([^;{]*\)\s*;", text)) - {"sizeof"})


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    names = declared_functions()
    assert len(names) >= 10, names
    for name in names:
        assert hasattr(lib, name), name
    assert set(pkg.EXPORTS) == set(names)


def test_plan_bytes_and_validation_on_host():
    assert pkg.demag_plan_bytes((32, 32, 4, 4e-9, 4e-9, 4e-9)) > 0
    assert pkg.demag_plan_bytes((28, 32, 4, 4e-9, 4e-9, 4e-9)) == 0
    assert pkg.demag_plan_bytes((32, 32, 256, 4e-9, 4e-9, 4e-9)) == 0
    assert pkg.demag_plan_bytes((32, 32, 4, -4e-9, 4e-9, 4e-9)) == 0
    assert pkg.demag_plan_bytes((32, 32, 4, 4e-9, 4e-9, 4e-9), flags=7) == 0
    assert pkg.demag_plan_bytes((32, 32, 4, 4e-9, 4e-9, 4e-9), flags=3) == 0
    # the split-precision MFMA form needs the FP32 five-pass workspace; the
    # two-term split is refused (no plan, no bytes)
    x3 = pkg.demag_plan_bytes((32, 32, 4, 4e-9, 4e-9, 4e-9), flags=pkg.DEMAG_BF16X3_MFMA)
    assert x3 > 0
    assert pkg.demag_plan_bytes((32, 32, 4, 4e-9, 4e-9, 4e-9), flags=pkg.DEMAG_BF16X2_MFMA) == 0
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup((32, 32, 4, 4e-9, 4e-9, 4e-9), pkg.DEMAG_BF16X2_MFMA)
    assert e.value.status == pkg.DEMAG_EUNSUPPORTED
    assert b"BF16X2" in pkg.load().demag_last_error()
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup((28, 32, 4, 4e-9, 4e-9, 4e-9))
    assert e.value.status == pkg.DEMAG_EUNSUPPORTED
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup((0, 32, 4, 4e-9, 4e-9, 4e-9))
    assert e.value.status == pkg.DEMAG_EINVAL
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup((8, 8, 8, 4e-9, float("nan"), 4e-9))
    assert e.value.status == pkg.DEMAG_EINVAL
    with pytest.raises(pkg.DemagError) as e:
        pkg.atom_setup((16, 16, 8, 0.4e-9, 3))
    assert e.value.status == pkg.DEMAG_EINVAL
    lib = pkg.load()
    assert lib.demag_field(None, None, None, None) == pkg.DEMAG_EINVAL
    assert lib.llg_step(None, None, None, 1e-13, 1, None) == pkg.DEMAG_EINVAL
    assert lib.demag_destroy(None) == pkg.DEMAG_EINVAL
    assert b"NULL" in lib.demag_last_error()


def test_plan_bytes_formula():
    # five-pass form (n_z > 16): packed kernel + S1 + the y/z chunk buffer
    nx, ny, nz = 512, 512, 32
    X1, Y1, Z1 = nx + 1, ny + 1, nz + 1
    plane = 3 * nz * 2 * ny * 8                  # one kx plane of the y/z spectra
    planes = min(X1, (128 << 20) // plane)       # a chunk buffer is capped at 128 MB
    expect = 6 * Z1 * X1 * Y1 * 4 + 3 * nz * X1 * ny * 8 + planes * plane
    assert pkg.demag_plan_bytes((nx, ny, nz, 4e-9, 4e-9, 4e-9)) == expect
    # 1024x1024x32 needs 13 chunks: the buffer holds 128 MB of kx planes
    nx, ny, nz = 1024, 1024, 32
    X1, Y1, Z1 = nx + 1, ny + 1, nz + 1
    plane = 3 * nz * 2 * ny * 8
    planes = (128 << 20) // plane
    assert planes < X1
    expect = 6 * Z1 * X1 * Y1 * 4 + 3 * nz * X1 * ny * 8 + planes * plane
    assert pkg.demag_plan_bytes((nx, ny, nz, 4e-9, 4e-9, 4e-9)) == expect
    # the MFMA forms always take the five-pass form
    nx, ny, nz = 512, 512, 16
    X1, Y1, Z1 = nx + 1, ny + 1, nz + 1
    plane = 3 * nz * 2 * ny * 8
    planes = min(X1, (128 << 20) // plane)
    expect = 6 * Z1 * X1 * Y1 * 4 + 3 * nz * X1 * ny * 8 + planes * plane
    assert pkg.demag_plan_bytes((nx, ny, nz, 4e-9, 4e-9, 4e-9), flags=pkg.DEMAG_BF16X3_MFMA) == expect
    # three-kernel thin-mesh form: packed kernel + T[3][2nz][ceil((nx+1)/4)][ny][4]
    for nx, ny, nz in [(512, 512, 16), (32, 32, 4), (64, 16, 1), (1024, 512, 2)]:
        X1, Y1, Z1 = nx + 1, ny + 1, (nz + 1 if nz > 1 else 1)
        NZ = 2 * nz if nz > 1 else 1
        expect = 6 * Z1 * X1 * Y1 * 4 + 3 * NZ * ((X1 + 3) // 4) * ny * 4 * 8
        assert pkg.demag_plan_bytes((nx, ny, nz, 4e-9, 4e-9, 4e-9)) == expect, (nx, ny, nz)

def test_periodic_plan_bytes_and_flags():
    """Periodic axes: no padding (N_d = n_d, D1 = n_d/2 + 1), always the
    five-pass form, FP32 only; an image count needs a periodic axis."""
    for (nx, ny, nz), (px, py, pz) in [((512, 512, 16), (1, 1, 0)), ((64, 32, 8), (0, 1, 1)),
                                       ((128, 1, 4), (1, 0, 1)), ((32, 32, 32), (1, 1, 1))]:
        N = [v if p else (1 if v == 1 else 2 * v) for v, p in zip((nx, ny, nz), (px, py, pz))]
        X1, Y1, Z1 = (1 if v == 1 else v // 2 + 1 for v in N)
        s1 = 3 * nz * X1 * ny * 8
        plane = 3 * nz * N[1] * 8
        planes = X1 if ny == 1 else min(X1, (128 << 20) // plane)
        expect = 6 * Z1 * X1 * Y1 * 4 + s1 + (planes * plane if ny > 1 else 0)
        flags = pkg.pbc_flags(px, py, pz, images=3)
        assert pkg.demag_plan_bytes((nx, ny, nz, 4e-9, 4e-9, 4e-9), flags=flags) == expect
        assert pkg.kernel_shape((nx, ny, nz), (px, py, pz)) == (6, Z1, X1, Y1)
    mesh = (64, 64, 4, 4e-9, 4e-9, 4e-9)
    assert pkg.demag_plan_bytes(mesh, flags=pkg.DEMAG_PBC_X | pkg.DEMAG_BF16X3_MFMA) == 0
    assert pkg.demag_plan_bytes(mesh, flags=5 << pkg.DEMAG_PBC_IMAGES_SHIFT) == 0
    assert pkg.demag_plan_bytes(mesh, flags=pkg.DEMAG_PBC_Z | pkg.DEMAG_POINT_DIPOLE
                                | pkg.DEMAG_EXTRAPOLATE_HD | (255 << 8)) > 0
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup(mesh, pkg.DEMAG_PBC_Y | pkg.DEMAG_BF16X2_MFMA)
    assert e.value.status == pkg.DEMAG_EUNSUPPORTED
    assert b"DEMAG_FP32" in pkg.load().demag_last_error()
    with pytest.raises(pkg.DemagError) as e:
        pkg.atom_setup((16, 16, 8, 0.4e-9, 4), pkg.pbc_flags(x=True, images=2))
    assert e.value.status == pkg.DEMAG_EUNSUPPORTED
    with pytest.raises(ValueError):
        pkg.pbc_flags(x=True, images=256)


def test_mixed_radix_sizes_on_host():
    """n_x, n_y = F 2^j (F = 3, 5, 15; j >= 1) are accepted with DEMAG_FP32 and
    open boundaries; other sizes and flags are refused before any device work."""
    cell = (5e-9, 5e-9, 5e-9)
    nx, ny, nz = 480, 240, 2
    Nx, Ny, Nz = 960, 480, 4
    X1, Y1, Z1 = 481, 241, 3
    plane = 3 * nz * Ny * 8
    planes = min(X1, (128 << 20) // plane)
    expect = 6 * Z1 * X1 * Y1 * 4 + 3 * nz * X1 * ny * 8 + planes * plane
    assert pkg.demag_plan_bytes((nx, ny, nz) + cell) == expect
    for n in [(6, 10, 1), (1920, 6, 2), (30, 1, 4), (1536, 1280, 1)]:
        assert pkg.demag_plan_bytes(n + cell) > 0, n
    for n in [(3, 8, 1), (14, 8, 1), (45, 8, 1), (8, 8, 6), (3840, 2, 1), (8, 7, 1)]:
        assert pkg.demag_plan_bytes(n + cell) == 0, n
    assert pkg.demag_plan_bytes((480, 240, 2) + cell, flags=pkg.DEMAG_BF16X3_MFMA) == 0
    assert pkg.demag_plan_bytes((480, 240, 2) + cell, flags=pkg.pbc_flags(x=True, images=1)) == 0
    with pytest.raises(pkg.DemagError) as e:
        pkg.demag_setup((480, 240, 2) + cell, pkg.DEMAG_BF16X2_MFMA)
    assert e.value.status == pkg.DEMAG_EUNSUPPORTED


def test_switching_epsilon_and_schedule_on_host():
    """The mean relative error of two recorded <m> trajectories, and the
    workload's steps dividing its recording interval."""
    from paper_2308_08447_amd import switching as sw
    import workloads as W
    a = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.6, 0.8, 0.0]]
    b = [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.6, 0.8, 0.0]]
    assert abs(sw.epsilon(a, b) - 2 ** 0.5 / 3) < 1e-15
    assert sw.epsilon(a, a) == 0.0
    cfg = W.SWITCHING
    for dt in (cfg["dt_ref"],) + tuple(cfg["dts"]):
        k = cfg["record_every"] / dt
        assert abs(k - round(k)) < 1e-9


def test_inplace_flag_on_host():
    """DEMAG_INPLACE combines with every other flag and does not change the
    plan's memory; an unknown bit is still refused."""
    mesh = (64, 32, 4, 4e-9, 4e-9, 4e-9)
    for f in (0, pkg.DEMAG_BF16X3_MFMA, pkg.DEMAG_EXTRAPOLATE_HD, pkg.pbc_flags(x=True, images=2)):
        assert pkg.demag_plan_bytes(mesh, flags=f | pkg.DEMAG_INPLACE) == pkg.demag_plan_bytes(mesh, flags=f) > 0
    assert pkg.demag_plan_bytes(mesh, flags=1 << 30) == 0


class _DeviceStandIn:
    """Has the attributes the binding checks on a torch GPU tensor (no GPU here)."""

    def __init__(self, n, dtype="torch.float32", contiguous=True, cuda=True):
        self.n, self.dtype, self.contiguous, self.is_cuda = n, dtype, contiguous, cuda

    def is_contiguous(self):
        return self.contiguous

    def numel(self):
        return self.n

    def data_ptr(self):
        return 0x1000                   # every check runs before the library is called


def test_binding_refuses_bad_tensors_before_the_library():
    """The C ABI takes plain pointers, so the binding checks torch arguments
    against the plan's mesh first: a host tensor, another dtype, a strided view
    or a short buffer raises ValueError and nothing is called."""
    torch = pytest.importorskip("torch")
    plan = 0x5EED0                      # a handle the binding knows, never dereferenced
    pkg._PLAN_CELLS[plan] = 8 * 4 * 2
    need = 3 * 8 * 4 * 2
    try:
        good = _DeviceStandIn(need)
        with pytest.raises(ValueError, match="GPU tensor"):
            pkg.demag_field(plan, torch.zeros(need), good)
        with pytest.raises(ValueError, match="float32"):
            pkg.demag_field(plan, _DeviceStandIn(need, dtype="torch.float64"), good)
        with pytest.raises(ValueError, match="contiguous"):
            pkg.llg_step(plan, _DeviceStandIn(need, contiguous=False), (8e5, 1.3e-11, 0.1, 2.2e5, (0, 0, 0)),
                         1e-13, 1)
        with pytest.raises(ValueError, match="needs 192"):
            pkg.llg_step_noalloc(plan, _DeviceStandIn(need - 1), (8e5, 1.3e-11, 0.1, 2.2e5, (0, 0, 0)),
                                 1e-13, 1)
        with pytest.raises(ValueError, match="needs 192"):
            pkg.atom_step(plan, _DeviceStandIn(10), (1e-21, 2.0, 0.1, 1.76e11, (0, 0, 0)), 1e-15, 1)
        with pytest.raises(ValueError, match="needs 3"):
            pkg.demag_field_mean(plan, good, _DeviceStandIn(2))
        with pytest.raises(ValueError, match="needs 100"):
            pkg.demag_get_kernel(plan, _DeviceStandIn(99), 100)
    finally:
        del pkg._PLAN_CELLS[plan]


def test_binding_refuses_bad_host_arrays_before_the_library():
    import numpy as np
    server = 0x5EED1
    mesh = (8, 4, 2, 4e-9, 4e-9, 4e-9)
    params = (8e5, 1.3e-11, 0.1, 2.2e5, (0, 0, 0))
    with pytest.raises(ValueError, match="the mesh has 192"):
        pkg.serve_submit(server, mesh, params, 1e-13, 1, np.zeros(191, np.float32))
    pkg._REQ_CELLS[(server, 7)] = 8 * 4 * 2
    try:
        with pytest.raises(ValueError, match="float32"):
            pkg.serve_wait(server, 7, np.zeros(192, np.float64))
        with pytest.raises(ValueError, match="the mesh has 192"):
            pkg.serve_wait(server, 7, np.zeros(100, np.float32))
        with pytest.raises(ValueError, match="C-contiguous"):
            pkg.serve_wait(server, 7, np.zeros((192, 2), np.float32)[:, 0])
    finally:
        del pkg._REQ_CELLS[(server, 7)]
