"""MI355X (gfx950) demagnetizing-field engine: Python binding of the C ABI.

Every function here only marshals arguments to the shared library
``libdemag.so`` built from ``csrc/`` (see ``include/demag.h``); every step of the
computation runs in the library's HIP kernels.  There is no fallback: if the
library is missing or cannot be loaded, ``load()`` raises.

Device arrays are passed as torch GPU tensors or as raw device addresses (ints);
streams as torch streams or raw handles.  A torch tensor is checked before the
call (on the GPU, float32, contiguous, at least 3 n_x n_y n_z floats for the
plan's mesh), as are the host arrays of the server (float32, C-contiguous, the
request's size): the ABI takes plain pointers and cannot tell a host or short
buffer from a field, so a bad one raises ValueError here instead of faulting
the GPU.  Raw addresses are passed through unchecked.
"""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdemag.so")

DEMAG_OK = 0
DEMAG_EINVAL = -1
DEMAG_ENOMEM = -2
DEMAG_EUNSUPPORTED = -3
DEMAG_EHIP = -4
DEMAG_EBUSY = -5
DEMAG_FP32 = 0
DEMAG_BF16X2_MFMA = 1   # radix-16 passes as 2-term split BF16 MFMA products
DEMAG_BF16X3_MFMA = 2   # 3-term split
DEMAG_INPLACE = 4         # demag_field may write H over M
DEMAG_EXTRAPOLATE_HD = 8  # one H_d per RK4 step, quartic extrapolation at the sub-steps
DEMAG_POINT_DIPOLE = 16   # point-dipole kernel of the lattice dipole-dipole field (Eq. 8)
DEMAG_PBC_X = 32          # periodic axes (image-sum kernel, no padding; FP32 only)
DEMAG_PBC_Y = 64
DEMAG_PBC_Z = 128
DEMAG_PBC_IMAGES_SHIFT = 8


def pbc_flags(x=False, y=False, z=False, images=0):
    """Plan flags for the periodic axes (x, y, z) with `images` (0..255) copies
    summed on each side, or-ed into DEMAG_FP32."""
    if not 0 <= int(images) <= 255:
        raise ValueError("images must be in 0..255")
    f = (DEMAG_PBC_X if x else 0) | (DEMAG_PBC_Y if y else 0) | (DEMAG_PBC_Z if z else 0)
    return f | (int(images) << DEMAG_PBC_IMAGES_SHIFT) if f else 0

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EUNSUPPORTED", -4: "EHIP", -5: "EBUSY"}

# symbols declared in include/demag.h
EXPORTS = (
    "demag_setup", "demag_field", "demag_plan_bytes", "demag_get_kernel", "demag_destroy",
    "llg_step", "llg_reset", "demag_field_mean", "atom_setup", "atom_step", "atom_destroy",
    "demag_timing_enable",
    "demag_timing_read", "demag_autotune", "demag_set_variant", "demag_get_variant",
    "demag_set_chunks", "demag_get_chunks", "demag_get_form", "serve_open", "serve_submit", "serve_wait",
    "serve_get_stats", "serve_close", "demag_last_error", "llg_step_noalloc", "llg_noalloc_max_cells",
)
SERVE_GRAPHS = 1
NVARIANTS = 3
STAGES = ("x_fwd", "y_fwd", "z_conv", "y_inv", "x_inv", "llg")


class demag_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double)]


class llg_params(ctypes.Structure):
    _fields_ = [("Ms", ctypes.c_double), ("A", ctypes.c_double), ("alpha", ctypes.c_double),
                ("gamma", ctypes.c_double), ("Hzee", ctypes.c_double * 3)]


class atom_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("a", ctypes.c_double), ("macro", ctypes.c_int32)]


class atom_params(ctypes.Structure):
    _fields_ = [("J", ctypes.c_double), ("mu_s", ctypes.c_double), ("alpha", ctypes.c_double),
                ("gamma", ctypes.c_double), ("Hzee", ctypes.c_double * 3)]


class serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("active", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("cell_steps", ctypes.c_double), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("iterations", ctypes.c_uint64),
                ("graph_captures", ctypes.c_uint64)]


class DemagError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path=None):
    """Load the HIP library (once).  Raises if it is missing: there is no fallback."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library not built: {p} (run python -m paper_2308_08447_amd.build)")
    # A process must hold exactly one HIP runtime.  PyTorch wheels bundle their own
    # libamdhip64 under the same soname; loading torch first makes the library bind
    # to that copy instead of pulling a second runtime in from /opt/rocm.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "demag_setup": ([P(demag_mesh), ctypes.c_uint32, vp, P(vp)], ctypes.c_int),
        "demag_field": ([vp, vp, vp, vp], ctypes.c_int),
        "demag_plan_bytes": ([P(demag_mesh), ctypes.c_uint32], sz),
        "demag_get_kernel": ([vp, vp, sz, vp], ctypes.c_int),
        "demag_destroy": ([vp], ctypes.c_int),
        "llg_step": ([vp, vp, P(llg_params), ctypes.c_double, ctypes.c_int32, vp], ctypes.c_int),
        "llg_reset": ([vp], ctypes.c_int),
        "llg_step_noalloc": ([vp, vp, P(llg_params), ctypes.c_double, ctypes.c_int32, vp], ctypes.c_int),
        "llg_noalloc_max_cells": ([], sz),
        "demag_field_mean": ([vp, vp, vp, vp], ctypes.c_int),
        "atom_setup": ([P(atom_mesh), ctypes.c_uint32, vp, P(vp)], ctypes.c_int),
        "atom_step": ([vp, vp, P(atom_params), ctypes.c_double, ctypes.c_int32, vp], ctypes.c_int),
        "atom_destroy": ([vp], ctypes.c_int),
        "demag_timing_enable": ([vp, ctypes.c_int32], ctypes.c_int),
        "demag_timing_read": ([vp, P(ctypes.c_double), P(ctypes.c_int32)], ctypes.c_int),
        "demag_autotune": ([vp, vp], ctypes.c_int),
        "demag_set_variant": ([vp, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
        "demag_get_variant": ([vp, ctypes.c_int32, P(ctypes.c_int32)], ctypes.c_int),
        "demag_set_chunks": ([vp, ctypes.c_int32], ctypes.c_int),
        "demag_get_chunks": ([vp, P(ctypes.c_int32)], ctypes.c_int),
        "demag_get_form": ([vp, P(ctypes.c_int32)], ctypes.c_int),
        "serve_open": ([sz, ctypes.c_int32, ctypes.c_uint32, P(vp)], ctypes.c_int),
        "serve_submit": ([vp, P(demag_mesh), P(llg_params), ctypes.c_double, ctypes.c_int32, vp,
                          P(ctypes.c_uint64)], ctypes.c_int),
        "serve_wait": ([vp, ctypes.c_uint64, vp, P(ctypes.c_double)], ctypes.c_int),
        "serve_get_stats": ([vp, P(serve_stats)], ctypes.c_int),
        "serve_close": ([vp], ctypes.c_int),
        "demag_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


def last_error():
    return load().demag_last_error().decode()


def _check(status):
    if status != DEMAG_OK:
        raise DemagError(status, last_error())
    return status


def _ptr(x):
    """Device pointer of a torch tensor (or an int address / None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


# Cell count of each live plan (demag and atomistic) and of each pending served
# request, so that tensor arguments can be checked before they reach a kernel:
# the C ABI takes plain pointers and cannot tell a host buffer, a float64 tensor
# or a short one from a valid field.
_PLAN_CELLS = {}
_REQ_CELLS = {}


def _cells(mesh):
    return int(mesh.nx) * int(mesh.ny) * int(mesh.nz)


def _dev(x, need, name):
    """Pointer of a device float32 buffer of at least `need` elements.  Torch
    tensors are checked (GPU, float32, contiguous, size); an int is taken as a
    raw device address, unchecked, as the C ABI takes it."""
    if x is None or isinstance(x, int):
        return x
    if not getattr(x, "is_cuda", False):
        raise ValueError(f"{name} must be a GPU tensor: the kernels cannot read host memory")
    if str(x.dtype) != "torch.float32":
        raise ValueError(f"{name} must be float32, not {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous ([3][nz][ny][nx], x fastest)")
    if need is not None and x.numel() < need:
        raise ValueError(f"{name} holds {x.numel()} floats; the plan needs {need}")
    return x.data_ptr()


def _field(plan, x, name):
    cells = _PLAN_CELLS.get(plan)
    return _dev(x, None if cells is None else 3 * cells, name)


def _host(a, need, name):
    """Host float32 C-contiguous numpy array of exactly `need` elements."""
    import numpy as np
    if not isinstance(a, np.ndarray) or a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"]:
        raise ValueError(f"{name} must be a C-contiguous float32 numpy array")
    if need is not None and a.size != need:
        raise ValueError(f"{name} holds {a.size} floats; the mesh has {need}")
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---------------------------------------------------------------- C-ABI mirrors
def demag_setup(mesh, flags=DEMAG_FP32, stream=None):
    """mesh = (nx, ny, nz, dx, dy, dz) or a demag_mesh; returns an opaque plan handle."""
    if not isinstance(mesh, demag_mesh):
        mesh = demag_mesh(*mesh)
    out = ctypes.c_void_p()
    _check(load().demag_setup(ctypes.byref(mesh), flags, _stream(stream), ctypes.byref(out)))
    _PLAN_CELLS[out.value] = _cells(mesh)
    return out.value


def demag_field(plan, M, H, stream=None):
    pm, ph = _field(plan, M, "M"), _field(plan, H, "H")
    return _check(load().demag_field(plan, pm, ph, _stream(stream)))


def demag_plan_bytes(mesh, flags=DEMAG_FP32):
    if not isinstance(mesh, demag_mesh):
        mesh = demag_mesh(*mesh)
    return load().demag_plan_bytes(ctypes.byref(mesh), flags)


def demag_get_kernel(plan, dst, count, stream=None):
    pd = _dev(dst, int(count), "dst")
    return _check(load().demag_get_kernel(plan, pd, count, _stream(stream)))


def demag_destroy(plan):
    _PLAN_CELLS.pop(plan, None)
    return _check(load().demag_destroy(plan))


def llg_step(plan, m, params, dt, nsteps, stream=None):
    """params = (Ms, A, alpha, gamma, (Hx, Hy, Hz)) or an llg_params."""
    if not isinstance(params, llg_params):
        Ms, A, alpha, gamma, hz = params
        params = llg_params(Ms, A, alpha, gamma, (ctypes.c_double * 3)(*hz))
    pm = _field(plan, m, "m")
    return _check(load().llg_step(plan, pm, ctypes.byref(params), dt, nsteps, _stream(stream)))


def llg_step_noalloc(plan, m, params, dt, nsteps, stream=None):
    """llg_step without device allocation (RK4 buffers in the library's fixed
    per-GPU array; meshes up to llg_noalloc_max_cells() cells)."""
    if not isinstance(params, llg_params):
        Ms, A, alpha, gamma, hz = params
        params = llg_params(Ms, A, alpha, gamma, (ctypes.c_double * 3)(*hz))
    pm = _field(plan, m, "m")
    return _check(load().llg_step_noalloc(plan, pm, ctypes.byref(params), dt, nsteps,
                                          _stream(stream)))


def llg_noalloc_max_cells():
    return int(load().llg_noalloc_max_cells())


def demag_field_mean(plan, v, out, stream=None):
    """out[0:3] (device) = mean of each component of the [3][N] field v (device)."""
    pv, po = _field(plan, v, "v"), _dev(out, 3, "out")
    return _check(load().demag_field_mean(plan, pv, po, _stream(stream)))


def llg_reset(plan):
    return _check(load().llg_reset(plan))


def demag_timing_enable(plan, max_records):
    return _check(load().demag_timing_enable(plan, max_records))


def demag_timing_read(plan):
    """{stage name: (total_ms, launches)} since the last read."""
    n = len(STAGES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int32 * n)()
    _check(load().demag_timing_read(plan, ms, cnt))
    return {STAGES[i]: (ms[i], cnt[i]) for i in range(n)}


def demag_autotune(plan, stream=None):
    return _check(load().demag_autotune(plan, _stream(stream)))


def demag_set_variant(plan, stage, variant):
    return _check(load().demag_set_variant(plan, stage, variant))


def demag_get_variant(plan, stage):
    v = ctypes.c_int32()
    _check(load().demag_get_variant(plan, stage, ctypes.byref(v)))
    return v.value


def demag_set_chunks(plan, nchunks):
    return _check(load().demag_set_chunks(plan, nchunks))


def demag_get_chunks(plan):
    v = ctypes.c_int32()
    _check(load().demag_get_chunks(plan, ctypes.byref(v)))
    return v.value


DEMAG_FORM_FIVE_PASS = 5
DEMAG_FORM_THIN = 3


def demag_get_form(plan):
    """DEMAG_FORM_FIVE_PASS or DEMAG_FORM_THIN (the three-kernel thin-mesh form)."""
    v = ctypes.c_int32()
    _check(load().demag_get_form(plan, ctypes.byref(v)))
    return v.value


def atom_setup(mesh, flags=DEMAG_FP32, stream=None):
    """mesh = (nx, ny, nz, a, macro) or an atom_mesh."""
    if not isinstance(mesh, atom_mesh):
        mesh = atom_mesh(*mesh)
    out = ctypes.c_void_p()
    _check(load().atom_setup(ctypes.byref(mesh), flags, _stream(stream), ctypes.byref(out)))
    _PLAN_CELLS[out.value] = _cells(mesh)
    return out.value


def atom_step(plan, S, params, dt, nsteps, stream=None):
    """params = (J, mu_s, alpha, gamma, (Hx, Hy, Hz)) or an atom_params."""
    if not isinstance(params, atom_params):
        J, mu_s, alpha, gamma, hz = params
        params = atom_params(J, mu_s, alpha, gamma, (ctypes.c_double * 3)(*hz))
    ps = _field(plan, S, "S")
    return _check(load().atom_step(plan, ps, ctypes.byref(params), dt, nsteps, _stream(stream)))


def atom_destroy(plan):
    _PLAN_CELLS.pop(plan, None)
    return _check(load().atom_destroy(plan))


def _llg(params):
    if isinstance(params, llg_params):
        return params
    Ms, A, alpha, gamma, hz = params
    return llg_params(Ms, A, alpha, gamma, (ctypes.c_double * 3)(*hz))


def serve_open(hbm_budget_bytes, max_active=64, flags=0):
    out = ctypes.c_void_p()
    _check(load().serve_open(int(hbm_budget_bytes), max_active, flags, ctypes.byref(out)))
    return out.value


def serve_submit(server, mesh, params, dt, nsteps, m0_host):
    """m0_host: C-contiguous float32 numpy array [3][nz][ny][nx] (copied)."""
    import numpy as np
    if not isinstance(mesh, demag_mesh):
        mesh = demag_mesh(*mesh)
    m0 = np.ascontiguousarray(m0_host, dtype=np.float32)
    pm = _host(m0, 3 * _cells(mesh), "m0_host")
    rid = ctypes.c_uint64()
    _check(load().serve_submit(server, ctypes.byref(mesh), ctypes.byref(_llg(params)), dt, nsteps,
                               pm, ctypes.byref(rid)))
    _REQ_CELLS[(server, rid.value)] = _cells(mesh)
    return rid.value


def serve_wait(server, request_id, m_out_host):
    """Blocks until done; fills m_out_host (float32, C-contiguous); returns latency in s."""
    cells = _REQ_CELLS.get((server, request_id))
    pm = _host(m_out_host, None if cells is None else 3 * cells, "m_out_host")
    lat = ctypes.c_double()
    _check(load().serve_wait(server, request_id, pm, ctypes.byref(lat)))
    _REQ_CELLS.pop((server, request_id), None)
    return lat.value


def serve_get_stats(server):
    st = serve_stats()
    _check(load().serve_get_stats(server, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in serve_stats._fields_}


def serve_close(server):
    for key in [k for k in _REQ_CELLS if k[0] == server]:
        del _REQ_CELLS[key]
    return _check(load().serve_close(server))


def kernel_shape(n, pbc=(False, False, False)):
    """(6, Z1, X1, Y1) of the packed kernel for a mesh n = (nx, ny, nz) with the
    periodic axes pbc: D1 = N/2 + 1 with N = 2n (open) or n (periodic), 1 for N = 1."""
    d = [1 if v == 1 else (v // 2 + 1 if p else v + 1) for v, p in zip(n, pbc)]
    return (6, d[2], d[0], d[1])
