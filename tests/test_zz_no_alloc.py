"""llg_step_noalloc: RK4 steps whose stage buffers are the library's fixed
per-GPU array instead of plan allocations.  Through the C ABI, its result must
be bitwise the result of llg_step (same kernels, same arithmetic), on two calls
in a row, the second on a smaller mesh (the array keeps the first call's
contents), and meshes above the fixed limit are refused on the host.
"""

import numpy as np
import pytest

import workloads as W
from oracle import llg as ollg

pytestmark = pytest.mark.gpu


def _steps(pkg, torch, n, seed, alpha, nsteps, noalloc):
    plan = pkg.demag_setup(tuple(n) + W.CELL_4NM)
    try:
        m = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed)).cuda()
        prm = (W.MS, W.A_EX, alpha, ollg.GAMMA, (1.0e3, -2.0e3, 5.0e2))
        if noalloc:
            pkg.llg_step_noalloc(plan, m, prm, 1e-13, nsteps)
        else:
            pkg.llg_step(plan, m, prm, 1e-13, nsteps)
        torch.cuda.synchronize()
        return m.cpu().numpy()
    finally:
        pkg.demag_destroy(plan)


def test_noalloc_equals_llg_step_twice_shrinking(gpu_lib):
    import torch
    import paper_2308_08447_amd as pkg
    assert torch.cuda.is_available()
    cases = [((128, 64, 8), 3, 0.1, 4), ((32, 32, 4), 5, 0.3, 3)]  # second call smaller
    for n, seed, alpha, nsteps in cases:
        print("llg_step_noalloc vs llg_step", n, "seed", seed, flush=True)
        got = _steps(pkg, torch, n, seed, alpha, nsteps, noalloc=True)
        ref = _steps(pkg, torch, n, seed, alpha, nsteps, noalloc=False)
        assert np.isfinite(got).all()
        assert np.array_equal(got, ref), f"{n}: max |diff| {np.abs(got - ref).max()}"


def test_noalloc_limits(gpu_lib):
    import torch
    import paper_2308_08447_amd as pkg
    assert torch.cuda.is_available()
    cap = pkg.llg_noalloc_max_cells()
    assert cap == (64 << 20) // 48
    # 512 x 512 x 16 cells need 201 MB of stage buffers: refused before any launch
    plan = pkg.demag_setup((512, 512, 16) + W.CELL_4NM)
    try:
        m = torch.zeros((3, 16, 512, 512), dtype=torch.float32, device="cuda")
        m[2] = 1.0
        with pytest.raises(RuntimeError, match="EINVAL"):
            pkg.llg_step_noalloc(plan, m, (W.MS, W.A_EX, 0.02, ollg.GAMMA, (0.0, 0.0, 0.0)), 1e-13, 1)
        assert float(m[2].min()) == 1.0 and float(m[0].abs().max()) == 0.0
    finally:
        pkg.demag_destroy(plan)
    plan = pkg.demag_setup((32, 32, 4) + W.CELL_4NM, pkg.DEMAG_EXTRAPOLATE_HD)
    try:
        m = torch.from_numpy(W.unit_vectors((4, 32, 32), 1)).cuda()
        with pytest.raises(RuntimeError, match="EUNSUPPORTED"):
            pkg.llg_step_noalloc(plan, m, (W.MS, W.A_EX, 0.02, ollg.GAMMA, (0.0, 0.0, 0.0)), 1e-13, 1)
    finally:
        pkg.demag_destroy(plan)
