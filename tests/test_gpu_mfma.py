"""Split-precision BF16 MFMA forms of the FFT stages against the FP64 oracle.

The radix-16 passes run as BF16 DFT-matrix products on the matrix cores with
FP32 accumulation (three-term operand splits); the result definition and the
tolerance are those of the FP32 path (rel-L2 <= 2e-5 per field).  The two-term
split is refused by demag_setup (it misses 2e-5 where the field is small against
the largest spectral values); its refusal is tested on the host in test_abi.
"""

import numpy as np
import pytest

import workloads as W
from oracle import demag as odemag
from oracle import llg as ollg
from oracle import newell as onewell

pytestmark = pytest.mark.gpu

TOL = 2e-5
MODES = [(2, "bf16x3")]

# every radix plan shape: L = 16 (single matrix pass), 2*16, 4*16, 8*16, 16*16,
# 8*16*16 (x of 2048), 16*16*16 (y of 4096), z of 32, 64, 128, 256; ragged tiles
SHAPES = [
    (16, 16, 16), (32, 32, 4), (64, 32, 8), (128, 64, 2), (256, 16, 2), (16, 256, 1),
    (8, 4, 64), (4, 4, 128), (2048, 4, 1), (4, 2048, 2), (8, 8, 8), (1, 1, 1), (2, 1, 1),
    (1, 8, 1), (32, 64, 1),
]


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def torch_dev(gpu_lib):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _field(pkg, torch, n, cell, M, flags):
    nx, ny, nz = n
    plan = pkg.demag_setup((nx, ny, nz) + tuple(cell), flags)
    try:
        Md = torch.from_numpy(M).cuda()
        Hd = torch.empty_like(Md)
        pkg.demag_field(plan, Md, Hd)
        torch.cuda.synchronize()
        return Hd.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("flags,name", MODES, ids=[m[1] for m in MODES])
@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_mfma_field_matches_oracle(gpu_lib, torch_dev, n, flags, name):
    import paper_2308_08447_amd as pkg
    _say("mfma parity", name, n)
    cell = W.CELL_4NM
    M = W.magnetisation(n, seed=sum(n) + 7)
    H = _field(pkg, torch_dev, n, cell, M, flags)
    Href = odemag.demag_fft(M.astype(np.float64), cell)
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("flags,name", MODES, ids=[m[1] for m in MODES])
def test_mfma_thin_film(gpu_lib, torch_dev, flags, name):
    """512x512x16 (4 nm cubes), seeded random M: whole-field parity."""
    import paper_2308_08447_amd as pkg
    n, cell = W.THIN_FILM["n"], W.THIN_FILM["cell"]
    _say("mfma thin film", name)
    M = W.magnetisation(n, seed=0)
    H = _field(pkg, torch_dev, n, cell, M, flags)
    errs = odemag.rel_l2_per_field(H, odemag.demag_fft(M.astype(np.float64), cell, workers=8))
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("flags,name", MODES, ids=[m[1] for m in MODES])
def test_mfma_large_film_sparse_sources(gpu_lib, torch_dev, flags, name):
    """1024x1024x32 (4 nm cubes): M non-zero in 400 random cells, exact direct
    sum of Eq. (1) at 16 sampled targets."""
    import paper_2308_08447_amd as pkg
    n, cell = W.LARGE_FILM["n"], W.LARGE_FILM["cell"]
    _say("mfma large film sparse sources", name)
    M, src, tg = W.sparse_sources(n, 400, 16, seed=12)
    H = _field(pkg, torch_dev, n, cell, M, flags)
    Mv = M[:, src[:, 2], src[:, 1], src[:, 0]].astype(np.float64)
    ref = np.zeros((3, len(tg)))
    for t, (x, y, z) in enumerate(tg):
        T = odemag.tensor3(onewell.tensor(x - src[:, 0], y - src[:, 1], z - src[:, 2], cell))
        for a in range(3):
            ref[a, t] = -sum(np.dot(T[a][b], Mv[b]) for b in range(3))
    got = np.stack([H[:, z, y, x] for x, y, z in tg], 1)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say("  rel-L2 at targets", err)
    assert err <= TOL


@pytest.mark.parametrize("flags,name", MODES, ids=[m[1] for m in MODES])
def test_mfma_deterministic(gpu_lib, torch_dev, flags, name):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n = (64, 64, 8)
    M = torch.from_numpy(W.magnetisation(n, seed=5)).cuda()
    plan = pkg.demag_setup(n + W.CELL_4NM, flags)
    try:
        H1, H2 = torch.empty_like(M), torch.empty_like(M)
        pkg.demag_field(plan, M, H1)
        pkg.demag_field(plan, M, H2)
        torch.cuda.synchronize()
        assert torch.equal(H1, H2)
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("flags,name", MODES, ids=[m[1] for m in MODES])
def test_mfma_llg_matches_oracle(gpu_lib, torch_dev, flags, name):
    """Three RK4 steps of a 64x32x4 film (Zeeman field on) with the MFMA demag."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n, steps = (64, 32, 4), 3
    _say("mfma llg parity", name, n, steps)
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=13)
    alpha, dt, Hz = 0.02, 1e-13, (1e4, -2e4, 3e4)
    plan = pkg.demag_setup(n + W.CELL_4NM, flags)
    try:
        m = torch.from_numpy(m0).cuda()
        pkg.llg_step(plan, m, (W.MS, W.A_EX, alpha, ollg.GAMMA, Hz), dt, steps)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    ref = ollg.LLG(n, W.CELL_4NM, W.MS, W.A_EX, alpha, Hzee=Hz).run(m0.astype(np.float64), dt, steps)
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of m", err)
    assert err <= TOL
