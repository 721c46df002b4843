"""Mesh sizes 3, 5 or 15 times a power of two along x and y (radix-3 and radix-5
passes) against the FP64 oracle, through the C ABI.  Tolerance: relative L2
<= 2e-5 per field component, as for the power-of-two meshes."""

import numpy as np
import pytest

import workloads as W
from oracle import demag as odemag
from oracle import llg as ollg

pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def torch_dev(gpu_lib):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)


def _field(pkg, torch, n, cell, M):
    plan = pkg.demag_setup(tuple(n) + tuple(cell))
    try:
        assert pkg.demag_get_form(plan) == pkg.DEMAG_FORM_FIVE_PASS
        Md = torch.from_numpy(M).cuda()
        Hd = torch.empty_like(Md)
        pkg.demag_field(plan, Md, Hd)
        torch.cuda.synchronize()
        return Hd.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)


# every odd factor with short and long power-of-two parts, mixed with power-of-two
# and single-cell axes; the switching problem's mesh 480 x 240 x 2
SHAPES = [
    (6, 10, 2), (30, 12, 4), (480, 240, 2), (10, 6, 1), (12, 20, 8), (96, 160, 4),
    (1920, 6, 1), (6, 1920, 1), (1536, 4, 2), (4, 1280, 1), (60, 1, 4), (1, 120, 2),
    (24, 64, 16), (640, 30, 1), (48, 960, 1),
]


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_mixed_field_matches_oracle(torch_dev, n):
    import paper_2308_08447_amd as pkg
    _say("mixed-radix field parity", n)
    cell = (5e-9, 5e-9, 5e-9)
    M = W.magnetisation(n, seed=sum(n) + 3)
    H = _field(pkg, torch_dev, n, cell, M)
    Href = odemag.demag_fft(M.astype(np.float64), cell, workers=8)
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("n,cell", [((30, 12, 4), (5e-9, 4e-9, 3e-9)), ((480, 240, 2), (5e-9,) * 3)])
def test_mixed_kernel_matches_oracle_spectrum(torch_dev, n, cell):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("mixed-radix kernel spectrum", n, cell)
    plan = pkg.demag_setup(tuple(n) + tuple(cell))
    try:
        shape = pkg.kernel_shape(n)
        K = torch.empty(int(np.prod(shape)), dtype=torch.float32, device="cuda")
        pkg.demag_get_kernel(plan, K, K.numel())
        torch.cuda.synchronize()
        K = K.cpu().numpy().reshape(shape).astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    op = odemag.DemagFFT(n, cell)
    Nx, Ny, Nz = op.N
    _, Z1, X1, Y1 = shape
    ref = np.stack([-op.Khat[c].real[:Z1, :Y1, :X1].transpose(0, 2, 1) / (Nx * Ny * Nz)
                    for c in range(6)])
    err = np.abs(K - ref).max(axis=(1, 2, 3)) / np.abs(ref).max()
    _say("  max error per component / max |K|", err)
    assert np.all(err <= 1e-6), err


def test_mixed_variants_and_chunks_are_bit_identical(torch_dev):
    """Chunking of the y/z stages does not change a mixed-size result."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n = (480, 240, 2)
    M = torch.from_numpy(W.magnetisation(n, seed=8)).cuda()
    plan = pkg.demag_setup(n + (5e-9,) * 3)
    try:
        H1, H2 = torch.empty_like(M), torch.empty_like(M)
        pkg.demag_field(plan, M, H1)
        pkg.demag_set_chunks(plan, 7)
        pkg.demag_field(plan, M, H2)
        torch.cuda.synchronize()
        assert torch.equal(H1, H2)
    finally:
        pkg.demag_destroy(plan)


def test_mixed_llg_matches_oracle(torch_dev):
    """Three RK4 steps of the switching problem's mesh (480 x 240 x 2, 5 nm
    cells) from a random state with the switching field on."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.SWITCHING
    n, cell = cfg["n"], cfg["cell"]
    steps, dt = 3, 2e-13
    _say("mixed-radix llg parity", n, steps)
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=31)
    prm = (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, cfg["H_switch"])
    plan = pkg.demag_setup(n + cell)
    try:
        m = torch.from_numpy(m0).cuda()
        pkg.llg_step(plan, m, prm, dt, steps)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    ref = ollg.LLG(n, cell, cfg["Ms"], cfg["A"], cfg["alpha"], Hzee=cfg["H_switch"],
                   workers=8).run(m0.astype(np.float64), dt, steps)
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of m", err)
    assert err <= TOL


@pytest.mark.parametrize("n", [(480, 240, 2), (96, 160, 4)], ids=lambda n: "x".join(map(str, n)))
def test_mixed_autotune_keeps_the_result(torch_dev, n):
    """Autotuning a mixed-radix plan (one tile shape; chunk counts searched)
    leaves its result bitwise unchanged."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    M = torch.from_numpy(W.magnetisation(n, seed=12)).cuda()
    plan = pkg.demag_setup(tuple(n) + (5e-9,) * 3)
    try:
        H1, H2 = torch.empty_like(M), torch.empty_like(M)
        pkg.demag_field(plan, M, H1)
        pkg.demag_autotune(plan)
        pkg.demag_field(plan, M, H2)
        torch.cuda.synchronize()
        assert torch.equal(H1, H2)
    finally:
        pkg.demag_destroy(plan)
