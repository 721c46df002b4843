"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerance: relative L2 <= 2e-5 per field component for the demagnetizing field
(FP32 FFT stages; the expected error is ~1e-7).  Inputs are the same seeded FP32
arrays on both sides (workloads.magnetisation), so input rounding is not error.
"""

import numpy as np
import pytest

import workloads as W
from oracle import atomistic as oatom
from oracle import demag as odemag
from oracle import llg as ollg
from oracle import newell as onewell

pytestmark = pytest.mark.gpu

TOL = 2e-5


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)


def _gpu_field(pkg, torch, n, cell, M):
    nx, ny, nz = n
    plan = pkg.demag_setup((nx, ny, nz) + tuple(cell))
    try:
        Md = torch.from_numpy(M).cuda()
        Hd = torch.empty_like(Md)
        pkg.demag_field(plan, Md, Hd)
        torch.cuda.synchronize()
        return Hd.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)


SHAPES = [
    (32, 32, 4), (1, 1, 1), (2, 1, 1), (1, 8, 1), (8, 1, 1), (16, 1, 4), (4, 4, 2),
    (8, 8, 8), (64, 32, 8), (128, 64, 2), (32, 64, 1), (8, 4, 64), (4, 4, 128),
    (256, 16, 2), (16, 256, 1), (2048, 4, 1), (4, 2048, 2),
    # three-kernel thin-mesh form (32 <= nx <= 1024, 16 <= ny <= 1024, nz <= 16)
    (1024, 64, 4), (512, 32, 16), (128, 512, 16), (64, 16, 16), (32, 16, 1), (1024, 16, 16),
    (256, 128, 8), (32, 512, 2), (64, 1024, 2), (256, 1024, 1), (32, 1024, 16),
    # five-pass form beside it (n_z = 32)
    (32, 16, 32), (128, 32, 32),
]


@pytest.mark.parametrize("n", SHAPES, ids=lambda n: "x".join(map(str, n)))
def test_field_matches_oracle(gpu_lib, torch_dev, n):
    import paper_2308_08447_amd as pkg
    _say("demag_field parity", n)
    cell = W.CELL_4NM
    M = W.magnetisation(n, seed=sum(n))
    H = _gpu_field(pkg, torch_dev, n, cell, M)
    Href = odemag.demag_fft(M.astype(np.float64), cell)
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("n", [(8, 8, 4), (32, 16, 4)], ids=["8x8x4", "32x16x4"])
def test_field_matches_direct_sum_small(gpu_lib, torch_dev, n):
    import paper_2308_08447_amd as pkg
    cell = (4e-9, 3e-9, 2e-9)
    _say("demag_field vs direct sum", n, cell)
    M = W.magnetisation(n, seed=3)
    H = _gpu_field(pkg, torch_dev, n, cell, M)
    Href = odemag.demag_direct(M.astype(np.float64), cell)
    assert max(odemag.rel_l2_per_field(H, Href)) <= TOL


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_demag_small_config(gpu_lib, torch_dev, seed):
    """32x32x4 cells of 4 nm, Ms = 8e5, seeded random unit M: FP64 oracle and direct sum."""
    import paper_2308_08447_amd as pkg
    n, cell = W.DEMAG_SMALL["n"], W.DEMAG_SMALL["cell"]
    _say("demag 32x32x4 seed", seed)
    M = W.magnetisation(n, seed)
    H = _gpu_field(pkg, torch_dev, n, cell, M)
    Href = odemag.demag_fft(M.astype(np.float64), cell)
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL
    targets = np.array([[0, 0, 0], [31, 31, 3], [13, 7, 2], [31, 0, 1]])
    direct = odemag.demag_at(M.astype(np.float64), cell, targets)
    for t, (x, y, z) in enumerate(targets):
        np.testing.assert_allclose(H[:, z, y, x], direct[:, t], rtol=0,
                                   atol=TOL * np.abs(Href).max())


@pytest.mark.parametrize("n,cell", [((16, 8, 4), (4e-9, 4e-9, 4e-9)), ((8, 1, 2), (1e-9, 2e-9, 3e-9)),
                                    ((1, 1, 1), (2e-9, 2e-9, 2e-9)), ((32, 32, 4), W.CELL_4NM)])
def test_kernel_matches_oracle_spectrum(gpu_lib, torch_dev, n, cell):
    """The packed FP32 kernel equals -N^/(NxNyNz) of the oracle's transformed tensor."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("kernel spectrum", n, cell)
    nx, ny, nz = n
    plan = pkg.demag_setup((nx, ny, nz) + tuple(cell))
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
    # oracle rfftn output is [kz][ky][kx] with kx <= Nx/2
    ref = np.stack([-op.Khat[c].real[:Z1, :Y1, :X1].transpose(0, 2, 1) / (Nx * Ny * Nz)
                    for c in range(6)])
    scale = np.abs(ref).max()  # one scale: some components vanish identically by parity
    err = np.abs(K - ref).max(axis=(1, 2, 3)) / scale
    _say("  max error per component / max |K|", err)
    assert np.all(err <= 1e-6), err


def test_field_full_thin_film(gpu_lib, torch_dev):
    """512x512x16 (4 nm cubes), seeded random M: whole field against the FP64 oracle."""
    import paper_2308_08447_amd as pkg
    n, cell = W.THIN_FILM["n"], W.THIN_FILM["cell"]
    _say("demag 512x512x16 full-field parity")
    M = W.magnetisation(n, 0)
    H = _gpu_field(pkg, torch_dev, n, cell, M)
    Href = odemag.DemagFFT(n, cell, workers=8)(M.astype(np.float64))
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL


def _sparse_direct(M, src, tg, cell):
    """H at the targets = -sum over the non-zero source cells of N(t - s) M_s."""
    Mv = M[:, src[:, 2], src[:, 1], src[:, 0]].astype(np.float64)
    out = np.zeros((3, len(tg)))
    for t, (x, y, z) in enumerate(tg):
        T = odemag.tensor3(onewell.tensor(x - src[:, 0], y - src[:, 1], z - src[:, 2], cell))
        for a in range(3):
            out[a, t] = -sum(np.dot(T[a][b], Mv[b]) for b in range(3))
    return out


@pytest.mark.parametrize("n,cell", [((1024, 1024, 32), W.CELL_4NM),
                                    ((256, 256, 64), (1.6e-9, 1.6e-9, 1.6e-9))],
                         ids=["1024x1024x32", "256x256x64-macro"])
def test_full_size_sparse_sources(gpu_lib, torch_dev, n, cell):
    """Full-size meshes (the large film and the atomistic macrocell mesh): M is
    non-zero in 400 random cells, so the exact direct sum of Eq. (1) at sampled
    targets is cheap; the whole FFT pipeline still runs at full size."""
    import paper_2308_08447_amd as pkg
    _say("sparse-source parity", n)
    M, src, tg = W.sparse_sources(n, 400, 16, seed=11)
    H = _gpu_field(pkg, torch_dev, n, cell, M)
    ref = _sparse_direct(M, src, tg, cell)
    got = np.stack([H[:, z, y, x] for x, y, z in tg], 1)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say("  rel-L2 at targets", err)
    assert err <= TOL


def test_field_is_deterministic(gpu_lib, torch_dev):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n = (64, 64, 8)
    _say("determinism", n)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        M = torch.from_numpy(W.magnetisation(n, 5)).cuda()
        H1, H2 = torch.empty_like(M), torch.empty_like(M)
        pkg.demag_field(plan, M, H1)
        pkg.demag_field(plan, M, H2)
        torch.cuda.synchronize()
        assert torch.equal(H1, H2)
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("n", [(64, 32, 8), (32, 64, 1), (16, 8, 32), (128, 4, 2), (16, 1, 8),
                               (32, 64, 32), (32, 16, 32)],
                         ids=lambda n: "x".join(map(str, n)))
def test_variants_are_bit_identical(gpu_lib, torch_dev, n):
    """Every tile-shape variant of every stage, and the autotuned choice, give the
    same bits (the per-line arithmetic does not depend on the tile shape).  At
    N_z = 64 the z stage's variants are different kernels: the register form
    (variants 0 and 2) and the lean LDS form (variant 1) at 32x64x32, the
    register form and the general kernel at 32x16x32."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("variants", n)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        M = torch.from_numpy(W.magnetisation(n, 8)).cuda()
        ref = torch.empty_like(M)
        pkg.demag_field(plan, M, ref)
        for v in range(pkg.NVARIANTS):
            for st in range(5):
                pkg.demag_set_variant(plan, st, v)
            H = torch.empty_like(M)
            pkg.demag_field(plan, M, H)
            torch.cuda.synchronize()
            assert torch.equal(H, ref), v
        for v in range(pkg.NVARIANTS):
            for st in range(5):
                pkg.demag_set_variant(plan, st, v)
            for nch in (1, 2, 3, 7):
                pkg.demag_set_chunks(plan, nch)
                H = torch.empty_like(M)
                pkg.demag_field(plan, M, H)
                torch.cuda.synchronize()
                assert torch.equal(H, ref), (v, nch)
        pkg.demag_autotune(plan)
        chosen = [pkg.demag_get_variant(plan, st) for st in range(5)]
        _say("  autotuned variants", chosen, "chunks", pkg.demag_get_chunks(plan))
        H = torch.empty_like(M)
        pkg.demag_field(plan, M, H)
        torch.cuda.synchronize()
        assert torch.equal(H, ref)
        Href = odemag.demag_fft(M.cpu().numpy().astype(np.float64), W.CELL_4NM)
        assert max(odemag.rel_l2_per_field(ref.cpu().numpy(), Href)) <= TOL
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("n", [(64, 256, 4), (32, 512, 2), (1024, 32, 16), (32, 1024, 2)],
                         ids=lambda n: "x".join(map(str, n)))
def test_thin_form_variants(gpu_lib, torch_dev, n):
    """Thin-mesh form: the row pairs per round of the two xz kernels (variants of
    stages 0 and 4) give the same bits; the y convolution's variants (0: 128
    threads, radix order 16 8 8; 1: 256 threads, 16 16 4, one plane per block;
    2: as 1 with both mirror planes per block) each meet the contract against
    the oracle, 1 and 2 bit for bit the same; the autotuned plan reproduces the
    bits of the variants it picked."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("thin-form variants", n)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        assert pkg.demag_get_form(plan) == pkg.DEMAG_FORM_THIN
        M = torch.from_numpy(W.magnetisation(n, 9)).cuda()
        Href = odemag.demag_fft(M.cpu().numpy().astype(np.float64), W.CELL_4NM)
        per_conv = {}
        for vc in (0, 1, 2):
            pkg.demag_set_variant(plan, 2, vc)
            ref = None
            for v in range(pkg.NVARIANTS):
                pkg.demag_set_variant(plan, 0, v)
                pkg.demag_set_variant(plan, 4, (v + 1) % pkg.NVARIANTS)
                H = torch.empty_like(M)
                pkg.demag_field(plan, M, H)
                torch.cuda.synchronize()
                if ref is None:
                    ref = H
                assert torch.equal(H, ref), (vc, v)
            errs = odemag.rel_l2_per_field(ref.cpu().numpy().astype(np.float64), Href)
            _say("  y conv variant", vc, "rel-L2", errs)
            assert max(errs) <= TOL, (vc, errs)
            per_conv[vc] = ref
        assert torch.equal(per_conv[1], per_conv[2])
        pkg.demag_autotune(plan)
        chosen = [pkg.demag_get_variant(plan, st) for st in range(5)]
        _say("  autotuned variants", chosen)
        H = torch.empty_like(M)
        pkg.demag_field(plan, M, H)
        torch.cuda.synchronize()
        assert torch.equal(H, per_conv[chosen[2]])
    finally:
        pkg.demag_destroy(plan)


def test_abi_rejects_bad_arguments(gpu_lib, torch_dev):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    plan = pkg.demag_setup((8, 8, 2) + W.CELL_4NM)
    try:
        M = torch.zeros(3 * 8 * 8 * 2, device="cuda")
        with pytest.raises(pkg.DemagError) as e:
            pkg.demag_field(plan, M, M)
        assert e.value.status == pkg.DEMAG_EINVAL
        with pytest.raises(pkg.DemagError):
            pkg.llg_step(plan, M, (8e5, 1.3e-11, 0.1, 2.21e5, (0, 0, 0)), 1e-13, -1)
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("n,nch", [((128, 64, 8), 1), ((64, 32, 32), 3)], ids=["thin", "five-pass"])
def test_stage_timing_counts_and_bounds(gpu_lib, torch_dev, n, nch):
    """Per-stage timing: each timed launch takes its record's two events, so
    every stage launch is counted once, each recorded time is positive, the
    recorded kernel times of K evaluations add up to no more than their wall
    time, and the field is the same bits as untimed.  RK4 steps record four
    LLG stage launches each."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("stage timing", n, nch)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        thin = pkg.demag_get_form(plan) == pkg.DEMAG_FORM_THIN
        if not thin:
            pkg.demag_set_chunks(plan, nch)
        nch = pkg.demag_get_chunks(plan)
        M = torch.from_numpy(W.magnetisation(n, 3)).cuda()
        ref = torch.empty_like(M)
        pkg.demag_field(plan, M, ref)
        K = 3
        pkg.demag_timing_enable(plan, K * nch)
        H = torch.empty_like(M)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(K):
            pkg.demag_field(plan, M, H)
        e1.record()
        torch.cuda.synchronize()
        rec = pkg.demag_timing_read(plan)
        wall_ms = e0.elapsed_time(e1)
        want = {"x_fwd": K, "z_conv": K, "x_inv": K} if thin else \
            {"x_fwd": K, "y_fwd": K * nch, "z_conv": K * nch, "y_inv": K * nch, "x_inv": K}
        _say("  records", rec, "wall ms", wall_ms)
        for st, cnt in want.items():
            assert rec[st][1] == cnt, (st, rec[st])
            assert rec[st][0] > 0.0, (st, rec[st])
        assert rec["llg"][1] == 0
        assert sum(rec[st][0] for st in want) <= wall_ms
        assert torch.equal(H, ref)
        m = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed=4)).cuda()
        pkg.demag_timing_enable(plan, 4 * 2 * nch)
        pkg.llg_step(plan, m, (W.MS, W.A_EX, 0.1, ollg.GAMMA, (0, 0, 0)), 1e-13, 2)
        torch.cuda.synchronize()
        rec = pkg.demag_timing_read(plan)
        assert rec["llg"][1] == 8 and rec["llg"][0] > 0.0
        assert rec["x_fwd"][1] == 8
        pkg.demag_timing_enable(plan, 0)
    finally:
        pkg.demag_destroy(plan)


# ------------------------------------------------------------------ LLG (RK4)
@pytest.mark.parametrize("n,steps", [((16, 8, 2), 1), ((16, 8, 2), 10), ((32, 32, 4), 10),
                                     ((1, 1, 1), 20), ((64, 1, 1), 5)])
def test_llg_matches_oracle(gpu_lib, torch_dev, n, steps):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("llg_step parity", n, steps)
    nx, ny, nz = n
    m0 = W.unit_vectors((nz, ny, nx), seed=11)
    alpha, dt, Hz = 0.02, 1e-13, (1e4, -2e4, 3e4)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        m = torch.from_numpy(m0).cuda()
        pkg.llg_step(plan, m, (W.MS, W.A_EX, alpha, ollg.GAMMA, Hz), dt, steps)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    prob = ollg.LLG(n, W.CELL_4NM, W.MS, W.A_EX, alpha, Hzee=Hz)
    ref = prob.run(m0.astype(np.float64), dt, steps)
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of m", err)
    assert err <= TOL
    np.testing.assert_allclose(np.linalg.norm(got, axis=0), 1.0, atol=1e-6)


def test_llg_thin_film_one_step(gpu_lib, torch_dev):
    """512x512x16 thin film (A = 1.3e-11, alpha = 0.02, dt = 1e-13): one RK4 step."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.THIN_FILM
    n = cfg["n"]
    _say("llg 512x512x16 one step")
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=0)
    plan = pkg.demag_setup(n + cfg["cell"])
    try:
        m = torch.from_numpy(m0).cuda()
        pkg.llg_step(plan, m, (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, (0, 0, 0)), cfg["dt"], 1)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    prob = ollg.LLG(n, cfg["cell"], cfg["Ms"], cfg["A"], cfg["alpha"], workers=8)
    ref = prob.rk4_step(m0.astype(np.float64), cfg["dt"])
    # compare the change of m (the step itself), the stricter measure
    d_got, d_ref = got - m0, ref - m0
    err = odemag.rel_l2(d_got, d_ref)
    _say("  rel-L2 of the step increment", err, " of m", odemag.rel_l2(got, ref))
    assert odemag.rel_l2(got, ref) <= TOL
    assert err <= 1e-3


# ------------------------------------------------------------------ H_d extrapolation
def _extrap_run(pkg, torch, n, flags, m0, params, dt, chunks):
    plan = pkg.demag_setup(n + W.CELL_4NM, flags)
    try:
        m = torch.from_numpy(m0).cuda()
        for k in chunks:   # several llg_step calls: the history persists between them
            pkg.llg_step(plan, m, params, dt, k)
        torch.cuda.synchronize()
        return m.cpu().numpy()
    finally:
        pkg.demag_destroy(plan)


@pytest.mark.parametrize("n,flags,chunks", [((64, 32, 4), 8, (3, 9)), ((16, 16, 8), 8, (10,)),
                                            ((128, 64, 2), 8, (5, 1, 4)), ((32, 32, 4), 8 | 2, (9,))],
                         ids=["64x32x4", "16x16x8-fivepass", "128x64x2", "32x32x4-bf16x3"])
def test_llg_extrapolated_matches_oracle(gpu_lib, torch_dev, n, flags, chunks):
    """One H_d per RK4 step, quartic extrapolation at the sub-steps after five steps."""
    import paper_2308_08447_amd as pkg
    _say("extrapolated llg parity", n, flags, chunks)
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=31)
    alpha, dt, Hz = 0.02, 1e-13, (1e4, -2e4, 3e4)
    params = (W.MS, W.A_EX, alpha, ollg.GAMMA, Hz)
    got = _extrap_run(pkg, torch_dev, n, flags, m0, params, dt, chunks).astype(np.float64)
    prob = ollg.LLGExtrapolated(n, W.CELL_4NM, W.MS, W.A_EX, alpha, Hzee=Hz)
    ref = prob.run(m0.astype(np.float64), dt, sum(chunks))
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of m", err, " of the increment", odemag.rel_l2(got - m0, ref - m0))
    assert err <= TOL
    assert odemag.rel_l2(got - m0, ref - m0) <= 1e-3


def test_llg_reset_and_step_change(gpu_lib, torch_dev):
    """llg_reset starts a new trajectory (same bits as a fresh plan); a new dt
    restarts the history like the oracle does."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n = (64, 32, 4)
    params = (W.MS, W.A_EX, 0.05, ollg.GAMMA, (0.0, 0.0, 2e4))
    mA = W.unit_vectors((4, 32, 64), seed=41)
    mB = W.unit_vectors((4, 32, 64), seed=42)
    plan = pkg.demag_setup(n + W.CELL_4NM, pkg.DEMAG_EXTRAPOLATE_HD)
    try:
        m = torch.from_numpy(mA).cuda()
        pkg.llg_step(plan, m, params, 1e-13, 7)
        pkg.llg_reset(plan)
        m = torch.from_numpy(mB).cuda()
        pkg.llg_step(plan, m, params, 1e-13, 8)
        torch.cuda.synchronize()
        after_reset = m.cpu().numpy()
    finally:
        pkg.demag_destroy(plan)
    fresh = _extrap_run(pkg, torch, n, pkg.DEMAG_EXTRAPOLATE_HD, mB, params, 1e-13, (8,))
    assert np.array_equal(after_reset, fresh)
    # dt change: 6 steps of 1e-13 then 7 of 5e-14
    plan = pkg.demag_setup(n + W.CELL_4NM, pkg.DEMAG_EXTRAPOLATE_HD)
    try:
        m = torch.from_numpy(mA).cuda()
        pkg.llg_step(plan, m, params, 1e-13, 6)
        pkg.llg_step(plan, m, params, 5e-14, 7)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    prob = ollg.LLGExtrapolated(n, W.CELL_4NM, W.MS, W.A_EX, 0.05, Hzee=(0.0, 0.0, 2e4))
    ref = prob.run(prob.run(mA.astype(np.float64), 1e-13, 6), 5e-14, 7)
    assert odemag.rel_l2(got, ref) <= TOL


def test_llg_extrapolated_thin_film(gpu_lib, torch_dev):
    """512x512x16 thin film (A = 1.3e-11, alpha = 0.02, dt = 1e-13): 7 steps, the
    last two with extrapolated sub-step fields."""
    import paper_2308_08447_amd as pkg
    cfg = W.THIN_FILM
    n = cfg["n"]
    _say("extrapolated llg 512x512x16, 7 steps")
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=0)
    params = (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, (0, 0, 0))
    got = _extrap_run(pkg, torch_dev, n, pkg.DEMAG_EXTRAPOLATE_HD, m0, params, cfg["dt"], (7,))
    prob = ollg.LLGExtrapolated(n, cfg["cell"], cfg["Ms"], cfg["A"], cfg["alpha"], workers=8)
    ref = prob.run(m0.astype(np.float64), cfg["dt"], 7)
    d_err = odemag.rel_l2(got.astype(np.float64) - m0, ref - m0)
    _say("  rel-L2 of m", odemag.rel_l2(got.astype(np.float64), ref), " of the increment", d_err)
    assert odemag.rel_l2(got.astype(np.float64), ref) <= TOL
    assert d_err <= 1e-3


# ------------------------------------------------------------------ point-dipole kernel (Eq. 8)
@pytest.mark.parametrize("n,cell", [((8, 8, 8), (4e-10, 4e-10, 4e-10)), ((32, 32, 4), (4e-10, 4e-10, 4e-10)),
                                    ((64, 16, 2), (3e-10, 4e-10, 5e-10)), ((16, 16, 1), (4e-10, 4e-10, 4e-10)),
                                    ((128, 64, 8), (4e-10, 4e-10, 4e-10))],
                         ids=["8x8x8", "32x32x4", "64x16x2-noncubic", "16x16x1", "128x64x8"])
def test_point_dipole_field_matches_oracle(gpu_lib, torch_dev, n, cell):
    """demag_field with the point-dipole kernel of Eq. (8) (lattice dipole-dipole field)."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("point-dipole parity", n, cell)
    M = W.magnetisation(n, seed=sum(n) + 3)
    plan = pkg.demag_setup(n + cell, pkg.DEMAG_POINT_DIPOLE)
    try:
        Md = torch.from_numpy(M).cuda()
        Hd = torch.empty_like(Md)
        pkg.demag_field(plan, Md, Hd)
        torch.cuda.synchronize()
        H = Hd.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    Href = odemag.demag_fft(M.astype(np.float64), cell, kind="dipole")
    errs = odemag.rel_l2_per_field(H, Href)
    _say("  rel-L2 per field", errs)
    assert max(errs) <= TOL, errs
    if np.prod(n) <= 512:
        assert max(odemag.rel_l2_per_field(H, odemag.demag_direct(M.astype(np.float64), cell,
                                                                  kind="dipole"))) <= TOL


def test_atomistic_full_dipole_dipole(gpu_lib, torch_dev):
    """Atom plan with macro = 1 and the point-dipole kernel: every spin interacts
    with every other through Eq. (8) (no macrocells), two Heun steps."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n, steps = (32, 16, 8), 2
    cfg = W.ATOMISTIC
    S0 = W.unit_vectors((n[2], n[1], n[0]), seed=23)
    hz = (0.0, 0.0, 5e5)
    plan = pkg.atom_setup(n + (cfg["a"], 1), pkg.DEMAG_POINT_DIPOLE)
    try:
        S = torch.from_numpy(S0).cuda()
        pkg.atom_step(plan, S, (cfg["J"], cfg["mu_s"], cfg["alpha"], ollg.GAMMA, hz), cfg["dt"], steps)
        torch.cuda.synchronize()
        got = S.cpu().numpy().astype(np.float64)
    finally:
        pkg.atom_destroy(plan)
    prob = oatom.Atomistic(n, cfg["a"], 1, cfg["J"], cfg["mu_s"], cfg["alpha"], Hzee=hz, kind="dipole")
    ref = prob.run(S0.astype(np.float64), cfg["dt"], steps)
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of S", err, " increment", odemag.rel_l2(got - S0, ref - S0))
    assert err <= TOL
    assert odemag.rel_l2(got - S0, ref - S0) <= 1e-3


# ------------------------------------------------------------------ atomistic
@pytest.mark.parametrize("n,macro,steps", [((16, 16, 8), 4, 1), ((16, 16, 8), 4, 5), ((8, 8, 8), 2, 3),
                                           ((4, 4, 4), 4, 2), ((96, 24, 12), 3, 2), ((12, 6, 6), 3, 2),
                                           ((256, 8, 4), 4, 1)])
def test_atomistic_matches_oracle(gpu_lib, torch_dev, n, macro, steps):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("atom_step parity", n, macro, steps)
    cfg = W.ATOMISTIC
    nx, ny, nz = n
    S0 = W.unit_vectors((nz, ny, nx), seed=21)
    hz = (0.0, 0.0, 5e5)
    plan = pkg.atom_setup((nx, ny, nz, cfg["a"], macro))
    try:
        S = torch.from_numpy(S0).cuda()
        pkg.atom_step(plan, S, (cfg["J"], cfg["mu_s"], cfg["alpha"], ollg.GAMMA, hz), cfg["dt"], steps)
        torch.cuda.synchronize()
        got = S.cpu().numpy().astype(np.float64)
    finally:
        pkg.atom_destroy(plan)
    prob = oatom.Atomistic(n, cfg["a"], macro, cfg["J"], cfg["mu_s"], cfg["alpha"], Hzee=hz)
    ref = prob.run(S0.astype(np.float64), cfg["dt"], steps)
    err = odemag.rel_l2(got, ref)
    _say("  rel-L2 of S", err, " increment", odemag.rel_l2(got - S0, ref - S0))
    assert err <= TOL


@pytest.mark.parametrize("n", [(64, 32, 4), (480, 240, 2), (512, 512, 16)],
                         ids=lambda n: "x".join(map(str, n)))
def test_llg_graph_replay_is_bitwise_eager(gpu_lib, torch_dev, n):
    """llg_step with nsteps >= 2 replays a captured step: bitwise the result of
    single eager steps, also after the parameters, the field array and the
    chunk count change (each forces a new capture)."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("llg graph replay", n)
    m0 = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed=23)).cuda()
    cell = (5e-9,) * 3
    p1 = (W.MS, W.A_EX, 0.02, ollg.GAMMA, (1e4, -2e4, 3e4))
    p2 = (W.MS, W.A_EX, 0.3, ollg.GAMMA, (-2e4, 1e3, 0.0))
    plan = pkg.demag_setup(n + cell)
    try:
        eager, graph = m0.clone(), m0.clone()
        other = m0.clone()
        for prm, k in ((p1, 4), (p2, 3), (p1, 2)):
            for _ in range(k):
                pkg.llg_step(plan, eager, prm, 1e-13, 1)
            pkg.llg_step(plan, graph, prm, 1e-13, k)
            pkg.llg_step(plan, other, prm, 1e-13, k)    # another array: new capture
        torch.cuda.synchronize()
        assert torch.equal(eager, graph)
        assert torch.equal(eager, other)
        if n[1] > 1:
            pkg.demag_set_chunks(plan, min(3, pkg.kernel_shape(n)[2]))
            a, b = eager.clone(), eager.clone()
            for _ in range(2):
                pkg.llg_step(plan, a, p2, 2e-13, 1)
            pkg.llg_step(plan, b, p2, 2e-13, 2)
            torch.cuda.synchronize()
            assert torch.equal(a, b)
    finally:
        pkg.demag_destroy(plan)


def test_llg_trajectory_50_steps_sub_problem(gpu_lib, torch_dev):
    """50 RK4 steps of a 128x128x16 film (4 nm, alpha = 0.02, no Zeeman field)
    from random M: the mean relative error of <m>(t) between the GPU and the
    FP64 oracle stays below the 1e-4 single-precision floor, and the energy
    of both trajectories (evaluated by the oracle) never increases."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n, steps, every = (128, 128, 16), 50, 5
    cfg = W.THIN_FILM
    _say("llg trajectory", n, steps)
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=0)
    prm = (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, (0.0, 0.0, 0.0))
    prob = ollg.LLG(n, cfg["cell"], cfg["Ms"], cfg["A"], cfg["alpha"], workers=8)
    plan = pkg.demag_setup(n + cfg["cell"])
    try:
        m = torch.from_numpy(m0).cuda()
        ref = m0.astype(np.float64)
        eps, e_gpu, e_ref = [], [prob.energy(ref)], [prob.energy(ref)]
        for k in range(steps // every):
            pkg.llg_step(plan, m, prm, cfg["dt"], every)
            ref = prob.run(ref, cfg["dt"], every)
            got = m.cpu().numpy().astype(np.float64)
            a, b = got.reshape(3, -1).mean(axis=1), ref.reshape(3, -1).mean(axis=1)
            eps.append(float(np.linalg.norm(a - b)))
            e_gpu.append(prob.energy(got))
            e_ref.append(prob.energy(ref))
    finally:
        pkg.demag_destroy(plan)
    _say("  |<m> - <m_ref>| every 5 steps", ["%.2e" % v for v in eps])
    _say("  rel-L2 of m after 50 steps", odemag.rel_l2(got, ref))
    assert np.mean(eps) < 1e-4
    assert all(b <= a for a, b in zip(e_gpu, e_gpu[1:]))
    assert all(b <= a for a, b in zip(e_ref, e_ref[1:]))


def test_thin_film_1000_steps_energy_and_extrapolation(gpu_lib, torch_dev):
    """The thin-film workload over its 1000 RK4 steps (512x512x16, alpha = 0.02,
    no Zeeman field, random start), plain and with the extrapolated H_d (one
    evaluation per step).  Energies are evaluated by the oracle every 100 steps.
    * Both energy curves never increase, and they agree within 1%.
    * The two trajectories agree closely while the relaxation is predictable
      (|<m> - <m_extrap>| < 1e-6 after 100 steps, < 1e-5 after 200).  From a
      random start any small difference then grows exponentially, so the later
      divergence is reported, not bounded."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.THIN_FILM
    n, cell, every, steps = cfg["n"], cfg["cell"], 100, cfg["steps"]
    _say("thin film 1000 steps: energy and extrapolated-H_d trajectory")
    prm = (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, (0.0, 0.0, 0.0))
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=0)
    prob = ollg.LLG(n, cell, cfg["Ms"], cfg["A"], cfg["alpha"], workers=8)
    plain = pkg.demag_setup(n + cell)
    extrap = pkg.demag_setup(n + cell, pkg.DEMAG_EXTRAPOLATE_HD)
    try:
        a = torch.from_numpy(m0).cuda()
        b = a.clone()
        e0 = prob.energy(m0.astype(np.float64))
        ea, eb, eps = [e0], [e0], []
        for k in range(steps // every):
            pkg.llg_step(plain, a, prm, cfg["dt"], every)
            pkg.llg_step(extrap, b, prm, cfg["dt"], every)
            torch.cuda.synchronize()
            ma = a.cpu().numpy().astype(np.float64)
            mb = b.cpu().numpy().astype(np.float64)
            ea.append(prob.energy(ma))
            eb.append(prob.energy(mb))
            eps.append(float(np.linalg.norm(ma.reshape(3, -1).mean(1) - mb.reshape(3, -1).mean(1))))
    finally:
        pkg.demag_destroy(plain)
        pkg.demag_destroy(extrap)
    _say("  energy (J) every 100 steps, plain   ", ["%.6e" % e for e in ea])
    _say("  energy (J) every 100 steps, extrap. ", ["%.6e" % e for e in eb])
    _say("  |<m> - <m_extrap>| every 100 steps", ["%.2e" % v for v in eps])
    for e in (ea, eb):
        assert all(e1 <= e0 for e0, e1 in zip(e, e[1:]))
    assert max(abs(x - y) / abs(x) for x, y in zip(ea, eb)) < 1e-2
    assert eps[0] < 1e-6 and eps[1] < 1e-5


@pytest.mark.parametrize("n,flags", [((512, 512, 16), 0), ((16, 8, 32), 0), ((64, 32, 8), 2),
                                     ((32, 16, 4), "pbc"), ((480, 240, 2), 0)],
                         ids=["thin", "five-pass", "bf16x3", "periodic", "mixed-radix"])
def test_inplace_field_equals_out_of_place(gpu_lib, torch_dev, n, flags):
    """With DEMAG_INPLACE, demag_field(M, M) leaves bitwise the field that
    demag_field(M, H) writes to a separate array."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    if flags == "pbc":
        flags = pkg.pbc_flags(x=True, y=True, images=2)
    M = torch.from_numpy(W.magnetisation(n, seed=41)).cuda()
    plan = pkg.demag_setup(tuple(n) + (5e-9,) * 3, flags | pkg.DEMAG_INPLACE)
    try:
        H = torch.empty_like(M)
        pkg.demag_field(plan, M, H)
        A = M.clone()
        pkg.demag_field(plan, A, A)
        torch.cuda.synchronize()
        assert torch.equal(A, H)
    finally:
        pkg.demag_destroy(plan)
