"""Full-size parity of the HIP path against the FP64 oracle, and the atomistic
Heun march across its z chunks.

* Atomistic lattices whose n_z crosses the 16-plane z chunks of the marching
  Heun stages (two and more chunk boundaries, a partial last chunk), and one
  Heun step of the full 1024x1024x256 lattice with 4^3 macrocells (Sec. IV,
  Eqs. 7, 9, 10), compared plane by plane on sampled z planes that include
  every chunk boundary, the lattice faces and macrocell boundaries.
* Ten RK4 steps of the 512x512x16 thin film (Eq. 5, Sec. III) against the
  oracle's ten steps.
* The 1024x1024x32 film and the 256x256x64 macrocell mesh with sparse sources:
  the exact direct sum of Eq. (1) at >= 256 targets that include all eight
  corners and points on all six faces (the truncated-store faces x = n_x - 1,
  y = n_y - 1, z = n_z - 1 among them), with a worst-element bound next to
  the relative L2 error.

Tolerance: relative L2 <= 2e-5 (the FP32 contract); the worst element is
bounded relative to the largest reference element, at the same 2e-5.
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
MZC = 16   # z planes per chunk of the marching Heun stages


@pytest.fixture(scope="module")
def torch_dev(gpu_lib):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------------ atomistic
@pytest.mark.parametrize("n,macro,steps", [((160, 20, 40), 5, 2), ((256, 32, 64), 4, 2),
                                           ((48, 12, 24), 3, 2)],
                         ids=["160x20x40-m5", "256x32x64-m4", "48x12x24-m3"])
def test_atomistic_across_z_chunks(gpu_lib, torch_dev, n, macro, steps):
    """n_z = 40 (chunks 16, 16, 8), 64 (four full chunks), 24 (16, 8): spins on
    both sides of every chunk boundary take their z neighbours from the other
    chunk; Zeeman field on, two Heun steps."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("atom_step across z chunks", n, macro, steps)
    assert n[2] > MZC
    cfg = W.ATOMISTIC
    nx, ny, nz = n
    S0 = W.unit_vectors((nz, ny, nx), seed=31)
    hz = (1e5, -2e5, 5e5)
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
    inc = odemag.rel_l2(got - S0, ref - S0)
    # the planes on both sides of each chunk boundary, on their own
    bnd = sorted({z for c in range(MZC, nz, MZC) for z in (c - 1, c)})
    err_b = odemag.rel_l2(got[:, bnd], ref[:, bnd])
    _say("  rel-L2 of S", err, " increment", inc, " boundary planes", bnd, err_b)
    assert err <= TOL
    assert err_b <= TOL
    assert inc <= 1e-4


class _SlabHeun:
    """One Heun step of the oracle's atomistic problem (oracle.atomistic), taken
    in z slabs so that the full lattice fits in host memory: the same field,
    right-hand side and step as Atomistic.heun_step, evaluated on a slab plus
    one halo plane on each side (the exchange of Eq. 7 reaches one plane)."""

    def __init__(self, prob, S0):
        self.p = prob
        self.S0 = S0                                  # (3, nz, ny, nx) float64
        self.nz = S0.shape[1]
        self.m = prob.macro

    def _field(self, S, Hm, z0, z1):
        """Total field on planes [z0, z1) from spins S and macrocell field Hm."""
        p = self.p
        lo, hi = max(z0 - 1, 0), min(z1 + 1, self.nz)
        ex = oatom.exchange_field(S[:, lo:hi], p.J, p.mu_s)[:, z0 - lo:z0 - lo + (z1 - z0)]
        m0 = z0 // self.m   # first macrocell plane the slab touches
        hd = oatom.broadcast_macro(Hm[:, m0:(z1 - 1) // self.m + 1], self.m)
        return ex + hd[:, z0 - m0 * self.m:z1 - m0 * self.m] + p.Hzee

    def _rhs(self, S, Hm, z0, z1):
        return ollg.llg_rhs(S[:, z0:z1], self._field(S, Hm, z0, z1), self.p.alpha, self.p.gamma)

    def step_planes(self, dt, planes, slab=16):
        p = self.p
        Hd0 = p.demag(oatom.macro_average(self.S0, self.m, p.a, p.mu_s))
        Sp = np.empty_like(self.S0)
        f0 = {}
        for z0 in range(0, self.nz, slab):
            z1 = min(z0 + slab, self.nz)
            f = self._rhs(self.S0, Hd0, z0, z1)
            Sp[:, z0:z1] = self.S0[:, z0:z1] + dt * f
            for z in planes:
                if z0 <= z < z1:
                    f0[z] = f[:, z - z0]
        Hd1 = p.demag(oatom.macro_average(Sp, self.m, p.a, p.mu_s))
        out = {}
        for z in planes:
            f1 = self._rhs(Sp, Hd1, z, z + 1)[:, 0]
            v = self.S0[:, z] + 0.5 * dt * (f0[z] + f1)
            out[z] = v / np.linalg.norm(v, axis=0, keepdims=True)
        return out


@pytest.mark.timeout(1200)
def test_atomistic_full_lattice_one_step(gpu_lib, torch_dev):
    """One Heun step of the 1024x1024x256 lattice (a = 0.4 nm, 4^3 macrocells,
    J = 1e-21 J, mu_s = 1 mu_B, alpha = 0.05, dt = 1e-15 s, T = 0) against the
    oracle on sampled whole z planes: the lattice faces, every plane on either
    side of a 16-plane chunk boundary of the first, middle and last chunks, and
    macrocell-boundary planes."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.ATOMISTIC
    n = cfg["n"]
    nx, ny, nz = n
    _say("atom_step full lattice", n)
    S0 = W.unit_vectors((nz, ny, nx), seed=0)
    prm = (cfg["J"], cfg["mu_s"], cfg["alpha"], ollg.GAMMA, (0.0, 0.0, 0.0))
    planes = [0, 1, 3, 4, 15, 16, 17, 31, 32, 127, 128, 129, 143, 144, 239, 240, 252, 254, 255]
    plan = pkg.atom_setup((nx, ny, nz, cfg["a"], cfg["macro"]))
    try:
        S = torch.from_numpy(S0).cuda()
        pkg.atom_step(plan, S, prm, cfg["dt"], 1)
        torch.cuda.synchronize()
        got = {z: S[:, z].cpu().numpy().astype(np.float64) for z in planes}
        del S
    finally:
        pkg.atom_destroy(plan)
    _say("  GPU step done; oracle step on the sampled planes")
    prob = oatom.Atomistic(n, cfg["a"], cfg["macro"], cfg["J"], cfg["mu_s"], cfg["alpha"], workers=16)
    S064 = S0.astype(np.float64)
    del S0
    ref = _SlabHeun(prob, S064).step_planes(cfg["dt"], planes)
    worst = 0.0
    worst_inc = 0.0
    for z in planes:
        e = odemag.rel_l2(got[z], ref[z])
        inc = odemag.rel_l2(got[z] - S064[:, z], ref[z] - S064[:, z])
        worst, worst_inc = max(worst, e), max(worst_inc, inc)
        _say(f"  plane {z}: rel-L2 of S {e:.3e}, of the increment {inc:.3e}")
    assert worst <= TOL
    assert worst_inc <= 1e-4


# ------------------------------------------------------------------ LLG
@pytest.mark.timeout(600)
def test_llg_thin_film_ten_steps(gpu_lib, torch_dev):
    """Ten RK4 steps of the 512x512x16 thin film (A = 1.3e-11 J/m, alpha = 0.02,
    dt = 1e-13 s, seeded random m): rel-L2 of m <= 2e-5; the increment's error
    is reported and bounded loosely (it grows with the relaxation's
    sensitivity to rounding)."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.THIN_FILM
    n, steps = cfg["n"], 10
    _say("llg 512x512x16 ten steps")
    m0 = W.unit_vectors((n[2], n[1], n[0]), seed=0)
    prm = (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, (0.0, 0.0, 0.0))
    plan = pkg.demag_setup(n + cfg["cell"])
    try:
        m = torch.from_numpy(m0).cuda()
        for _ in range(steps):
            pkg.llg_step(plan, m, prm, cfg["dt"], 1)
        torch.cuda.synchronize()
        got = m.cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    prob = ollg.LLG(n, cfg["cell"], cfg["Ms"], cfg["A"], cfg["alpha"], workers=16)
    ref = prob.run(m0.astype(np.float64), cfg["dt"], steps)
    err = odemag.rel_l2(got, ref)
    inc = odemag.rel_l2(got - m0, ref - m0)
    _say("  rel-L2 of m", err, " of the increment", inc)
    assert err <= TOL
    assert inc <= 1e-3


# ------------------------------------------------------------------ sparse sources, dense targets
def _targets(n, seed, per_face=48, interior=64):
    """The 8 corners, per_face random points on each of the 6 faces and
    `interior` random points, as rows (x, y, z)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    pts = [(x, y, z) for x in (0, nx - 1) for y in (0, ny - 1) for z in (0, nz - 1)]
    for axis, size in ((0, nx), (1, ny), (2, nz)):
        for v in (0, size - 1):
            for _ in range(per_face):
                p = [int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))]
                p[axis] = v
                pts.append(tuple(p))
    for _ in range(interior):
        pts.append((int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz))))
    return np.array(sorted(set(pts)))


def _direct_at(M, src, tg, cell):
    """H at the targets = -sum over the non-zero source cells of N(t - s) M_s
    (the direct sum of Eq. 1 restricted to the sources)."""
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
def test_full_size_dense_targets(gpu_lib, torch_dev, n, cell):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    _say("sparse sources, dense targets", n)
    M, src, _ = W.sparse_sources(n, 400, 1, seed=41)
    tg = _targets(n, seed=42)
    assert len(tg) >= 256
    plan = pkg.demag_setup(n + tuple(cell))
    try:
        Md = torch.from_numpy(M).cuda()
        Hd = torch.empty_like(Md)
        pkg.demag_field(plan, Md, Hd)
        torch.cuda.synchronize()
        t = torch.from_numpy(tg).cuda()
        got = Hd[:, t[:, 2], t[:, 1], t[:, 0]].cpu().numpy().astype(np.float64)
    finally:
        pkg.demag_destroy(plan)
    ref = _direct_at(M, src, tg, cell)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    worst = np.abs(got - ref).max() / np.abs(ref).max()
    faces = {}
    for axis, size, name in ((0, n[0], "x"), (1, n[1], "y"), (2, n[2], "z")):
        sel = tg[:, axis] == size - 1
        faces[name] = np.linalg.norm(got[:, sel] - ref[:, sel]) / np.linalg.norm(ref[:, sel])
    _say(f"  {len(tg)} targets: rel-L2 {err:.3e}, worst element / max |H| {worst:.3e}, "
         f"last faces {faces}")
    assert err <= TOL
    assert worst <= TOL
    assert max(faces.values()) <= TOL


def test_large_film_z_variants_bitwise(gpu_lib, torch_dev):
    """1024x1024x32: the z stage's variants are the register form with 32 and
    64 columns per block (0, 2) and the lean LDS form (1).  All three run the
    same per-column arithmetic, so the full field is bitwise the same for each
    (and for several chunk counts, and with per-stage timing events on); the
    default one is checked against the direct sum above."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    n = (1024, 1024, 32)
    _say("z variants bitwise", n)
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        M = torch.from_numpy(W.magnetisation(n, 5)).cuda()
        ref = torch.empty_like(M)
        pkg.demag_field(plan, M, ref)
        for v in range(pkg.NVARIANTS):
            for nch in (13, 20):
                pkg.demag_set_variant(plan, 2, v)
                pkg.demag_set_chunks(plan, nch)
                H = torch.empty_like(M)
                pkg.demag_field(plan, M, H)
                torch.cuda.synchronize()
                _say("  variant", v, "chunks", nch, "equal", bool(torch.equal(H, ref)))
                assert torch.equal(H, ref), (v, nch)
        # per-stage timing events around every launch leave the result alone
        pkg.demag_timing_enable(plan, 64)
        H = torch.empty_like(M)
        pkg.demag_field(plan, M, H)
        torch.cuda.synchronize()
        pkg.demag_timing_enable(plan, 0)
        assert torch.equal(H, ref)
    finally:
        pkg.demag_destroy(plan)


def test_large_film_llg_graph_replay_chunked(gpu_lib, torch_dev):
    """1024x1024x32 takes 13 or more chunks per H_d (39 or more y/z launches).
    llg_step with nsteps = 2 captures one RK4 step as a HIP graph and replays
    it: bitwise the result of two eager steps, after a chunk-count change too."""
    import paper_2308_08447_amd as pkg
    from oracle import llg as ollg
    torch = torch_dev
    n = (1024, 1024, 32)
    _say("llg graph replay, chunked", n)
    m0 = torch.from_numpy(W.unit_vectors((n[2], n[1], n[0]), seed=29)).cuda()
    prm = (W.MS, W.A_EX, 0.1, ollg.GAMMA, (1e4, 0.0, -1e4))
    plan = pkg.demag_setup(n + W.CELL_4NM)
    try:
        for nch in (pkg.demag_get_chunks(plan), 20):
            pkg.demag_set_chunks(plan, nch)
            eager, graph = m0.clone(), m0.clone()
            for _ in range(2):
                pkg.llg_step(plan, eager, prm, 1e-13, 1)
            pkg.llg_step(plan, graph, prm, 1e-13, 2)
            torch.cuda.synchronize()
            _say("  chunks", nch, "equal", bool(torch.equal(eager, graph)))
            assert torch.equal(eager, graph), nch
    finally:
        pkg.demag_destroy(plan)
