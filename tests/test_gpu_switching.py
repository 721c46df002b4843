"""The switching problem of the precision study (Sec. II, Fig. 2) on the GPU:
480x240x2 cells of 5 nm, S state, then H = (-20, 1, 0) kA/m.

* The first steps of the switching trajectory against the FP64 oracle from the
  same S state (rel-L2 <= 2e-5).
* The whole 1 ns event: the S state points along +x, the field reverses it,
  and the mean relative error between the 400 fs and 100 fs trajectories stays
  below 1e-4, the single-precision floor the paper reports.
"""

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


@pytest.fixture(scope="module")
def s_state(torch_dev):
    """(plan, S state on the device); the plan lives for the module."""
    import paper_2308_08447_amd as pkg
    from paper_2308_08447_amd import switching as sw
    torch = torch_dev
    cfg = W.SWITCHING
    n = cfg["n"]
    _say("switching: preparing the S state")
    plan = pkg.demag_setup(n + cfg["cell"])
    m = torch.empty((3, n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    sw.s_state(pkg, plan, m, cfg)
    torch.cuda.synchronize()
    yield plan, m.clone()
    pkg.demag_destroy(plan)


def test_field_mean_is_exact_and_reproducible(torch_dev, s_state):
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    plan, _ = s_state
    n = W.SWITCHING["n"]
    v = torch.from_numpy(W.magnetisation(n, seed=6)).cuda()
    out = torch.empty((2, 3), dtype=torch.float32, device="cuda")
    pkg.demag_field_mean(plan, v, out[0])
    pkg.demag_field_mean(plan, v, out[1])
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = v.cpu().numpy().astype(np.float64).reshape(3, -1).mean(axis=1)
    assert np.array_equal(got[0], got[1])
    np.testing.assert_allclose(got[0], ref, rtol=0, atol=1e-6 * np.abs(v.cpu().numpy()).max())


def test_switching_start_matches_oracle(torch_dev, s_state):
    """Five RK4 steps of 400 fs under the switching field from the S state."""
    import paper_2308_08447_amd as pkg
    torch = torch_dev
    cfg = W.SWITCHING
    plan, s0 = s_state
    steps, dt = 5, 4e-13
    _say("switching: first steps vs the oracle", steps, dt)
    m = s0.clone()
    pkg.llg_step(plan, m, (cfg["Ms"], cfg["A"], cfg["alpha"], ollg.GAMMA, cfg["H_switch"]), dt, steps)
    torch.cuda.synchronize()
    got = m.cpu().numpy().astype(np.float64)
    start = s0.cpu().numpy().astype(np.float64)
    ref = ollg.LLG(cfg["n"], cfg["cell"], cfg["Ms"], cfg["A"], cfg["alpha"], Hzee=cfg["H_switch"],
                   workers=8).run(start, dt, steps)
    err = odemag.rel_l2(got - start, ref - start)
    _say("  rel-L2 of the increment", err, "of m", odemag.rel_l2(got, ref))
    assert odemag.rel_l2(got, ref) <= TOL
    assert err <= 1e-3


def test_switching_event_and_step_convergence(torch_dev, s_state):
    import paper_2308_08447_amd as pkg
    from paper_2308_08447_amd import switching as sw
    torch = torch_dev
    cfg = W.SWITCHING
    plan, s0 = s_state
    recs = {}
    for dt in (4e-13, 1e-13):
        _say("switching: 1 ns at", dt)
        m = s0.clone()
        recs[dt] = sw.switch(pkg, plan, m, cfg, dt).cpu().numpy().astype(np.float64)
    a, b = recs[4e-13], recs[1e-13]
    _say("  S state <m>", a[0], "final <m>", a[-1], b[-1])
    assert a[0, 0] > 0.5 and abs(a[0, 2]) < 0.05           # S state along +x, in plane
    assert a[-1, 0] < -0.5 and b[-1, 0] < -0.5             # switched
    eps = sw.epsilon(a, b)
    _say("  epsilon(400 fs vs 100 fs)", eps)
    assert eps < 1e-4
