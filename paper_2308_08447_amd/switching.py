"""The switching problem of the precision study (Sec. II, Fig. 2) driven through
the C ABI: an S state prepared by a decreasing saturating field, then a
switching field, with the average magnetization recorded on the device, and
the mean relative error between two recorded trajectories.

Every step runs in the library (llg_step, demag_field_mean); this module only
sequences the calls and owns the device buffers.
"""

import math

GAMMA = 2.21276e5   # mu0 * gamma_e, m/(A s)


def _params(cfg, alpha, H):
    return (cfg["Ms"], cfg["A"], alpha, GAMMA, tuple(H))


def s_state(pkg, plan, m, cfg, stream=None):
    """Saturate along [1,1,1] and lower the field to zero in cfg["ramp_steps"]
    equal decrements of cfg["ramp_time"] each, then relax for cfg["relax_time"]
    at zero field (damping cfg["alpha_prep"], step cfg["dt_prep"]).  m (device
    [3][nz][ny][nx]) is overwritten with the result.  Returns the RK4 steps taken."""
    import torch
    dt = cfg["dt_prep"]
    u = 1.0 / math.sqrt(3.0)
    m.copy_(torch.full_like(m, u))
    steps = 0
    per = int(round(cfg["ramp_time"] / dt))
    for k in range(cfg["ramp_steps"]):
        h = cfg["H_sat"] * (1.0 - k / cfg["ramp_steps"]) * u
        pkg.llg_step(plan, m, _params(cfg, cfg["alpha_prep"], (h, h, h)), dt, per, stream)
        steps += per
    per = int(round(cfg["relax_time"] / dt))
    pkg.llg_step(plan, m, _params(cfg, cfg["alpha_prep"], (0.0, 0.0, 0.0)), dt, per, stream)
    return steps + per


def switch(pkg, plan, m, cfg, dt, stream=None):
    """Apply cfg["H_switch"] with damping cfg["alpha"] for cfg["t_switch"] at step
    dt, recording <m> every cfg["record_every"] (which dt must divide).  m is
    advanced in place.  Returns a device tensor [npoints + 1][3] of <m>, the
    first row at t = 0."""
    import torch
    every = int(round(cfg["record_every"] / dt))
    if abs(every * dt - cfg["record_every"]) > 1e-6 * cfg["record_every"]:
        raise ValueError("dt must divide the recording interval")
    npts = int(round(cfg["t_switch"] / cfg["record_every"]))
    rec = torch.empty((npts + 1, 3), dtype=torch.float32, device=m.device)
    prm = _params(cfg, cfg["alpha"], cfg["H_switch"])
    pkg.demag_field_mean(plan, m, rec[0], stream)
    for i in range(npts):
        pkg.llg_step(plan, m, prm, dt, every, stream)
        pkg.demag_field_mean(plan, m, rec[i + 1], stream)
    return rec


def epsilon(rec, ref):
    """Mean relative error of Sec. II: sum_i |M(t_i) - M~(t_i)| / (n Ms) over the
    n common recorded points, M = Ms <m> (host arrays [n][3] of <m>)."""
    n = min(len(rec), len(ref))
    tot = 0.0
    for i in range(n):
        tot += math.sqrt(sum((float(rec[i][c]) - float(ref[i][c])) ** 2 for c in range(3)))
    return tot / n
