"""Why the linear shape's finite-difference gate is looser than the quadratic
one: the loss of a linear-shape rollout is smooth only while no particle's
shape window changes between the two perturbed runs.  The windows of the
linear shape change where a particle crosses a cell face (the node
weights) or the middle of a cell (the staggered components' weights).

In FP64, along one seeded unit direction in the momenta, the central
difference at eps from 1e-2 down to 1e-7 is compared with the adjoint's
directional derivative, and beside each eps the particles whose window
pattern (cell, and offset below or above 1/2 per axis, at every step) differs
between the +eps and -eps runs are counted.  Once that count reaches zero the
difference meets the 1e-4 gate; the error shrinks with the count."""
import numpy as np
import pytest
import torch

from test_gpu_adjoint import c5_like

pytestmark = pytest.mark.gpu


def patterns(roll, src, u0, steps):
    """Loss and the per-step window patterns of every particle (the rollout's
    fixed particle order) for initial momenta u0."""
    s = roll.sim
    zeros = [torch.zeros(s.ncells, dtype=roll.dtype, device=s.device) for _ in range(3)]
    E = [zeros[0], src.to(roll.dtype).contiguous(), zeros[2]]
    B = [torch.zeros_like(zeros[0]) for _ in range(3)]
    u = [u0[d][roll.perm].to(roll.dtype).contiguous() for d in range(3)]
    roll._set_state(roll.cell0, roll.off0, u, E, B)
    n = roll.npart
    pats = []
    for _ in range(steps):
        roll._step()
        cur = roll.h.current()
        half = (cur["off"][0][:n] >= 0.5).long() + 2 * (cur["off"][1][:n] >= 0.5).long()
        pats.append(cur["cell"][:n].long() * 4 + half)
    return roll._energy(), torch.stack(pats)


def test_fd_error_vanishes_with_the_window_changes():
    from paper_1503_02464_amd.autograd import Rollout, rollout_loss
    steps = 40
    w, g, sp, src = c5_like(64, 16, steps)
    roll = Rollout(2, g.n, g.dx, g.dt, g.order, "fp64", sp, steps, 20)
    s = torch.tensor(src, dtype=torch.float64, device="cuda", requires_grad=True)
    u0 = torch.tensor(sp["u"], dtype=torch.float64, device="cuda", requires_grad=True)
    L = rollout_loss(roll, s, u0)
    L.backward()
    v = np.random.default_rng(777).normal(size=sp["u"].shape)
    v /= np.linalg.norm(v)
    vt = torch.tensor(v, device="cuda")
    want = float((u0.grad * vt).sum().item())
    rows = []
    for eps in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        lp, pp = patterns(roll, s.detach(), u0.detach() + eps * vt, steps)
        lm, pm = patterns(roll, s.detach(), u0.detach() - eps * vt, steps)
        changed = int((pp != pm).any(dim=0).sum().item())
        fd = (lp - lm) / (2 * eps)
        rows.append((eps, changed, abs(fd - want) / abs(want)))
    roll.sim.close()
    print("eps, particles whose windows differ, |FD - adjoint| / |adjoint|:", rows)
    counts = [r[1] for r in rows]
    assert counts[0] > 0 and counts[-1] == 0, rows  # the sweep spans both regimes
    assert all(a >= b for a, b in zip(counts, counts[1:])), rows  # fewer changes as eps shrinks
    for eps, changed, err in rows:
        if changed == 0:
            assert err <= 1e-4, (eps, err)  # smooth: the 1e-4 finite-difference gate holds
    assert max(r[2] for r in rows if r[1] > 0) > max(r[2] for r in rows if r[1] == 0), rows
