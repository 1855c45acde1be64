"""The hand-written adjoint (reverse mode) of the HIP library: transpose
identity of the Yee part, gradients of K-step rollouts against the torch-CPU
FP64 autograd reference, and central finite differences of the GPU forward."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import grid, make_sim
from oracle import torch_ref as T
from paper_1503_02464_amd import inputs

pytestmark = pytest.mark.gpu


def dot(a, b):
    return float(sum(np.sum(np.asarray(x, np.float64) * np.asarray(y, np.float64)) for x, y in zip(a, b)))


@pytest.mark.parametrize("dims", [2, 3])
def test_yee_adjoint_is_transpose(dims):
    """<Y(E,B,J), (lE,lB)> = <(E,B), Y^T(lE,lB)> + <J, lJ> for the Yee step Y."""
    g = grid(dims, (12, 10, 8)[:dims], dx=0.1, cfl=0.8)
    r = inputs.rng(200 + dims)
    E, B, J = (r.normal(size=(3, g.ncells)) for _ in range(3))
    lE, lB = (r.normal(size=(3, g.ncells)) for _ in range(2))
    s = make_sim(g, "fp64", (2, 2, 2) if dims == 3 else (2, 2, 1), max_particles=1)
    s.set_fields(E, B, J)
    s.yee_step()
    f1 = s.get_fields()
    s.set_fields(lE, lB, np.zeros_like(J))
    s._call(s.lib.pic_yee_adjoint(s.ctx, __import__("ctypes").byref(s.fstruct), None), "pic_yee_adjoint")
    import torch as _t
    _t.cuda.synchronize()
    la = s.get_fields()
    lhs = dot([f1["E"], f1["B"]], [lE, lB])
    rhs = dot([E, B, J], [la["E"], la["B"], la["J"]])
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + abs(rhs)), (lhs, rhs)
    s.close()


def torch_rollout_grad(g, sp, src, steps):
    tg = T.Grid(g.dims, g.n, g.dx, g.dt, g.order)
    x = torch.tensor(sp["cell"] + sp["off"], dtype=T.TD)
    s = torch.tensor(src, dtype=T.TD, requires_grad=True)
    u0 = torch.tensor(sp["u"], dtype=T.TD, requires_grad=True)
    zeros = torch.zeros((3, g.ncells), dtype=T.TD)
    E = torch.stack([zeros[0], zeros[1] + s, zeros[2]])
    L = T.rollout_loss(tg, E, zeros.clone(), [dict(q=sp["q"], m=sp["m"], x=x, u=u0, w=torch.tensor(sp["w"]))],
                       steps)
    L.backward()
    return float(L), s.grad.numpy(), u0.grad.numpy()


def gpu_rollout(g, sp, src, steps, every, prec="fp64"):
    from paper_1503_02464_amd.autograd import Rollout, rollout_loss
    roll = Rollout(g.dims, g.n, g.dx, g.dt, g.order, prec, sp, steps, every)
    s = torch.tensor(src, dtype=torch.float64, device="cuda", requires_grad=True)
    u0 = torch.tensor(sp["u"], dtype=torch.float64, device="cuda", requires_grad=True)
    L = rollout_loss(roll, s, u0)
    L.backward()
    return roll, float(L), s.grad.cpu().numpy(), u0.grad.cpu().numpy()


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


CASES = [(2, 1, (12, 10)), (2, 2, (12, 10)), (3, 1, (8, 6, 6)), (3, 2, (8, 6, 6))]


@pytest.mark.parametrize("dims,order,n", CASES, ids=[f"{d}d-m{m}" for d, m, _ in CASES])
def test_rollout_gradient_matches_torch_reference(dims, order, n):
    g = grid(dims, n, dx=0.05, cfl=0.7, order=order)
    dV = 0.05 ** dims
    sp = inputs.uniform_plasma(g.n, dims, 3, 0.05, dV / 3, seed=210 + dims)
    src = inputs.rng(211).normal(0, 0.01, g.ncells)
    steps = 7
    Lr, gs_r, gu_r = torch_rollout_grad(g, sp, src, steps)
    roll, Lg, gs, gu = gpu_rollout(g, sp, src, steps, every=3)
    assert abs(Lg - Lr) <= 1e-12 * Lr
    assert rel(gs, gs_r) < 1e-9, rel(gs, gs_r)
    assert rel(gu, gu_r) < 1e-9, rel(gu, gu_r)
    roll.sim.close()


def directional_fd(roll, src, u0, vs, vu, eps):
    s = torch.tensor(src, dtype=torch.float64, device="cuda")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda")
    vs_t = torch.tensor(vs, dtype=torch.float64, device="cuda")
    vu_t = torch.tensor(vu, dtype=torch.float64, device="cuda")
    lp = roll.forward(s + eps * vs_t, u + eps * vu_t)
    lm = roll.forward(s - eps * vs_t, u - eps * vu_t)
    return (lp - lm) / (2 * eps)


def c5_like(n, ppc, steps):
    from paper_1503_02464_amd.configs import diff_2d
    w = diff_2d(n)
    w.ppc = ppc
    g = grid(2, w.n[:2], dx=w.dx[0], cfl=w.cfl, order=w.order)
    sp = inputs.uniform_plasma(w.n, 2, ppc, w.u_sigma, w.density * w.cell_volume / ppc, w.seed)
    src = inputs.rng(w.seed + 1).normal(0, w.extra["src_sigma"], g.ncells)
    return w, g, sp, src


# (shape order, step, bound).  The quadratic shape makes the loss smooth
# enough for the 1e-4 gate at a step of 1e-3.  With the linear shape the loss
# is only piecewise smooth (particles cross the shape's kinks during the
# rollout), so a central difference straddles kinks and differs from the
# one-sided derivative by an amount that shrinks with the step; there the
# exact gate is the comparison with autograd above and these bounds only
# check the trend.
FD_CASES = [(2, 1e-3, 1e-4), (1, 1e-3, 1e-1), (1, 1e-5, 1e-2)]


@pytest.mark.parametrize("order,eps,bound", FD_CASES, ids=[f"m{o}-eps{e:g}" for o, e, _ in FD_CASES])
def test_rollout_gradient_matches_finite_differences_c5_shape(order, eps, bound):
    """The differentiable 2D workload's shape (16 ppc, 0.7 CFL) on a 64x64 box
    for 60 steps, checkpoints every 20: directional central differences along
    unit random directions over both parameter groups against the adjoint."""
    w, g, sp, src = c5_like(64, 16, 60)
    g = grid(2, w.n[:2], dx=w.dx[0], cfl=w.cfl, order=order)
    roll, L, gs, gu = gpu_rollout(g, sp, src, 60, 20)
    r = np.random.default_rng(220)
    errs = []
    for _ in range(4):
        vs = r.normal(size=gs.shape)
        vu = r.normal(size=gu.shape)
        nrm = math.sqrt(np.sum(vs * vs) + np.sum(vu * vu))
        vs, vu = vs / nrm, vu / nrm
        fd = directional_fd(roll, src, sp["u"], vs, vu, eps)
        gv = float(np.sum(gs * vs) + np.sum(gu * vu))
        errs.append(abs(gv - fd) / abs(fd))
    print("fd relative errors", order, eps, errs)
    assert max(errs) <= bound, errs
    roll.sim.close()


def test_per_entry_finite_differences_smooth_case():
    """Quadratic shape, 8x8 box, 2 ppc, 20 steps: individual gradient entries of
    both parameter groups against central differences of single entries."""
    g = grid(2, (8, 8), dx=0.05, cfl=0.7, order=2)
    sp = inputs.uniform_plasma(g.n, 2, 2, 0.02, 0.05 * 0.05 / 2, seed=240)
    src = inputs.rng(241).normal(0, 0.01, g.ncells)
    roll, L, gs, gu = gpu_rollout(g, sp, src, 20, 20)
    r = np.random.default_rng(242)
    eps = 1e-6
    for idx in r.choice(g.ncells, 12, replace=False):
        e = np.zeros_like(src)
        e[idx] = 1.0
        fd = directional_fd(roll, src, sp["u"], e, np.zeros_like(sp["u"]), eps)
        assert abs(gs[idx] - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.max(np.abs(gs))), (idx, gs[idx], fd)
    flat = r.choice(gu.size, 12, replace=False)
    for f in flat:
        e = np.zeros(gu.size)
        e[f] = 1.0
        fd = directional_fd(roll, src, sp["u"], np.zeros_like(src), e.reshape(gu.shape), eps)
        gv = gu.reshape(-1)[f]
        assert abs(gv - fd) <= 1e-4 * max(abs(fd), 1e-3 * np.max(np.abs(gu))), (f, gv, fd)
    roll.sim.close()


def test_checkpoint_interval_does_not_change_the_gradient():
    g = grid(2, (16, 16), dx=0.05, cfl=0.7, order=1)
    sp = inputs.uniform_plasma(g.n, 2, 4, 0.02, 0.05 * 0.05 / 4, seed=230)
    src = inputs.rng(231).normal(0, 0.01, g.ncells)
    r1, _, gs1, gu1 = gpu_rollout(g, sp, src, 12, 1)
    r2, _, gs2, gu2 = gpu_rollout(g, sp, src, 12, 12)
    r3, _, gs3, gu3 = gpu_rollout(g, sp, src, 12, 5)
    for a, b in ((gs1, gs2), (gs1, gs3), (gu1, gu2), (gu1, gu3)):
        assert rel(a, b) < 1e-12
    for r_ in (r1, r2, r3):
        r_.sim.close()


def test_fp32_rollout_gradient_against_fp64():
    """The FP32 state's gradient against the FP64 one on the same inputs, in
    L2 norm (per-particle entries can jump where FP32 rounding moves a
    particle across a kink of the linear shape): source gradient 1e-3, momentum
    gradient 1e-2, cosine of both above 0.9999."""
    w, g, sp, src = c5_like(64, 16, 40)
    sp32 = inputs.round_f32(sp)
    src32 = src.astype(np.float32).astype(np.float64)
    r64, L64, gs64, gu64 = gpu_rollout(g, sp32, src32, 40, 20, "fp64")
    r32, L32, gs32, gu32 = gpu_rollout(g, sp32, src32, 40, 20, "fp32")
    assert abs(L32 - L64) <= 1e-4 * L64

    def l2(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    def cos(a, b):
        return float(np.sum(a * b) / (np.linalg.norm(a) * np.linalg.norm(b)))

    print("fp32 gradient L2 errors", l2(gs32, gs64), l2(gu32, gu64))
    assert l2(gs32, gs64) < 1e-3 and l2(gu32, gu64) < 1e-2, (l2(gs32, gs64), l2(gu32, gu64))
    assert cos(gs32, gs64) > 0.9999 and cos(gu32, gu64) > 0.9999
    r64.sim.close()
    r32.sim.close()


@pytest.mark.parametrize("prec,steps", [("fp64", 24), ("fp32", 1)])
def test_rollout_forward_instance_matches_oracle(prec, steps):
    """The differentiable workload's own forward launch (2D, linear shape,
    16x16 tiles, slack 2, one sort and no re-sort, the fixed-geometry instance
    the rollout runs) against the FP64 oracle at 64^2 with 16 ppc and the E_y
    source in place: FP64 to 1e-12 after 24 steps, FP32 to its one-step
    tolerances from an FP32-exact state."""
    import oracle as O
    from gpu_helpers import compare_fields, compare_species, unique_weights
    from paper_1503_02464_amd.sim import Simulation
    w, g, sp, src = c5_like(64, 16, steps)
    sp = unique_weights(sp, 730, scale=w.density * w.cell_volume / 16)
    f = O.new_fields(g)
    f["E"][1] = src
    if prec == "fp32":
        sp = inputs.round_f32(sp)
        f = inputs.round_fields_f32(f)
    s = Simulation(2, g.n, g.dx, g.dt, 1, prec, tile=(16, 16), slack=2, sort_every=0,
                   max_particles=sp["w"].shape[0])
    s.set_fields(f["E"], f["B"])
    h = s.add_species(sp)
    ref = O.copy_species(sp)
    ref_f = {k: v.copy() for k, v in f.items()}
    for _ in range(steps):
        s.step(1)
        assert O.step(g, ref_f, [ref]) == 0
    s.check()
    compare_species(g, prec, s.get_species(h), ref, "rollout forward")
    compare_fields(prec, s.get_fields(), ref_f, what="rollout forward")
    s.close()
