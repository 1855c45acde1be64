"""The torch-CPU FP64 reference (used for reference gradients) against the C
oracle, and its autograd gradient against its own finite differences."""
import numpy as np
import pytest
import torch

import oracle as O
import pins
from oracle import torch_ref as T
from paper_1503_02464_amd import inputs


def to_torch(g, sp, f):
    tg = T.Grid(g.dims, g.n, g.dx, g.dt, g.order)
    x = torch.tensor(sp["cell"] + sp["off"], dtype=T.TD)
    tsp = dict(q=sp["q"], m=sp["m"], x=x, u=torch.tensor(sp["u"]), w=torch.tensor(sp["w"]))
    return tg, tsp, torch.tensor(f["E"]), torch.tensor(f["B"])


@pytest.mark.parametrize("dims,order", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_torch_reference_matches_oracle(dims, order):
    g = pins.grid(dims, (7, 6, 5)[:dims], dx=(0.1, 0.12, 0.09), cfl=0.9, order=order)
    sp = inputs.random_particles(g.n, dims, 300, 0.5, (0.5, 1.5), seed=3)
    f = inputs.random_fields(g.ncells, 0.3, seed=4)
    osp = O.copy_species(sp)
    of = {k: v.copy() for k, v in f.items()}
    for _ in range(3):
        O.step(g, of, [osp])
    tg, tsp, E, B = to_torch(g, sp, f)
    sps = [tsp]
    for _ in range(3):
        E, B, J, sps = T.step(tg, E, B, sps)
    n = np.array(g.n)[:, None]
    dx = (sps[0]["x"].numpy() - (osp["cell"] + osp["off"]) + n / 2) % n - n / 2
    assert np.max(np.abs(dx[:dims])) < 1e-13
    rel = lambda a, b: np.max(np.abs(a - b)) / np.max(np.abs(b))
    assert rel(sps[0]["u"].numpy(), osp["u"]) < 1e-13
    assert rel(E.numpy(), of["E"]) < 1e-13 and rel(B.numpy(), of["B"]) < 1e-13 and rel(J.numpy(), of["J"]) < 1e-13


def test_torch_reference_gradient_matches_finite_differences():
    """Smooth case (quadratic shape, no node crossed in the short rollout is not
    required): d loss / d(source, u0) along random unit directions."""
    g = pins.grid(2, (8, 8), dx=0.05, cfl=0.7, order=2)
    sp = inputs.uniform_plasma(g.n, 2, 2, 0.05, 0.05 * 0.05 / 2, seed=5)
    tg = T.Grid(2, g.n, g.dx, g.dt, 2)
    x = torch.tensor(sp["cell"] + sp["off"], dtype=T.TD)
    src0 = torch.tensor(inputs.rng(6).normal(0, 0.01, g.ncells))
    u00 = torch.tensor(sp["u"])
    zeros = torch.zeros((3, g.ncells), dtype=T.TD)

    def loss(src, u0):
        E = zeros.clone()
        E = torch.stack([E[0], E[1] + src, E[2]])
        sps = [dict(q=-1.0, m=1.0, x=x, u=u0, w=torch.tensor(sp["w"]))]
        return T.rollout_loss(tg, E, zeros.clone(), sps, 6)

    src = src0.clone().requires_grad_(True)
    u0 = u00.clone().requires_grad_(True)
    L = loss(src, u0)
    L.backward()
    r = np.random.default_rng(7)
    for _ in range(3):
        vs = torch.tensor(r.normal(size=g.ncells))
        vu = torch.tensor(r.normal(size=u00.shape))
        nrm = torch.sqrt((vs * vs).sum() + (vu * vu).sum())
        vs, vu = vs / nrm, vu / nrm
        eps = 1e-5
        with torch.no_grad():
            fd = (loss(src0 + eps * vs, u00 + eps * vu) - loss(src0 - eps * vs, u00 - eps * vu)) / (2 * eps)
        gv = (src.grad * vs).sum() + (u0.grad * vu).sum()
        assert abs(float(gv - fd)) <= 1e-6 * abs(float(fd)), (float(gv), float(fd))
