"""Shared helpers of the GPU parity tests: build matching oracle / library
contexts and feed both the same seeded inputs."""
import numpy as np
import torch

from oracle import ops
from oracle.grid import Grid
from oracle.krylov import Oracle
from paper_1905_11601_amd import inputs


def setup(n, kind, s, bc, Gr=1e6, Pr=0.71, prec=0):
    import paper_1905_11601_amd as fvk
    g = Grid(*n, kind=kind, s=s)
    orc = Oracle(g, ops.Params(Gr, Pr), bc)
    ctx = fvk.Ctx(*n, grid=kind, s=s, span_bc=bc, Gr=Gr, Pr=Pr, prec=prec)
    return g, orc, ctx


def coords(g):
    return (tuple(a.f for a in g.ax), tuple(a.c for a in g.ax), tuple(a.h for a in g.ax))


def base(g, bc, seed_u=1905, seed_t=1906):
    f, c, h = coords(g)
    return torch.as_tensor(inputs.synthetic_base(f, c, h, bc, seed_u=seed_u, seed_t=seed_t))


def krylov_input(g, orc, seed, project=True):
    x = torch.as_tensor(inputs.random_fields(g.n, seed))
    if project:
        x = orc.project(x)
    return x / torch.linalg.norm(x)


def dev(t):
    return t.to(torch.float64).contiguous().cuda()


def rel_err(a, b):
    a = a.detach().cpu().to(torch.float64).reshape(-1)
    b = b.detach().cpu().to(torch.float64).reshape(-1)
    return float((a - b).abs().max() / max(float(b.abs().max()), 1e-300))
