"""Helpers for the GPU parity tests: oracle + device mesh from one spec."""
import numpy as np

import oracle
from paper_2405_05640_amd import sem


def pair(spec, prepare=0):
    om = oracle.Mesh(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices, spec.periodic,
                     spec.dirichlet)
    gm = sem.Mesh.from_spec(spec, prepare=prepare)
    return om, gm


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
