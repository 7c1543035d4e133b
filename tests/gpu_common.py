"""Helpers shared by the GPU tests: device tensors from seeded inputs and
contexts of the HIP library.  Inputs come from ``synthetic``; expected values
come from ``oracle``; the HIP path is reached only through the C-ABI binding."""

import numpy as np


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    return t.cpu().numpy()


def make_ctx(U, mass, **kw):
    from paper_0707_0131_amd import binding as B
    lt, lz, ly, lx = U.shape[:4]
    p = B.eigcg_default_params(dims=(lx, ly, lz, lt), mass=mass, **kw)
    g = dev(U)
    ctx = B.eigcg_create(p, g)
    return ctx, g


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
