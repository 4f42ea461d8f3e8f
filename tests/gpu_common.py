"""Helpers shared by the GPU parity tests: build the same seeded problem for
the HIP path (mesh from the library's own GLL nodes) and for the oracle
(mesh from the oracle's GLL nodes); the two share only the generator."""
from __future__ import annotations

import sys

import numpy as np

from paper_2503_02134_amd import workloads as W


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def make_pair(orc, mx, ctx, ne, N, seed=None, kseed=None, helm_h=0.0, rhs="manufactured",
              rhs_seed=0, views=None):
    """Returns (bm_gpu, gpu_mesh, bm_orc, orc_mesh, f_gpu(np), f_orc(np))."""
    xg, _ = mx.mxsem_gll(N)
    xo, _ = orc.gll(N)
    bmg = W.box_mesh(ne, N, xg, seed=seed)
    bmo = W.box_mesh(ne, N, xo, seed=seed)
    kg = ko = None
    if kseed is not None:
        kg = W.lognormal_k(bmg, kseed)
        ko = W.lognormal_k(bmo, kseed)
    kw = {} if views is None else {"views": views}
    gm = mx.Mesh(ctx, bmg.E, N, bmg.xyz, bmg.glo, bmg.bnd, kcoef=kg, helm_h=helm_h, **kw)
    om = orc.Mesh(bmo.E, N, bmo.xyz, bmo.glo, bmo.bnd, kcoef=ko, helm_h=helm_h)
    if rhs == "manufactured":
        fg, _ = W.manufactured(bmg)
        fo, _ = W.manufactured(bmo)
    else:
        fg = W.random_smooth_rhs(bmg, rhs_seed)
        fo = W.random_smooth_rhs(bmo, rhs_seed)
    return bmg, gm, bmo, om, fg, fo


def rel_l2(a, b, c=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if c is None:
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return float(np.sqrt(np.sum(c * (a - b) ** 2)) / max(np.sqrt(np.sum(c * b * b)), 1e-300))
