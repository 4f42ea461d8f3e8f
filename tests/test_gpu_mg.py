"""Two-level Schwarz / multigrid preconditioner through the C ABI vs the
FP64 oracle: the preconditioner applied alone, node by node, in FP64 and
FP32, with one and with several lattice levels; FP64 and mixed-refinement
solves with it against the oracle's solution; refusals.

Tolerances: FP64 apply <= 1e-12 max|z| (the same operations, in another
order: the oracle contracts x, y, z, the kernel z, y, x; the coarsest level
is a dense inverse on the GPU and a Cholesky solve in the oracle).  FP32
apply <= 5e-5 max|z|: each element solve is six FP32 contractions through
eigenvector matrices with entries up to about 1/sqrt(min B) and a division
by the eigenvalue sums, a few hundred roundings of 2^-24 on terms up to
the solution's size, while the coarse correction stays FP64."""
import numpy as np
import pytest
import torch

from gpu_common import log, rel_l2
from paper_2503_02134_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_2503_02134_amd import mxsem
    mxsem.lib()
    return mxsem


@pytest.fixture(scope="module")
def ctx(mx):
    c = mx.Context(0)
    yield c
    c.close()


def _pair(orc, mx, ctx, ne, N, seed=None, kseed=None, hh=0.0, rhs_seed=None):
    xg, _ = mx.mxsem_gll(N)
    xo, _ = orc.gll(N)
    bmg = W.box_mesh(ne, N, xg, seed=seed)
    bmo = W.box_mesh(ne, N, xo, seed=seed)
    kg = None if kseed is None else W.lognormal_k(bmg, kseed)
    ko = None if kseed is None else W.lognormal_k(bmo, kseed)
    views = mx.VIEW_F64 | mx.VIEW_F32 | mx.VIEW_BF16 | mx.VIEW_MG
    gm = mx.Mesh(ctx, bmg.E, N, bmg.xyz, bmg.glo, bmg.bnd, kcoef=kg, helm_h=hh, views=views)
    om = orc.Mesh(bmo.E, N, bmo.xyz, bmo.glo, bmo.bnd, kcoef=ko, helm_h=hh)
    omg = orc.MG(om, ne, bmo.xyz, ko)
    return bmg, gm, bmo, om, omg


CASES = [(4, 4, 3, None, 0.0), (4, 3, None, 5, 1.0), (16, 2, 2, None, 0.0), (6, 5, 1, 4, 0.5)]


@pytest.mark.parametrize("ne,N,seed,kseed,hh", CASES)
def test_apply_matches_oracle(orc, mx, ctx, ne, N, seed, kseed, hh):
    bmg, gm, bmo, om, omg = _pair(orc, mx, ctx, ne, N, seed, kseed, hh)
    log(f"multigrid apply {ne}^3 N={N}: {omg.nlev} lattice levels "
        f"{[omg.level_nu(l) for l in range(omg.nlev)]}")
    g = np.random.default_rng(ne + N).standard_normal(bmo.glo.max() + 1)
    r = om.mask_apply(g[bmo.glo.reshape(-1)])
    zo = omg.apply(r)
    z64 = gm.precond(torch.as_tensor(r, device="cuda"), pc=mx.PC_MG).cpu().numpy()
    z32 = gm.precond(torch.as_tensor(r, dtype=torch.float32, device="cuda"),
                     pc=mx.PC_MG).cpu().numpy().astype(np.float64)
    sc = np.abs(zo).max()
    e64, e32 = np.abs(z64 - zo).max() / sc, np.abs(z32 - zo).max() / sc
    log(f"  max|z - z_oracle| / max|z|: FP64 {e64:.1e}, FP32 {e32:.1e}")
    assert e64 <= 1e-12 and e32 <= 5e-5
    assert np.all(z64[om.mask.astype(bool)] == 0.0)


@pytest.mark.parametrize("ne,N,seed,kseed,hh", [(8, 4, 3, None, 0.0), (6, 5, 1, 4, 0.5)])
def test_solves_match_oracle(orc, mx, ctx, ne, N, seed, kseed, hh):
    bmg, gm, bmo, om, omg = _pair(orc, mx, ctx, ne, N, seed, kseed, hh)
    bo = om.rhs(W.random_smooth_rhs(bmo, 11))
    b = gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 11), device="cuda"))
    xs, _ = om.pcg(bo, tol=1e-13, maxit=20000)
    xo, so = om.pcg(bo, tol=1e-10, maxit=5000, mg=omg)
    _, sj = om.pcg(bo, tol=1e-10, maxit=5000)
    x64, s64 = gm.solve(b, mode=mx.MODE_FP64, pc=mx.PC_MG, tol=1e-10, max_iter=5000)
    xir, sir = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_MG, tol=1e-10, max_iter=5000)
    e64 = rel_l2(x64.cpu().numpy(), xs, om.c)
    eir = rel_l2(xir.cpu().numpy(), xs, om.c)
    log(f"  {ne}^3 N={N}: oracle multigrid PCG {so.iterations} it (Jacobi {sj.iterations}); "
        f"GPU FP64 {s64.iterations} it err {e64:.1e}; mixed refinement {sir.iterations}+"
        f"{sir.outer} it err {eir:.1e}")
    assert so.reason == orc.CONVERGED and s64.reason == mx.CONVERGED and sir.reason == mx.CONVERGED
    assert abs(s64.iterations - so.iterations) <= 2
    assert e64 <= 1e-9 and eir <= 1e-8 and sir.rel_res <= 1e-10
    assert s64.fallback_used == 0


def test_refusals(orc, mx, ctx):
    xg, _ = mx.mxsem_gll(3)
    bm = W.box_mesh(3, 3, xg)
    plain = mx.Mesh(ctx, bm.E, 3, bm.xyz, bm.glo, bm.bnd)
    b = plain.mass_rhs(torch.as_tensor(W.manufactured(bm)[0], device="cuda"))
    with pytest.raises(mx.MxsemError) as ei:
        plain.solve(b, pc=mx.PC_MG)
    assert ei.value.code == mx.EINVAL
    with pytest.raises(mx.MxsemError) as ei:
        plain.precond(b, pc=mx.PC_MG)
    assert ei.value.code == mx.EINVAL
    # not a box: elements out of lexicographic order
    perm = np.arange(bm.E)[::-1]
    n3 = 4 ** 3
    with pytest.raises(mx.MxsemError) as ei:
        mx.Mesh(ctx, bm.E, 3, bm.xyz.reshape(bm.E, -1)[perm], bm.glo.reshape(bm.E, n3)[perm],
                bm.bnd.reshape(bm.E, n3)[perm], views=mx.VIEW_F64 | mx.VIEW_MG)
    assert ei.value.code == mx.ENOTSUP
    # batches run Jacobi or identity only
    mgm = mx.Mesh(ctx, bm.E, 3, bm.xyz, bm.glo, bm.bnd, views=mx.VIEW_F64 | mx.VIEW_MG)
    bt = mx.mxsem_batch_create(ctx.h, [mgm.h])
    try:
        with pytest.raises(mx.MxsemError) as ei:
            mx.mxsem_batch_solve(bt, mx.solve_opts(pc=mx.PC_MG), [b], [torch.zeros_like(b)])
        assert ei.value.code == mx.ENOTSUP
    finally:
        mx.mxsem_batch_destroy(bt)
    plain.close()
    mgm.close()
