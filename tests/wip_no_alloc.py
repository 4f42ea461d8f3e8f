"""The allocation-free dot (mxsem_dot_ex_noalloc) through the C ABI against
mxsem_dot_ex, which runs the same kernels with the mesh's own partial-sum
buffer: equal bit for bit, on two calls in a row (the second on a smaller
mesh, so it reads only partials its own first kernel wrote over the first
call's), in every accumulation the dot offers; meshes beyond the scratch
array's limit are refused."""
import numpy as np
import pytest
import torch

from gpu_common import log
from paper_2503_02134_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    from paper_2503_02134_amd import mxsem
    mxsem.lib()
    return mxsem


def _mesh(mx, ctx, ne, N, seed):
    xg, _ = mx.mxsem_gll(N)
    bm = W.box_mesh(ne, N, xg, seed=seed)
    return bm, mx.Mesh(ctx, bm.E, N, bm.xyz, bm.glo, bm.bnd)


CASES = [("F64", "DOT_F64"), ("F32", "DOT_F64"), ("F32", "DOT_F32"), ("F32", "DOT_DOT2"),
         ("F64", "DOT_DEFAULT")]


def test_noalloc_dot_equals_dot_ex(mx):
    ctx = mx.Context(0)
    try:
        big = _mesh(mx, ctx, 16, 7, 2)    # 2,097,152 entries: 1024 partials
        small = _mesh(mx, ctx, 3, 5, 4)   # 5,832 entries: 3 partials
        for io_name, acc_name in CASES:
            io, acc = getattr(mx, io_name), getattr(mx, acc_name)
            dt = torch.float64 if io == mx.F64 else torch.float32
            for (bm, gm), seed in ((big, 11), (small, 12)):
                g = torch.Generator().manual_seed(seed)
                a = torch.randn(gm.nloc, generator=g, dtype=torch.float64).to(dt).cuda()
                b = torch.randn(gm.nloc, generator=g, dtype=torch.float64).to(dt).cuda()
                ref = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
                got = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
                mx.mxsem_dot_ex(gm.h, io, acc, a, b, ref)
                mx.mxsem_dot_ex_noalloc(gm.h, io, acc, a, b, got)
                r, v = float(ref.item()), float(got.item())
                log(f"  {io_name} {acc_name} nloc={gm.nloc}: dot_ex {r!r} noalloc {v!r}")
                assert np.isfinite(r) and v == r
        # a second context on the same device uses the same array
        ctx2 = mx.Context(0)
        try:
            xg, _ = mx.mxsem_gll(3)
            bm = W.box_mesh(2, 3, xg)
            gm2 = mx.Mesh(ctx2, bm.E, 3, bm.xyz, bm.glo, bm.bnd)
            a = torch.ones(gm2.nloc, dtype=torch.float64, device="cuda")
            ref = torch.zeros(1, dtype=torch.float64, device="cuda")
            got = torch.zeros(1, dtype=torch.float64, device="cuda")
            mx.mxsem_dot_ex(gm2.h, mx.F64, mx.DOT_F64, a, a, ref)
            mx.mxsem_dot_ex_noalloc(gm2.h, mx.F64, mx.DOT_F64, a, a, got)
            # sum of c = 1/m over all copies = number of global nodes (7^3)
            assert float(got.item()) == float(ref.item()) == 343.0
        finally:
            ctx2.close()
    finally:
        ctx.close()


def test_noalloc_dot_refuses_meshes_beyond_its_scratch(mx):
    """The limit is 16,777,216 local entries (8192 partials of 2048);
    33^3 elements of order 7 hold 18,399,744: refused before any launch."""
    ctx = mx.Context(0)
    try:
        xg, _ = mx.mxsem_gll(7)
        bm = W.box_mesh(33, 7, xg)
        gm = mx.Mesh(ctx, bm.E, 7, bm.xyz, bm.glo, bm.bnd, views=mx.VIEW_F64)
        assert gm.nloc > mx.NOALLOC_MAX_ENTRIES
        a = torch.zeros(gm.nloc, dtype=torch.float64, device="cuda")
        out = torch.zeros(1, dtype=torch.float64, device="cuda")
        with pytest.raises(mx.MxsemError) as ei:
            mx.mxsem_dot_ex_noalloc(gm.h, mx.F64, mx.DOT_F64, a, a, out)
        assert ei.value.code == mx.EINVAL and "scratch" in str(ei.value)
        gm.close()
    finally:
        ctx.close()
