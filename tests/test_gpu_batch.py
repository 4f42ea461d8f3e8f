"""Batched solves of uneven problems (different E and N) in shared graph
launches: each member equals its standalone solve bitwise (same tiles),
reaches the oracle solution, and the tuning cache round-trips."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import log, rel_l2
from paper_2503_02134_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [(2, 5, 4001), (3, 7, 4002), (2, 9, 4003), (4, 5, 4004), (3, 9, 4005)]


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


def _problems(mx, ctx):
    out = []
    for ne, N, seed in CASES:
        xi, _ = mx.mxsem_gll(N)
        bm = W.box_mesh(ne, N, xi)
        m = mx.Mesh(ctx, bm.E, N, bm.xyz, bm.glo, bm.bnd)
        f = W.random_smooth_rhs(bm, seed)
        b = m.mass_rhs(torch.as_tensor(f, device="cuda"))
        out.append((m, b))
    return out


@pytest.mark.parametrize("mode,extra", [("MODE_FP64", ""), ("MODE_MIXED_IR", ""),
                                        ("MODE_MIXED_IR", "dot2"),
                                        ("MODE_FP32_ALL", "pairwise")])
def test_batch_equals_standalone_bitwise(mx, ctx, mode, extra):
    """Also with Dot2 dots, and with FP32 sums in the pairwise order (every
    element a rank): the options travel per problem through the shared
    launches."""
    log(f"batch vs standalone, {mode} {extra}")
    probs = _problems(mx, ctx)
    md = getattr(mx, mode)
    kw = {"dot2": dict(dot=mx.DOT_DOT2),
          "pairwise": dict(gs_order=mx.GS_ORDER_PAIRWISE, pc=mx.PC_IDENTITY)}.get(extra, {})
    tol = 1e-7 if extra == "pairwise" else 1e-10
    alone = []
    for m, b in probs:
        x, st = m.solve(b, mode=md, tol=tol, max_iter=4000, **kw)
        alone.append((x.clone(), st))
    bt = mx.mxsem_batch_create(ctx.h, [m.h for m, _ in probs])
    try:
        xs = [torch.zeros_like(b) for _, b in probs]
        sts = mx.mxsem_batch_solve(bt, mx.solve_opts(mode=md, tol=tol, max_iter=4000, **kw),
                                   [b for _, b in probs], xs)
    finally:
        mx.mxsem_batch_destroy(bt)
    for (xa, sa), xb, sb in zip(alone, xs, sts):
        log(f"  alone it={sa.iterations} outer={sa.outer} | batch it={sb.iterations} "
            f"outer={sb.outer} res={sb.rel_res:.2e}")
        assert sb.reason == sa.reason
        assert extra == "pairwise" or sb.reason == mx.CONVERGED
        assert sb.iterations == sa.iterations and sb.outer == sa.outer
        assert torch.equal(xa, xb)


def test_batch_reaches_oracle(orc, mx, ctx):
    log("batch mixed refinement vs oracle")
    probs = _problems(mx, ctx)
    bt = mx.mxsem_batch_create(ctx.h, [m.h for m, _ in probs])
    xs = [torch.zeros_like(b) for _, b in probs]
    try:
        sts = mx.mxsem_batch_solve(bt, mx.solve_opts(mode=mx.MODE_MIXED_IR, tol=1e-10,
                                                     max_iter=4000), [b for _, b in probs], xs)
    finally:
        mx.mxsem_batch_destroy(bt)
    for (ne, N, seed), x, st in zip(CASES, xs, sts):
        xo, _ = orc.gll(N)
        bmo = W.box_mesh(ne, N, xo)
        om = orc.Mesh(bmo.E, N, bmo.xyz, bmo.glo, bmo.bnd)
        xstar, _ = om.pcg(om.rhs(W.random_smooth_rhs(bmo, seed)), tol=1e-13, maxit=5000)
        err = rel_l2(x.cpu().numpy(), xstar, om.c)
        log(f"  ne={ne} N={N}: it={st.iterations} outer={st.outer} err={err:.2e}")
        assert st.reason == mx.CONVERGED and err <= 1e-8


def test_tuning_cache_round_trip(mx, ctx, tmp_path):
    log("autotune cache")
    probs = _problems(mx, ctx)[:2]
    path = str(tmp_path / "tune.json")
    bt = mx.mxsem_batch_create(ctx.h, [m.h for m, _ in probs], tune_cache=path)
    mx.mxsem_batch_destroy(bt)
    kv = json.load(open(path))
    assert len(kv) == 2 and all(k.startswith("gfx950:N") for k in kv)
    for k, v in kv.items():
        # tile + 100 x thread mapping (2: two columns per thread, N = 5 and 9 only)
        N = int(k.split(":")[1][1:])
        e, c = v % 100, v // 100
        assert 1 <= e and ((e * (N + 1) ** 2 + 63) // 64) * 64 <= 256
        assert c in (0, 1, 2) and (c < 2 or N in (5, 9))
    # a second batch reads the file instead of tuning again
    mtime = os.path.getmtime(path)
    probs2 = _problems(mx, ctx)[:2]
    bt = mx.mxsem_batch_create(ctx.h, [m.h for m, _ in probs2], tune_cache=path)
    mx.mxsem_batch_destroy(bt)
    assert os.path.getmtime(path) == mtime


@pytest.mark.parametrize("N,prec", [(5, "F32"), (9, "F32"), (7, "F32"), (5, "F64")])
def test_autotune_picks_a_valid_tile_and_mapping(mx, ctx, N, prec):
    """The autotuner times every tile with each thread mapping the order has
    (two for N = 5 and 9 with FP32 vectors, one otherwise) and returns one
    that a mesh accepts."""
    epb, cols = mx.mxsem_autotune(ctx.h, N, 512, getattr(mx, prec))
    log(f"autotune N={N} {prec}: epb={epb} cols={cols}")
    assert 1 <= epb and ((epb * (N + 1) ** 2 + 63) // 64) * 64 <= 256
    assert cols in ((1, 2) if (N in (5, 9) and prec == "F32") else (0,))


def test_batch_rejects_bad_input(mx, ctx):
    probs = _problems(mx, ctx)[:1]
    with pytest.raises(mx.MxsemError):
        mx.mxsem_batch_create(ctx.h, [probs[0][0].h, probs[0][0].h])
