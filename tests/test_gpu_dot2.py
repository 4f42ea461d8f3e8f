"""Dot accumulation (FP64, FP32, compensated Dot2; Sec. 5.2.1) and the
gather-scatter summation order (one sum per node, or the pairwise exchange
between ranks; Sec. 4.2.1) on the GPU, through the C ABI, against the oracle.

Bars:
  gather-scatter, both orders, FP32 or FP64 sums   bitwise (same definition)
  Dot2 dot                                          |d - x'y| <= u|x'y| + gamma_n^2 |x|'|y|
  FP32 dot                                          |d - x'y| <= gamma_n |x|'|y|
  FP64-accumulated dot of FP32 inputs               |d - x'y| <= 1e-15 |x|'|y|
  solves                                            see each test
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

from gpu_common import log, make_pair, rel_l2
from test_oracle_dot2 import U32, _gamma, exact_dot, ill_conditioned

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


def _t(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("b", [6, 12, 18])
def test_dot_accumulations_against_exact(orc, mx, ctx, b):
    """Weighted dots of FP32 vectors on a 4^3-element N = 7 mesh (32,768
    entries: 16 workgroups of partials), data built so that the terms
    fl(a_i c_i) b_i cancel (condition up to about 1e11)."""
    log(f"dot accumulations b={b}")
    bmg, gm, bmo, om, _, _ = make_pair(orc, mx, ctx, 4, 7, 3)
    n = gm.nloc
    rng = np.random.default_rng(200 + b)
    x, y, ex = ill_conditioned(n, b, rng)
    mult = (1.0 / om.c).astype(np.float32)
    a = (x * mult).astype(np.float32)  # a_i c_i = x_i exactly (c = 1/m, m a power of two)
    assert np.array_equal((a * (1.0 / mult).astype(np.float32)).astype(np.float32), x)
    absdot = float(np.sum(np.abs(x.astype(np.float64) * y)))
    ta, tb = _t(a, torch.float32), _t(y, torch.float32)
    d64 = gm.dot(ta, tb, acc=mx.DOT_F64)
    d32 = gm.dot(ta, tb, acc=mx.DOT_F32)
    dd2 = gm.dot(ta, tb, acc=mx.DOT_DOT2)
    o2 = float(om.dot_c_f32(a, y, dot2=True))
    e64, e32, e2 = (abs(float(Fraction(d) - ex)) for d in (d64, d32, dd2))
    log(f"  exact={float(ex):.6e} cond={2 * absdot / abs(float(ex)):.2e} "
        f"err f64={e64:.2e} f32={e32:.2e} dot2={e2:.2e} oracle dot2 err="
        f"{abs(float(Fraction(o2) - ex)):.2e}")
    assert e64 <= 1e-15 * absdot
    assert e32 <= _gamma(n) * absdot
    assert np.float32(dd2) == dd2 and np.float32(d32) == d32  # FP32 results
    bound2 = U32 * abs(float(ex)) + _gamma(n) ** 2 * absdot
    assert e2 <= bound2
    assert abs(dd2 - o2) <= 2 * bound2


def test_dot_ex_rejects_fp64_with_fp32_accumulation(mx, ctx, orc):
    bmg, gm, _, _, _, _ = make_pair(orc, mx, ctx, 2, 3)
    v = torch.ones(gm.nloc, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    for acc in (mx.DOT_F32, mx.DOT_DOT2):
        with pytest.raises(mx.MxsemError) as ei:
            mx.mxsem_dot_ex(gm.h, mx.F64, acc, v, v, out)
        assert ei.value.code == mx.ENOTSUP


@pytest.mark.parametrize("acc", ["F32", "F64"])
@pytest.mark.parametrize("order", ["one", "pairwise", "pairwise_2x2x2", "pairwise_1x3x2"])
def test_gather_scatter_orders_bitwise(orc, mx, ctx, acc, order):
    """FP32 gather-scatter with FP32 or FP64 sums, in one order per node or
    in the pairwise order (every element its own rank, or blocks of
    elements), equals the oracle's bit for bit on a deformed 4^3-element
    N = 5 mesh (copy counts 1, 2, 4, 8; several tiles)."""
    log(f"gs order acc={acc} order={order}")
    bmg, gm, bmo, om, _, _ = make_pair(orc, mx, ctx, 4, 5, 4)
    from paper_2503_02134_amd import workloads as W
    erank = None
    if order.startswith("pairwise_"):
        erank = W.block_ranks(4, *(int(c) for c in order.split("_")[1].split("x")))
    gm.set_ranks(erank)
    rng = np.random.default_rng(21)
    v = (rng.standard_normal(gm.nloc) * 10.0 ** rng.integers(-5, 6, gm.nloc)).astype(np.float32)
    pw = order != "one"
    got = gm.gs(_t(v, torch.float32), acc=getattr(mx, acc), pairwise=pw).cpu().numpy()
    want = om.gs_f32(v, acc64=(acc == "F64"), pairwise=pw, erank=erank)
    np.testing.assert_array_equal(got, want)
    gm.set_ranks(None)


def test_gather_scatter_pairwise_needs_fp32(orc, mx, ctx):
    bmg, gm, _, _, _, _ = make_pair(orc, mx, ctx, 2, 3)
    v = torch.ones(gm.nloc, dtype=torch.float64, device="cuda")
    with pytest.raises(mx.MxsemError) as ei:
        gm.gs(v, acc=mx.F64, pairwise=True)
    assert ei.value.code == mx.ENOTSUP
    with pytest.raises(mx.MxsemError) as ei:
        gm.set_ranks(np.full(gm.E, -1, np.int32))
    assert ei.value.code == mx.EINVAL


def test_solve_option_checks(orc, mx, ctx):
    """Dot modes and the per-copy order exist for PCG with FP32 vectors only."""
    bmg, gm, _, _, fg, _ = make_pair(orc, mx, ctx, 2, 3)
    b = gm.mass_rhs(_t(fg))
    bad = [dict(mode=mx.MODE_FP64, dot=mx.DOT_F32),
           dict(mode=mx.MODE_MIXED_IR_BF16G, dot=mx.DOT_DOT2),
           dict(mode=mx.MODE_MIXED, dot=mx.DOT_DOT2, method=mx.METHOD_FCG),
           dict(mode=mx.MODE_MIXED_IR, gs_order=mx.GS_ORDER_PAIRWISE),
           dict(mode=mx.MODE_FP64, gs_order=mx.GS_ORDER_PAIRWISE),
           dict(mode=mx.MODE_MIXED, dot=7),
           dict(mode=mx.MODE_MIXED, gs_order=2),
           dict(mode=mx.MODE_MIXED_IR_BF16P, dot=mx.DOT_DOT2),
           dict(mode=mx.MODE_MIXED_IR_BF16P, method=mx.METHOD_FCG),
           dict(mode=6)]
    for kw in bad:
        with pytest.raises(mx.MxsemError):
            gm.solve(b, tol=1e-8, max_iter=50, **kw)


@pytest.mark.parametrize("pc", ["PC_JACOBI", "PC_IDENTITY"])
def test_mixed_recipe_with_each_dot_and_order(orc, mx, ctx, pc):
    """The paper's mixed loop (FP32 body, FP64 gather-scatter sums) with FP64,
    FP32 and Dot2 dots and both gather-scatter orders, on the deformed 6^3
    N = 7 mesh: every variant drives the recursive residual to 1e-10 and
    stays as close to the FP64 solution as the FP64-dot recipe does (the
    FP32 operator's floor); Dot2 takes the FP64-dot iteration count within
    5%.  With FP64 sums the pairwise order changes nothing visible."""
    bmg, gm, bmo, om, fg, fo = make_pair(orc, mx, ctx, 6, 7, 2)
    xs, _ = om.pcg(om.rhs(fo), pc=getattr(orc, pc), tol=1e-13, maxit=8000)
    bg = gm.mass_rhs(_t(fg))
    its = {}
    for dot in ("DOT_F64", "DOT_F32", "DOT_DOT2"):
        for order in ("GS_ORDER_ONE", "GS_ORDER_PAIRWISE"):
            log(f"mixed {pc} {dot} {order}")
            x, st = gm.solve(bg, mode=mx.MODE_MIXED, pc=getattr(mx, pc), tol=1e-10,
                             max_iter=8000, dot=getattr(mx, dot), gs_order=getattr(mx, order))
            err = rel_l2(x.cpu().numpy(), xs, om.c)
            log(f"  it={st.iterations} reason={st.reason} rec={st.rel_res_recursive:.2e} "
                f"true={st.rel_res:.2e} err={err:.2e}")
            assert st.reason == mx.CONVERGED and st.rel_res_recursive <= 1e-10
            assert err < 1e-5
            its[dot, order] = st.iterations
    base = its["DOT_F64", "GS_ORDER_ONE"]
    assert abs(its["DOT_DOT2", "GS_ORDER_ONE"] - base) <= 0.05 * base
    assert abs(its["DOT_F64", "GS_ORDER_PAIRWISE"] - base) <= 0.05 * base


def test_fp32_sums_in_pairwise_order(orc, mx, ctx):
    """FP32 gather-scatter sums in the pairwise order: with one rank the solve
    is the one-order solve bit for bit; with two ranks (their partial sums
    associate differently from the one order, but a + b = b + a) every
    node's copies stay equal and the solve converges; with every element a
    rank of its own (FP32 and Dot2 dots) the solve runs to its end without
    breakdown and the copies of the iterate differ (what makes the
    multi-rank FP32 runs of the paper stagnate)."""
    from paper_2503_02134_amd import workloads as W
    bmg, gm, bmo, om, fg, fo = make_pair(orc, mx, ctx, 6, 7, 2)
    bg = gm.mass_rhs(_t(fg))
    kw = dict(mode=mx.MODE_FP32_ALL, pc=mx.PC_IDENTITY, tol=1e-9, max_iter=3000)
    x1, s1 = gm.solve(bg, **kw)
    gm.set_ranks(W.block_ranks(6, 1, 1, 1))
    x2, s2 = gm.solve(bg, gs_order=mx.GS_ORDER_PAIRWISE, **kw)
    log(f"fp32_all pairwise, one rank: it={s2.iterations} reason={s2.reason}")
    assert s2.iterations == s1.iterations and torch.equal(x1, x2)
    gm.set_ranks(W.block_ranks(6, 1, 1, 2))
    x2, s2 = gm.solve(bg, gs_order=mx.GS_ORDER_PAIRWISE, **kw)
    xv = x2.cpu().numpy()
    spread = np.max(np.abs(xv - om.gs(xv * om.c)))
    log(f"fp32_all pairwise, two ranks: it={s2.iterations} reason={s2.reason} spread={spread:.1e}")
    assert s2.reason == mx.CONVERGED and spread == 0.0
    gm.set_ranks(None)
    for dot in ("DOT_F32", "DOT_DOT2"):
        log(f"fp32_all pairwise, every element a rank, {dot}")
        x, st = gm.solve(bg, dot=getattr(mx, dot), gs_order=mx.GS_ORDER_PAIRWISE, **kw)
        log(f"  it={st.iterations} reason={st.reason} rec={st.rel_res_recursive:.2e} "
            f"true={st.rel_res:.2e}")
        assert st.reason in (mx.CONVERGED, mx.STAGNATED, mx.MAX_ITER)
        assert np.isfinite(st.rel_res) and st.rel_res < 1.0
        xv = x.cpu().numpy()
        spread = np.max(np.abs(xv - om.gs(xv * om.c)))  # 0 when all copies agree
        log(f"  largest difference between a copy and its node's mean: {spread:.2e}")
        assert spread > 0.0


def test_rank_count_dependent_stagnation(orc, mx, ctx):
    """The paper's rank-count result (Sec. 4.2.1, evaluation table) on one
    GPU: FP32 gather-scatter sums in the pairwise exchange's order converge
    with one and two ranks and stagnate with 2 x 2 x 2 ranks, while FP64 sums
    converge with 2 x 2 x 2 ranks (Jacobi CG, FP64 dots, recursive 1e-9, the
    deformed 8^3-element N = 7 mesh)."""
    from paper_2503_02134_amd import workloads as W
    bmg, gm, bmo, om, fg, fo = make_pair(orc, mx, ctx, 8, 7, 2, rhs="random", rhs_seed=20)
    bg = gm.mass_rhs(_t(fg))
    kw = dict(pc=mx.PC_JACOBI, tol=1e-9, max_iter=5000, dot=mx.DOT_F64,
              gs_order=mx.GS_ORDER_PAIRWISE)
    res = {}
    for layout in ((1, 1, 1), (1, 1, 2), (2, 2, 2)):
        gm.set_ranks(W.block_ranks(8, *layout))
        for gname, mode in (("fp32", mx.MODE_FP32_ALL), ("fp64", mx.MODE_MIXED)):
            _, st = gm.solve(bg, mode=mode, **kw)
            log(f"ranks {layout} gs {gname}: it={st.iterations} reason={st.reason} "
                f"rec={st.rel_res_recursive:.2e}")
            res[layout, gname] = st
    gm.set_ranks(None)
    for layout in ((1, 1, 1), (1, 1, 2)):
        assert res[layout, "fp32"].reason == mx.CONVERGED
    assert res[(2, 2, 2), "fp32"].reason == mx.STAGNATED
    assert res[(2, 2, 2), "fp32"].rel_res_recursive > 1e-8
    for layout in ((1, 1, 1), (1, 1, 2), (2, 2, 2)):
        assert res[layout, "fp64"].reason == mx.CONVERGED
        assert res[layout, "fp64"].iterations == res[(1, 1, 1), "fp64"].iterations
