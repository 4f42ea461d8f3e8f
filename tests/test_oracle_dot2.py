"""Pins of the oracle's FP32 reductions (the extended-precision study of
Sec. 5.2.1 and the gather-scatter summation orders of Sec. 4.2.1), no GPU.

Expected values come from exact rational arithmetic (fractions.Fraction),
from the published error bound of Dot2 (Ogita, Rump and Oishi 2005: the
result is as accurate as a dot computed in twice the working precision and
then rounded), and from brute force with numpy FP32 scalars on tiny inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2503_02134_amd import workloads as W

U32 = 2.0 ** -24  # FP32 unit roundoff


def _gamma(n, u=U32):
    return n * u / (1 - n * u)


def exact_dot(x, y) -> Fraction:
    return sum((Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)), Fraction(0))


def ill_conditioned(n, b, rng):
    """FP32 vectors whose dot product cancels: the first half has products
    of magnitude up to 2^(2b); each later pair is chosen to cancel the exact
    running sum down to a random term of decreasing size.  Returns x, y and
    the exact dot."""
    h = n // 2
    x = np.zeros(n, np.float32)
    y = np.zeros(n, np.float32)
    ex = rng.integers(0, b + 1, h)
    x[:h] = (rng.uniform(-1, 1, h) * 2.0 ** ex).astype(np.float32)
    y[:h] = (rng.uniform(-1, 1, h) * 2.0 ** rng.integers(0, b + 1, h)).astype(np.float32)
    s = exact_dot(x[:h], y[:h])
    for j in range(h, n):
        e = int(round(b * (n - 1 - j) / max(1, n - 1 - h)))
        x[j] = np.float32(rng.uniform(-1, 1) * 2.0 ** rng.integers(0, b + 1))
        target = rng.uniform(-1, 1) * 2.0 ** e
        y[j] = np.float32((target - float(s)) / float(x[j]))
        s += Fraction(float(x[j])) * Fraction(float(y[j]))
    return x, y, s


def _cond(x, y, exact):
    return 2 * float(np.sum(np.abs(x.astype(np.float64) * y.astype(np.float64)))) / abs(float(exact))


@pytest.mark.parametrize("b", [4, 8, 12, 16, 20, 24])
def test_dot2_within_published_bound(orc, b):
    """|Dot2 - x'y| <= u |x'y| + gamma_n^2 |x|'|y| (u = 2^-24) on dots whose
    condition number runs from about 1e2 to 1e15; the exact dot is rational
    arithmetic on the FP32 inputs."""
    rng = np.random.default_rng(100 + b)
    n = 200
    x, y, ex = ill_conditioned(n, b, rng)
    absdot = float(np.sum(np.abs(x.astype(np.float64) * y.astype(np.float64))))
    r = orc.dot2_f32(x, y)
    err = abs(Fraction(float(r)) - ex)
    assert float(err) <= U32 * abs(float(ex)) + _gamma(n) ** 2 * absdot


def test_dot2_compensates_where_fp32_fails(orc):
    """At condition numbers 1e5..1e7 Dot2 is within 2u of the exact value
    (its bound is dominated by u |x'y|), while the recursive FP32 dot of the
    same data is off by far more than u: a Dot2 without the product errors or
    without the TwoSum errors would fall back to the FP32 accuracy."""
    rng = np.random.default_rng(7)
    worst_fp32 = 0.0
    for _ in range(12):
        x, y, ex = ill_conditioned(300, 11, rng)
        c = _cond(x, y, ex)
        if not 1e5 <= c <= 1e8:
            continue
        rel2 = abs(float(Fraction(float(orc.dot2_f32(x, y))) - ex)) / abs(float(ex))
        rel1 = abs(float(Fraction(float(orc.dot_f32(x, y))) - ex)) / abs(float(ex))
        assert rel2 <= 2 * U32 + _gamma(300) ** 2 * c
        worst_fp32 = max(worst_fp32, rel1)
    assert worst_fp32 > 100 * U32


def test_dot2_exact_cases(orc):
    """Exactly representable sums come out exact: integer data, a single
    product (fl(x y)), and the textbook cancellation 1e8 + 1 - 1e8."""
    rng = np.random.default_rng(3)
    x = rng.integers(-1000, 1000, 500).astype(np.float32)
    y = rng.integers(-1000, 1000, 500).astype(np.float32)
    assert float(orc.dot2_f32(x, y)) == float(np.dot(x.astype(np.int64), y.astype(np.int64)))
    a, b = np.float32(1.1), np.float32(3.3)
    assert orc.dot2_f32([a], [b]) == np.float32(a * b)
    assert orc.dot2_f32([1e8, 1.0, -1e8], [1.0, 1.0, 1.0]) == np.float32(1.0)
    assert orc.dot_f32([1e8, 1.0, -1e8], [1.0, 1.0, 1.0]) == np.float32(0.0)


def test_fp32_recursive_dot_brute_force(orc):
    """The recursive FP32 dot is s = fl(s + fl(x_i y_i)) in index order:
    numpy FP32 scalars, one operation at a time."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal(257).astype(np.float32)
    y = rng.standard_normal(257).astype(np.float32)
    s = np.float32(0)
    for a, b in zip(x, y):
        s = np.float32(s + np.float32(a * b))
    assert orc.dot_f32(x, y) == s


def _tiny_mesh(orc, ne=2, N=2):
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=None)
    return bm, orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd)


def _groups(bm):
    glo = np.asarray(bm.glo).reshape(-1)
    order = np.argsort(glo, kind="stable")
    out = {}
    for i in order:
        out.setdefault(int(glo[i]), []).append(int(i))
    return [g for g in out.values()]


def _expected_gs(v, groups, n3, acc64, pairwise, erank):
    """Gather-scatter of an FP32 vector taken one addition at a time (numpy
    FP32 scalars, or Python floats for FP64 sums rounded once to FP32)."""
    out = v.copy()

    def add(vals):
        if acc64:
            s = 0.0
            for a in vals:
                s = s + float(a)
            return s
        s = vals[0]
        for a in vals[1:]:
            s = np.float32(s + a)
        return s

    for g in groups:
        if not pairwise:
            val = np.float32(add([v[i] for i in g]))
            for i in g:
                out[i] = val
            continue
        rank = [int(erank[i // n3]) if erank is not None else i // n3 for i in g]
        ranks = sorted(set(rank))
        part = {R: add([v[i] for i, r in zip(g, rank) if r == R]) for R in ranks}
        for i, R in zip(g, rank):
            terms = [part[R]] + [part[Q] for Q in ranks if Q != R]
            if acc64:
                s = 0.0
                for t in terms:
                    s = s + t
            else:
                s = terms[0]
                for t in terms[1:]:
                    s = np.float32(s + t)
            out[i] = np.float32(s)
    return out


@pytest.mark.parametrize("acc64", [False, True])
@pytest.mark.parametrize("ranks", [None, (1, 1, 1), (1, 1, 2), (2, 2, 1), (2, 2, 2)])
def test_gs_f32_orders_brute_force(orc, acc64, ranks):
    """FP32 gather-scatter, one order per node and the pairwise order (every
    element its own rank, or px x py x pz blocks of elements), against sums
    taken one addition at a time, on a 4^3-element N = 2 box (copy counts
    1, 2, 4, 8)."""
    bm, M = _tiny_mesh(orc, ne=4, N=2)
    n3 = 27
    erank = None if ranks is None else W.block_ranks(4, *ranks)
    rng = np.random.default_rng(11)
    v = (rng.standard_normal(M.nloc) * 10.0 ** rng.integers(-3, 4, M.nloc)).astype(np.float32)
    groups = _groups(bm)
    assert {len(g) for g in groups} == {1, 2, 4, 8}
    one = M.gs_f32(v, acc64, pairwise=False)
    assert np.array_equal(one, _expected_gs(v, groups, n3, acc64, False, None))
    pw = M.gs_f32(v, acc64, pairwise=True, erank=erank)
    assert np.array_equal(pw, _expected_gs(v, groups, n3, acc64, True, erank))


def test_gs_f32_order_properties(orc):
    """With one order all copies of a node are equal, and with FP64 sums the
    result is the FP64 gather-scatter rounded to FP32.  In the pairwise order
    with FP32 sums, one rank or two ranks keep every node's copies equal
    (a + b = b + a), while with 2 x 2 x 2 ranks, or every element a rank of
    its own, copies of nodes shared by four or eight ranks differ somewhere."""
    bm, M = _tiny_mesh(orc, ne=4, N=3)
    rng = np.random.default_rng(12)
    v = (rng.standard_normal(M.nloc) * 10.0 ** rng.integers(-4, 5, M.nloc)).astype(np.float32)
    one64 = M.gs_f32(v, True, pairwise=False)
    assert np.array_equal(one64, M.gs(v.astype(np.float64)).astype(np.float32))
    one32 = M.gs_f32(v, False, pairwise=False)
    groups = _groups(bm)

    def n_split(x):
        return sum(int(np.any(x[g] != x[g][0])) for g in groups)

    assert n_split(one32) == 0
    assert n_split(M.gs_f32(v, False, True, W.block_ranks(4, 1, 1, 1))) == 0
    assert np.array_equal(M.gs_f32(v, False, True, W.block_ranks(4, 1, 1, 1)), one32)
    assert n_split(M.gs_f32(v, False, True, W.block_ranks(4, 1, 1, 2))) == 0
    assert n_split(M.gs_f32(v, False, True, W.block_ranks(4, 2, 2, 2))) > 0
    per_elem = M.gs_f32(v, False, True, None)
    assert n_split(per_elem) > 0
    for g in groups:  # two copies (two ranks) always agree
        if len(g) == 2:
            assert per_elem[g[0]] == per_elem[g[1]]


def test_weighted_fp32_dot_definition(orc):
    """(a, b)_c in FP32: the terms are (fl(a_i c_i), b_i); on a box mesh the
    weights 1/m are powers of two, so a_i c_i is exact and the Dot2 result
    is within the Dot2 bound of the exact weighted dot."""
    bm, M = _tiny_mesh(orc, ne=3, N=3)
    rng = np.random.default_rng(13)
    a = rng.standard_normal(M.nloc).astype(np.float32)
    b = rng.standard_normal(M.nloc).astype(np.float32)
    c = M.c
    assert np.all(np.isin(c, [1.0, 0.5, 0.25, 0.125]))
    t = (a * c.astype(np.float32)).astype(np.float32)
    ex = exact_dot(t, b)
    absdot = float(np.sum(np.abs(t.astype(np.float64) * b)))
    r2 = M.dot_c_f32(a, b, dot2=True)
    assert abs(float(Fraction(float(r2)) - ex)) <= U32 * abs(float(ex)) + _gamma(M.nloc) ** 2 * absdot
    assert M.dot_c_f32(a, b, dot2=False) == orc.dot_f32(t, b)
