"""Synthetic input generators (no GPU): conformity, boundary flags, seeds,
deformation support, field statistics."""
import numpy as np

from paper_2503_02134_amd import workloads as W


def _xi(N):
    # any strictly increasing node set with endpoints +-1 serves the generator
    return np.concatenate([[-1.0], np.cos(np.pi * np.arange(N - 1, 0, -1) / N), [1.0]])


def test_equal_ids_iff_equal_coordinates():
    bm = W.box_mesh(3, 4, _xi(4), seed=2)
    P = bm.xyz.transpose(0, 2, 1).reshape(-1, 3)
    g = bm.glo.reshape(-1)
    # equal ids -> bitwise equal coordinates
    order = np.argsort(g, kind="stable")
    gs, Ps = g[order], P[order]
    same = gs[1:] == gs[:-1]
    assert np.all(Ps[1:][same] == Ps[:-1][same])
    # distinct ids -> distinct points
    uniq = np.unique(np.round(P, 12), axis=0)
    assert len(uniq) == len(np.unique(g))


def test_multiplicity_and_boundary_pattern():
    ne, N = 3, 3
    bm = W.box_mesh(ne, N, _xi(N))
    counts = np.bincount(bm.glo.reshape(-1))
    assert set(np.unique(counts)) == {1, 2, 4, 8}
    G1 = ne * N + 1
    assert len(counts) == G1 ** 3
    assert bm.bnd.sum() > 0
    onb = np.zeros(G1 ** 3, bool)
    onb[bm.glo.reshape(-1)[bm.bnd.reshape(-1) > 0]] = True
    assert onb.sum() == G1 ** 3 - (G1 - 2) ** 3


def test_deformation_vanishes_on_boundary_and_is_bounded():
    bm0 = W.box_mesh(4, 5, _xi(5))
    bm1 = W.box_mesh(4, 5, _xi(5), seed=7)
    d = bm1.gxyz - bm0.gxyz
    onb = np.zeros(len(d), bool)
    onb[bm0.glo.reshape(-1)[bm0.bnd.reshape(-1) > 0]] = True
    assert np.max(np.abs(d[onb])) < 1e-15
    assert 0.0 < np.max(np.abs(d)) <= 0.05 * bm0.h * (1 + 1e-12)


def test_seeds_reproducible():
    a = W.box_mesh(2, 3, _xi(3), seed=5)
    b = W.box_mesh(2, 3, _xi(3), seed=5)
    c = W.box_mesh(2, 3, _xi(3), seed=6)
    assert np.array_equal(a.xyz, b.xyz) and not np.array_equal(a.xyz, c.xyz)
    assert np.array_equal(W.random_smooth_rhs(a, 3), W.random_smooth_rhs(b, 3))


def test_lognormal_statistics():
    bm = W.box_mesh(6, 3, _xi(3))
    k = W.lognormal_k(bm, seed=5)
    g = np.log(k[np.unique(bm.glo.reshape(-1), return_index=True)[1]])
    assert abs(g.mean()) < 0.5 and 0.4 < g.std() < 1.6
    assert np.all(k > 0)


def test_batch_draws():
    d = W.batch_draws()
    assert len(d) == 64
    assert {x[0] for x in d} <= {8, 12, 16, 24} and {x[1] for x in d} <= {5, 7, 9}
    assert d == W.batch_draws()
