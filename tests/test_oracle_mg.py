"""Pins of the oracle's two-level Schwarz / multigrid preconditioner (no GPU).

  - each element's local solve equals numpy.linalg.solve with the separable
    extended-element operator built here by Kronecker products from 1-D
    matrices assembled independently (numpy GLL rule and derivative matrix,
    element lengths from the coordinates, the neighbours' face entries);
  - the coarse operator equals P^T A P with A the dense weak-form matrix
    (numpy Jacobians, quadrature) and P the trilinear hat functions of the
    element-vertex lattice evaluated at the GLL nodes;
  - every coarser lattice level equals P^T A P of the level above (dense);
  - the V-cycle and the whole preconditioner are symmetric and positive;
  - PCG with it reaches numpy.linalg.solve's solution, in several times
    fewer iterations than Jacobi PCG on an 8^3-element mesh.
"""
import numpy as np
import pytest

import refmath
from paper_2503_02134_amd import workloads as W


def _mesh(orc, ne, N, seed=None, kseed=None, hh=0.0, coarsest_max=512):
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=seed)
    k = None if kseed is None else W.lognormal_k(bm, kseed)
    om = orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd, kcoef=k, helm_h=hh)
    mg = orc.MG(om, ne, bm.xyz, k, coarsest_max=coarsest_max)
    return bm, om, mg, k


def _lengths(xyz_e, n):
    """mean distance between the end nodes of the element's lines, per direction"""
    X = xyz_e.reshape(3, n, n, n)  # [c][k][j][i]
    lx = np.linalg.norm(X[:, :, :, -1] - X[:, :, :, 0], axis=0).mean()
    ly = np.linalg.norm(X[:, :, -1, :] - X[:, :, 0, :], axis=0).mean()
    lz = np.linalg.norm(X[:, -1, :, :] - X[:, 0, :, :], axis=0).mean()
    return np.array([lx, ly, lz])


@pytest.mark.parametrize("seed,kseed,hh", [(None, None, 0.0), (4, None, 0.0), (4, 7, 1.5)])
def test_local_solve_is_the_separable_inverse(orc, seed, kseed, hh):
    ne, N = 4, 4
    n = N + 1
    bm, om, mg, k = _mesh(orc, ne, N, seed, kseed, hh)
    x, w = refmath.gll_numpy(N)
    D = refmath.lagrange_deriv(x)
    Ar = D.T @ np.diag(w) @ D
    E = bm.E
    L = np.array([_lengths(bm.xyz[e], n) for e in range(E)])
    r = om.mask_apply(np.random.default_rng(1).standard_normal(bm.glo.max() + 1)[bm.glo.reshape(-1)])
    zl = mg.schwarz_local(r)
    c = om.c
    for e in (0, 5, 21, E - 1):  # corner, edge, interior, corner elements
        ec = (e % ne, (e // ne) % ne, e // ne ** 2)
        strides = (1, ne, ne * ne)
        mats = []
        for d in range(3):
            l = L[e, d]
            A = (2.0 / l) * Ar.copy()
            B = np.diag(0.5 * l * w)
            if ec[d] > 0:
                ll = L[e - strides[d], d]
                A[0, 0] += (2.0 / ll) * Ar[N, N]
                B[0, 0] += 0.5 * ll * w[N]
            if ec[d] < ne - 1:
                lh = L[e + strides[d], d]
                A[N, N] += (2.0 / lh) * Ar[0, 0]
                B[N, N] += 0.5 * lh * w[0]
            for q, dir_ok in ((0, ec[d] == 0), (N, ec[d] == ne - 1)):
                if dir_ok:  # Dirichlet face: decoupled
                    A[q, :] = 0.0
                    A[:, q] = 0.0
                    A[q, q] = 1.0
                    B[q, q] = 1.0
            mats.append((A, B))
        (Ax, Bx), (Ay, By), (Az, Bz) = mats
        kb = 1.0 if k is None else k.reshape(E, -1)[e].mean()
        At = kb * (np.kron(Bz, np.kron(By, Ax)) + np.kron(Bz, np.kron(Ay, Bx))
                   + np.kron(Az, np.kron(By, Bx))) + hh * np.kron(Bz, np.kron(By, Bx))
        sl = slice(e * n ** 3, (e + 1) * n ** 3)
        ws = np.sqrt(c[sl])
        ref = ws * np.linalg.solve(At, ws * r[sl])
        np.testing.assert_allclose(zl[sl], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def _hat_matrix(bm, N, x):
    """P[f, I]: trilinear hats of the interior element-vertex lattice nodes at
    the unique GLL nodes f (box lattice ids)."""
    ne = bm.ne
    G1 = ne * N + 1
    gids = np.unique(bm.glo.reshape(-1))
    nu = ne - 1

    def hat(g, I):
        ex = np.minimum(g // N, ne - 1)
        xi = x[g - ex * N]
        return np.where(I == ex, 0.5 * (1 - xi), np.where(I == ex + 1, 0.5 * (1 + xi), 0.0))

    gx, gy, gz = gids % G1, (gids // G1) % G1, gids // G1 ** 2
    P = np.zeros((len(gids), nu ** 3))
    for K in range(1, ne):
        for J in range(1, ne):
            for I in range(1, ne):
                P[:, (I - 1) + nu * ((J - 1) + nu * (K - 1))] = hat(gx, I) * hat(gy, J) * hat(gz, K)
    return P, gids


@pytest.mark.parametrize("seed,kseed,hh", [(None, None, 0.0), (2, 3, 0.7)])
def test_coarse_operator_is_galerkin(orc, seed, kseed, hh):
    ne, N = 3, 3
    bm, om, mg, k = _mesh(orc, ne, N, seed, kseed, hh)
    A, gids, _ = refmath.assemble_dense(bm.xyz, bm.glo, N, k, hh)
    x, _ = refmath.gll_numpy(N)
    P, _ = _hat_matrix(bm, N, x)
    Ac = P.T @ A @ P
    A0 = mg.level_dense(0)
    np.testing.assert_allclose(A0, Ac, rtol=1e-11, atol=1e-12 * np.abs(Ac).max())


def test_lattice_levels_are_galerkin(orc):
    bm, om, mg, _ = _mesh(orc, 8, 2, seed=5, coarsest_max=27)
    assert mg.nlev == 2 and mg.level_nu(0) == 7 and mg.level_nu(1) == 3
    A0, A1 = mg.level_dense(0), mg.level_dense(1)

    def p1(f, c):
        d = f - 2 * c
        return 1.0 if d == 0 else 0.5 if abs(d) == 1 else 0.0

    nuf, nuc = 7, 3
    P = np.zeros((nuf ** 3, nuc ** 3))
    for K in range(1, nuf + 1):
        for J in range(1, nuf + 1):
            for I in range(1, nuf + 1):
                for ck in range(1, nuc + 1):
                    for cj in range(1, nuc + 1):
                        for ci in range(1, nuc + 1):
                            P[(I - 1) + nuf * ((J - 1) + nuf * (K - 1)),
                              (ci - 1) + nuc * ((cj - 1) + nuc * (ck - 1))] = (
                                p1(I, ci) * p1(J, cj) * p1(K, ck))
    np.testing.assert_allclose(A1, P.T @ A0 @ P, rtol=1e-12, atol=1e-13 * np.abs(A1).max())
    # the damping of each level is one over its row-sum bound of D^-1 A
    for l, A in enumerate((A0, A1)):
        bound = (np.abs(A).sum(axis=1) / np.diag(A)).max()
        assert abs(mg.level_omega(l) - 1.0 / bound) <= 1e-14


def test_preconditioner_is_symmetric_positive(orc):
    bm, om, mg, _ = _mesh(orc, 8, 3, seed=6, coarsest_max=27)
    rng = np.random.default_rng(3)
    nc = mg.level_nu(0) ** 3
    b1, b2 = rng.standard_normal(nc), rng.standard_normal(nc)
    v1, v2 = mg.vcycle(b1), mg.vcycle(b2)
    assert abs(v1 @ b2 - b1 @ v2) <= 1e-12 * abs(v1 @ b2)
    assert v1 @ b1 > 0 and v2 @ b2 > 0
    g = bm.glo.max() + 1
    u = om.mask_apply(rng.standard_normal(g)[bm.glo.reshape(-1)])
    v = om.mask_apply(rng.standard_normal(g)[bm.glo.reshape(-1)])
    Mu, Mv = mg.apply(u), mg.apply(v)
    assert abs(om.dot(Mu, v) - om.dot(u, Mv)) <= 1e-12 * abs(om.dot(Mu, v))
    assert om.dot(Mu, u) > 0 and om.dot(Mv, v) > 0
    # the result is continuous and zero on Dirichlet nodes
    np.testing.assert_allclose(om.gs(om.c * Mu), Mu, rtol=0, atol=1e-13 * np.abs(Mu).max())
    assert np.all(Mu[om.mask.astype(bool)] == 0.0)


def test_mg_pcg_solves_and_beats_jacobi(orc):
    bm, om, mg, _ = _mesh(orc, 2, 3, seed=1)
    b = om.rhs(W.random_smooth_rhs(bm, 2))
    x, st = om.pcg(b, tol=1e-12, maxit=500, mg=mg)
    A, gids, inv = refmath.assemble_dense(bm.xyz, bm.glo, 3)
    free = ~np.isin(gids, np.unique(bm.glo.reshape(-1)[bm.bnd.reshape(-1) != 0]))
    bu = np.zeros(len(gids))
    bu[inv.reshape(-1)] = b  # b is continuous
    xu = np.zeros(len(gids))
    xu[free] = np.linalg.solve(A[np.ix_(free, free)], bu[free])
    np.testing.assert_allclose(x, xu[inv.reshape(-1)], rtol=0, atol=1e-10 * np.abs(xu).max())
    bm8, om8, mg8, _ = _mesh(orc, 8, 4, seed=1)
    b8 = om8.rhs(W.manufactured(bm8)[0])
    _, sj = om8.pcg(b8, tol=1e-10, maxit=5000)
    _, sm = om8.pcg(b8, tol=1e-10, maxit=5000, mg=mg8)
    assert sm.reason == orc.CONVERGED and sm.rel_res_true <= 2e-10
    assert sm.iterations * 4 <= sj.iterations, (sm.iterations, sj.iterations)


def test_refuses_non_box_meshes(orc):
    xi, _ = orc.gll(2)
    bm = W.box_mesh(3, 2, xi)
    om = orc.Mesh(bm.E, 2, bm.xyz, bm.glo, np.zeros_like(bm.bnd))  # no Dirichlet boundary
    with pytest.raises(ValueError):
        orc.MG(om, 3, bm.xyz)
    om2 = orc.Mesh(bm.E, 2, bm.xyz, bm.glo, bm.bnd)
    with pytest.raises(ValueError):
        orc.MG(om2, 2, bm.xyz)  # E is not 2^3
