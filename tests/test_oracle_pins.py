"""Pins of the FP64 oracle against closed forms, invariants, brute force and
library routines (no GPU).  Each test names what fixes the expected value."""
import math
import os

import numpy as np
import pytest

import refmath
from paper_2503_02134_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([p.strip() for p in line.split("|")])
    return rows


def _ev(expr):
    return float(eval(expr, {"pi": math.pi}))


def _mesh(orc, ne, N, seed=None, kfield=None, helm_h=0.0):
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=seed)
    M = orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd, kcoef=kfield, helm_h=helm_h)
    return bm, M


# ---------------------------------------------------------------- O1 / O2
def test_gll_closed_forms(orc):
    """Golden GLL nodes/weights for N = 1..4 (textbook closed forms)."""
    for N, nodes, weights in _read_golden("gll_closed_forms.txt"):
        N = int(N)
        xi, w = orc.gll(N)
        np.testing.assert_allclose(xi, [_ev(t) for t in nodes.split(",")], atol=1e-15)
        np.testing.assert_allclose(w, [_ev(t) for t in weights.split(",")], rtol=1e-14)


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_gll_quadrature_exactness(orc, N):
    """GLL with N+1 points integrates x^k exactly for k <= 2N-1 and not 2N."""
    xi, w = orc.gll(N)
    assert abs(w.sum() - 2.0) < 1e-13
    for k in range(0, 2 * N):
        exact = (1 - (-1) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-13, (N, k)
    k = 2 * N
    assert abs(np.dot(w, xi ** k) - 2.0 / (k + 1)) > 1e-11
    # agrees with the numpy route (Legendre roots + moment system)
    xr, wr = refmath.gll_numpy(N)
    np.testing.assert_allclose(xi, xr, atol=2e-14)
    np.testing.assert_allclose(w, wr, atol=2e-12)


def test_deriv_closed_forms(orc):
    for N, rows in _read_golden("derivative_closed_forms.txt"):
        N = int(N)
        exp = np.array([[_ev(t) for t in r.split(",")] for r in rows.split(";")])
        np.testing.assert_allclose(orc.deriv(N), exp, atol=1e-15)


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_deriv_exact_on_polynomials(orc, N):
    """D differentiates x^k exactly (k <= N); rows sum to zero; centro-
    antisymmetry D_ij = -D_{N-i,N-j}; equals the barycentric route."""
    xi, _ = orc.gll(N)
    D = orc.deriv(N)
    for k in range(0, N + 1):
        dk = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(D @ xi ** k - dk)) < 1e-12 * max(1, N ** 2), (N, k)
    assert np.max(np.abs(D.sum(axis=1))) < 1e-12 * N ** 2
    np.testing.assert_allclose(D, -D[::-1, ::-1], atol=1e-12 * N ** 2)
    np.testing.assert_allclose(D, refmath.lagrange_deriv(refmath.gll_numpy(N)[0]),
                               atol=1e-10 * N ** 2)


# ---------------------------------------------------------------- O3
@pytest.mark.parametrize("N", [2, 5, 7])
def test_geometry_undeformed_closed_form(orc, N):
    """Cube elements of side h: G_rr = G_ss = G_tt = rho_i rho_j rho_k h/2,
    off-diagonal 0, B = rho_i rho_j rho_k h^3/8."""
    ne = 3
    bm, M = _mesh(orc, ne, N)
    _, w = orc.gll(N)
    h = 1.0 / ne
    www = np.einsum("k,j,i->kji", w, w, w).reshape(-1)
    G = M.G
    for q, val in ((0, h / 2), (3, h / 2), (5, h / 2)):
        np.testing.assert_allclose(G[:, q, :], np.broadcast_to(www * val, G[:, q, :].shape),
                                   rtol=1e-12)
    for q in (1, 2, 4):
        assert np.max(np.abs(G[:, q, :])) < 1e-14
    np.testing.assert_allclose(M.B.reshape(bm.E, -1),
                               np.broadcast_to(www * h ** 3 / 8, (bm.E, www.size)), rtol=1e-12)


def test_geometry_rejects_inverted_element(orc):
    xi, _ = orc.gll(2)
    bm = W.box_mesh(1, 2, xi)
    xyz = bm.xyz.copy()
    xyz[:, 0, :] *= -1.0  # mirror x: det J < 0
    with pytest.raises(ValueError):
        orc.Mesh(bm.E, 2, xyz, bm.glo, bm.bnd)


@pytest.mark.parametrize("N,seed", [(3, 11), (5, 12), (7, 13)])
def test_linear_field_energy_identity(orc, N, seed):
    """For u = a.x + b0 on a deformed mesh, sum_e u_L^T A_L u_L = |a|^2 sum B
    (D reproduces the isoparametric Jacobian exactly at the nodes), and
    A_L 1 = 0.  A wrong or transposed inverse Jacobian breaks this for a
    general vector a."""
    bm, M = _mesh(orc, 2, N, seed=seed)
    a = np.array([0.3, -1.7, 2.2])
    u = (np.einsum("c,ecp->ep", a, bm.xyz) + 0.25).reshape(-1)
    energy = np.dot(u, M.ax_local(u))
    assert abs(energy - np.dot(a, a) * M.B.sum()) < 1e-11 * np.dot(a, a) * M.B.sum()
    assert np.max(np.abs(M.ax_local(np.ones(M.nloc)))) < 1e-11


def test_linear_field_energy_identity_with_k(orc):
    """Constant k scales the energy by k; Helmholtz adds h u^T B u."""
    bm, M1 = _mesh(orc, 2, 4, seed=5)
    kf = np.full(bm.nloc, 2.5)
    _, Mk = _mesh(orc, 2, 4, seed=5, kfield=kf, helm_h=0.7)
    a = np.array([1.0, 0.5, -0.25])
    u = np.einsum("c,ecp->ep", a, bm.xyz).reshape(-1)
    e1 = np.dot(u, M1.ax_local(u))
    ek = np.dot(u, Mk.ax_local(u))
    assert abs(ek - (2.5 * e1 + 0.7 * np.dot(u * M1.B, u))) < 1e-11 * abs(ek)


# ---------------------------------------------------------------- O4-O7, O9
@pytest.mark.parametrize("N,seed,kf,hh", [(2, None, False, 0.0), (3, 21, False, 0.0),
                                          (4, 22, True, 1.0), (5, None, True, 0.5)])
def test_matrix_free_equals_dense(orc, N, seed, kf, hh):
    """2x2x2 mesh: the oracle's matrix-free apply equals the dense matrix
    assembled from weak-form element matrices (numpy route); the dense
    matrix is symmetric and PSD with one zero eigenvalue (Poisson, no
    Dirichlet); SPD once the Dirichlet rows/cols are removed; and the
    oracle's Jacobi diagonal equals the dense diagonal."""
    ne = 2
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=seed)
    kfield = W.lognormal_k(bm, seed=3, features=64) if kf else None
    M = orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd, kcoef=kfield, helm_h=hh)
    A, gids, inv = refmath.assemble_dense(bm.xyz, bm.glo, N, kfield, hh)
    scale = np.max(np.abs(A))
    assert np.max(np.abs(A - A.T)) < 1e-14 * scale * 10
    ev = np.linalg.eigvalsh(A)
    assert ev[0] > -1e-12 * ev[-1]
    if hh == 0.0:
        assert np.sum(np.abs(ev) < 1e-10 * ev[-1]) == 1
    rng = np.random.default_rng(0)
    # matrix-free local apply then QQ^T equals dense apply on a continuous u
    ug = rng.standard_normal(len(gids))
    uL = ug[inv].reshape(-1)
    w = M.gs(M.ax_local(uL))
    np.testing.assert_allclose(w, (A @ ug)[inv].reshape(-1), atol=1e-12 * scale)
    # masked operator = dense operator restricted to free nodes
    free_g = ~(bm.bnd.reshape(-1)[np.unique(inv.reshape(-1), return_index=True)[1]] > 0)
    Af = A[np.ix_(free_g, free_g)]
    assert np.linalg.eigvalsh(Af)[0] > 0
    ugm = ug * free_g
    wm = M.apply(ugm[inv].reshape(-1))
    np.testing.assert_allclose(wm, ((A @ ugm) * free_g)[inv].reshape(-1), atol=1e-12 * scale)
    # Jacobi diagonal (assembled, unmasked) equals diag(A)
    np.testing.assert_allclose(M.diag(), np.diag(A)[inv].reshape(-1), rtol=1e-12)
    dinv = M.dinv
    np.testing.assert_allclose(dinv, np.where(free_g, 1.0 / np.diag(A), 0.0)[inv].reshape(-1),
                               rtol=1e-12)


def test_patch_test_affine(orc):
    """On an undeformed mesh the assembled operator annihilates a linear
    field at every interior node (GLL exact for the integrands)."""
    bm, M = _mesh(orc, 3, 4)
    u = (0.5 * bm.xyz[:, 0] - 2 * bm.xyz[:, 1] + bm.xyz[:, 2] + 1).reshape(-1)
    w = M.gs(M.ax_local(u))
    interior = ~bm.bnd.reshape(-1).astype(bool)
    assert np.max(np.abs(w[interior])) < 1e-12


# ---------------------------------------------------------------- O5
def test_gather_scatter_invariants(orc):
    """QQ^T 1 = multiplicity in {1,2,4,8}; QQ^T is idempotent after the c
    weighting; (Qa, c Qb) = a.b over unique nodes; bitwise equal to a
    brute-force dictionary sum in ascending local order."""
    bm, M = _mesh(orc, 3, 3, seed=1)
    m = M.gs(np.ones(M.nloc))
    assert set(np.unique(m)) == {1.0, 2.0, 4.0, 8.0}
    np.testing.assert_array_equal(m, M.mult)
    np.testing.assert_array_equal(M.c, 1.0 / m)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(M.nloc)
    g1 = M.gs(v)
    np.testing.assert_allclose(M.gs(M.c * g1), g1, rtol=1e-14)
    ng = bm.glo.max() + 1
    a = rng.standard_normal(ng)
    b = rng.standard_normal(ng)
    l2g = bm.glo.reshape(-1)
    assert abs(M.dot(a[l2g], b[l2g]) - np.dot(a, b)) < 1e-12 * ng
    groups = {}
    for i, g in enumerate(l2g):
        groups.setdefault(int(g), []).append(i)
    brute = np.empty_like(v)
    for g, idx in groups.items():
        s = 0.0
        for i in sorted(idx):
            s += v[i]
        brute[idx] = s
    np.testing.assert_array_equal(g1, brute)
    assert M.ngroups == len(groups)


# ---------------------------------------------------------------- O10, O8
def test_hand_pins(orc):
    """Single free node problems solved by hand (golden file)."""
    for name, ne, N, acc, bc, uc in _read_golden("hand_pins.txt"):
        ne, N = int(ne), int(N)
        bm, M = _mesh(orc, ne, N)
        f, _ = W.manufactured(bm)
        b = M.rhs(f)
        free = ~bm.bnd.reshape(-1).astype(bool)
        assert abs(b[free][0] - _ev(bc)) < 1e-13
        diag = M.diag()
        assert abs(diag[free][0] - _ev(acc)) < 1e-13
        x, st = M.pcg(b, tol=1e-14, maxit=5)
        assert st.iterations == 1 and st.reason == 1
        assert abs(x[free][0] - _ev(uc)) < 1e-14, name
        np.testing.assert_allclose(x[free], _ev(uc), rtol=1e-14)


@pytest.mark.parametrize("N,ne,seed", [(2, 2, None), (3, 2, 31), (4, 2, 32), (3, 1, None)])
def test_pcg_equals_dense_solve(orc, N, ne, seed):
    """PCG (Jacobi and identity) equals numpy.linalg.solve on the free
    nodes to 1e-12, and the A-norm error decreases monotonically."""
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=seed)
    M = orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd)
    A, gids, inv = refmath.assemble_dense(bm.xyz, bm.glo, N)
    first = np.unique(inv.reshape(-1), return_index=True)[1]
    free_g = ~(bm.bnd.reshape(-1)[first] > 0)
    f = W.random_smooth_rhs(bm, seed=7)
    b = M.rhs(f)
    bg = b[first]
    xs = np.zeros(len(gids))
    xs[free_g] = np.linalg.solve(A[np.ix_(free_g, free_g)], bg[free_g])
    for pc in (orc.PC_JACOBI, orc.PC_IDENTITY):
        x, st = M.pcg(b, pc=pc, tol=1e-14, maxit=2000)
        np.testing.assert_allclose(x, xs[inv].reshape(-1), atol=1e-12 * np.max(np.abs(xs)))
    # monotone A-norm error of the Jacobi iterates
    errs = []
    for k in range(1, 12):
        xk, _ = M.pcg(b, pc=orc.PC_JACOBI, tol=0.0, maxit=k)
        e = xs - xk[first]
        errs.append(e @ A @ e)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) + 1e-28 for i in range(len(errs) - 1))


def test_spectral_convergence_in_N(orc):
    """E = 2^3, manufactured sin sin sin: the max nodal error falls
    geometrically with N (about 1e-9 by N = 10); the discrete solution is
    symmetric under x -> 1-x on the undeformed mesh."""
    errs = []
    for N in range(2, 11):
        bm, M = _mesh(orc, 2, N)
        f, u = W.manufactured(bm)
        x, st = M.pcg(M.rhs(f), tol=1e-13, maxit=2000)
        errs.append(np.max(np.abs(x - u)))
    for a, b in zip(errs[:-2], errs[2:]):
        assert b < a / 4
    assert errs[-1] < 1e-8
    # mirror symmetry at N = 5
    bm, M = _mesh(orc, 2, 5)
    f, _ = W.manufactured(bm)
    x, _ = M.pcg(M.rhs(f), tol=1e-14, maxit=2000)
    g = np.zeros(bm.glo.max() + 1)
    g[bm.glo.reshape(-1)] = x
    G1 = 2 * 5 + 1
    gg = g.reshape(G1, G1, G1)
    np.testing.assert_allclose(gg, gg[:, :, ::-1], atol=1e-12)
    np.testing.assert_allclose(gg, gg.transpose(2, 1, 0), atol=1e-12)


def test_algebraic_convergence_in_h(orc):
    """Fixed N = 3: halving h divides the B-weighted nodal L2 error by at
    least about 2^(N+1) = 16 (the L2 rate of order-N elements) and at most
    2^(2N) = 64 (nodal superconvergence); measured about 2^(N+2)."""
    N = 3
    errs = []
    for ne in (2, 4, 8):
        bm, M = _mesh(orc, ne, N)
        f, u = W.manufactured(bm)
        x, _ = M.pcg(M.rhs(f), tol=1e-13, maxit=5000)
        d = x - u
        errs.append(math.sqrt(np.sum(M.c * M.B * d * d)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 70 and 12 < r2 < 70, (r1, r2)


# ---------------------------------------------------------------- O13, O14
def test_iterative_refinement_logic(orc):
    """IR with tau_in = 1e-4 (FP64 inner): each outer step cuts the true
    residual by >= 1e-3, 1e-10 is reached within 4 outer steps, and the
    result equals the PCG solution."""
    bm, M = _mesh(orc, 3, 5, seed=41)
    f, _ = W.manufactured(bm)
    b = M.rhs(f)
    x, st, outer = M.ir(b, tol=1e-10, tau_in=1e-4, max_outer=10)
    assert st.reason == 1 and st.outer <= 4
    assert outer[0] == pytest.approx(1.0)
    assert all(outer[i + 1] <= 1e-3 * outer[i] for i in range(len(outer) - 1))
    xr, _ = M.pcg(b, tol=1e-13, maxit=5000)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) < 1e-9


def test_fcg_with_jacobi_matches_pcg(orc):
    """FCG(1) with the fixed SPD Jacobi map reproduces PCG's iteration
    count within 1 and its solution."""
    bm, M = _mesh(orc, 3, 5, seed=42)
    f, _ = W.manufactured(bm)
    b = M.rhs(f)
    x1, s1 = M.pcg(b, tol=1e-10, maxit=2000)
    x2, s2 = M.fcg(b, pc=orc.PC_JACOBI, tol=1e-10, maxit=2000)
    assert abs(s1.iterations - s2.iterations) <= 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-8


def test_maxiter_and_recursive_residual(orc):
    bm, M = _mesh(orc, 2, 4, seed=3)
    f, _ = W.manufactured(bm)
    b = M.rhs(f)
    _, s = M.pcg(b, tol=1e-30, maxit=3)
    assert s.reason == orc.MAXITER and s.iterations == 3
    # the FP64 recursive residual keeps falling far below the true one
    _, s = M.pcg(b, tol=1e-30, maxit=5000)
    assert s.reason == orc.CONVERGED
    assert s.rel_res_recursive <= 1e-30 and 1e-17 < s.rel_res_true < 1e-12
