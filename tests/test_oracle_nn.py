"""Pins of the oracle's learned flexible-CG preconditioner (no GPU):
forward pass against scipy's correlation, zero weights = Jacobi,
positive homogeneity, analytic gradients against central differences, Adam
against its closed form after one step."""
import numpy as np
import pytest

import refmath
from paper_2503_02134_amd import workloads as W


def _setup(orc, ne=2, N=3, seed=9, ch=4):
    xi, _ = orc.gll(N)
    bm = W.box_mesh(ne, N, xi, seed=seed)
    M = orc.Mesh(bm.E, N, bm.xyz, bm.glo, bm.bnd)
    W1, W2 = W.he_normal_weights(17, ch=ch)
    nn = orc.NN(W1, W2)
    return bm, M, nn


def _continuous(bm, M, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(bm.glo.max() + 1)
    return M.mask_apply(g[bm.glo.reshape(-1)])


def test_forward_matches_scipy_correlation(orc):
    """y per element equals two scipy.ndimage correlations with a ReLU in
    between, on the scaled input [r, dinv r]/||dinv r||_e."""
    bm, M, nn = _setup(orc)
    r = _continuous(bm, M, 1)
    zL, y = nn.local(M, r)
    n = bm.n
    dinv = M.dinv
    for e in range(bm.E):
        sl = slice(e * n ** 3, (e + 1) * n ** 3)
        dr = dinv[sl] * r[sl]
        s = np.linalg.norm(dr)
        x0 = [(r[sl] / s).reshape(n, n, n), (dr / s).reshape(n, n, n)]
        a1 = np.zeros((nn.ch, n, n, n))
        for c in range(nn.ch):
            for ci in range(2):
                a1[c] += refmath.conv3_same(x0[ci], nn.W1[c, ci])
        hh = np.maximum(a1, 0.0)
        ye = sum(refmath.conv3_same(hh[c], nn.W2[c]) for c in range(nn.ch)).reshape(-1)
        np.testing.assert_allclose(y[sl], ye, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(zL[sl], dr + s * ye, rtol=1e-12, atol=1e-13)


def test_zero_weights_is_jacobi(orc):
    bm, M, nn = _setup(orc)
    nn.set(np.zeros_like(nn.W1), np.zeros_like(nn.W2))
    r = _continuous(bm, M, 2)
    z = nn.apply(M, r)
    np.testing.assert_allclose(z, M.dinv * r, rtol=1e-14, atol=1e-300)
    # and FCG with it follows PCG(Jacobi)
    f = W.random_smooth_rhs(bm, 3)
    b = M.rhs(f)
    _, s1 = M.pcg(b, tol=1e-10)
    _, s2 = M.fcg(b, nn=nn, tol=1e-10)
    assert abs(s1.iterations - s2.iterations) <= 1


def test_positive_homogeneity_and_continuity(orc):
    bm, M, nn = _setup(orc)
    r = _continuous(bm, M, 4)
    z1 = nn.apply(M, r)
    z2 = nn.apply(M, 3.7 * r)
    np.testing.assert_allclose(z2, 3.7 * z1, rtol=1e-13, atol=1e-14 * np.max(np.abs(z2)))
    # z is continuous: every copy of a node holds the same value
    np.testing.assert_allclose(M.gs(M.c * z1), z1, rtol=1e-13, atol=1e-15)


def test_loss_gradient_central_differences(orc):
    """Analytic gradient of mean_s ||z_s - e_s||_A^2/||e_s||_A^2 against
    central differences on a sample of weights."""
    bm, M, nn = _setup(orc, ne=2, N=3, ch=4)
    R = np.stack([_continuous(bm, M, 10 + s) for s in range(2)])
    E = np.stack([_continuous(bm, M, 20 + s) for s in range(2)])
    loss, g1, g2 = nn.loss_grad(M, R, E)
    assert np.isfinite(loss) and loss > 0
    W1, W2 = nn.W1.copy(), nn.W2.copy()
    rng = np.random.default_rng(5)
    h = 1e-6
    gmax = max(np.max(np.abs(g1)), np.max(np.abs(g2)))
    for _ in range(12):
        which = rng.integers(0, 2)
        if which == 0:
            idx = tuple(rng.integers(0, s) for s in W1.shape)
            Wp, Wm = W1.copy(), W1.copy()
            Wp[idx] += h
            Wm[idx] -= h
            nn.set(Wp, W2)
            lp = nn.loss_grad(M, R, E)[0]
            nn.set(Wm, W2)
            lm = nn.loss_grad(M, R, E)[0]
            ga = g1[idx]
        else:
            idx = tuple(rng.integers(0, s) for s in W2.shape)
            Wp, Wm = W2.copy(), W2.copy()
            Wp[idx] += h
            Wm[idx] -= h
            nn.set(W1, Wp)
            lp = nn.loss_grad(M, R, E)[0]
            nn.set(W1, Wm)
            lm = nn.loss_grad(M, R, E)[0]
            ga = g2[idx]
        nn.set(W1, W2)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - ga) <= 1e-6 * gmax + 1e-6 * abs(ga), (which, idx, fd, ga)


def test_loss_is_zero_at_exact_error_map(orc):
    """With e = z(r) the loss is 0 and so is its gradient."""
    bm, M, nn = _setup(orc)
    r = _continuous(bm, M, 30)
    e = nn.apply(M, r)
    loss, g1, g2 = nn.loss_grad(M, r[None], e[None])
    assert loss < 1e-28
    assert np.max(np.abs(g1)) < 1e-12 and np.max(np.abs(g2)) < 1e-12


def test_adam_first_step_closed_form(orc):
    """After one Adam step from zero moments every parameter moves by
    -lr * sign(g) * |g| / (|g| + eps)."""
    rng = np.random.default_rng(0)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    th0 = th.copy()
    orc.adam(th, g, m, v, 1, lr=1e-3)
    np.testing.assert_allclose(th - th0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-13)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-13)
