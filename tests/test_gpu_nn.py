"""Learned flexible-CG preconditioner through the C ABI vs the FP64 oracle:
forward, loss and gradients, Adam, flexible CG, fallback and training.

Forward tolerance, node by node.  The network rounds its inputs x0, its
weights and its hidden activations h to BF16 (nearest even, unit roundoff
u = 2^-8) and accumulates in FP32.  With S1 = sum |W1| |x0| over a hidden
value's 54 terms and Y1 = sum |W2| S1 over an output's 864 terms:
  - a product of two BF16-rounded factors is off by at most (2u + u^2)
    of its magnitude, so a hidden pre-activation is off by (2u + u^2) S1
    plus the FP32 sum's gamma_54 S1;
  - ReLU is 1-Lipschitz and h's own rounding adds u |h| <= u S1;
  - the second layer adds W2's rounding, u |W2| |h|, and gamma_864;
so |y_gpu - y| <= (4u + 12u^2 + 1e-4) Y1 = 0.0164 Y1.  s_e's own rounding
cancels (the network is positively homogeneous), the Jacobi part and the
scaling add FP32 roundings (1e-6 of |dinv r| + s_e Y1), and the assembly
z = M QQ^T(c zL) adds the copies' bounds with the weights c.  The oracle
evaluates Y1 itself: its forward with |W1|, |W2| on |r| (dinv >= 0) gives
s_e Y1 + dinv |r|."""
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


def _pair(orc, mx, ctx, ne=3, N=7, kseed=5, hh=1.0):
    xg, _ = mx.mxsem_gll(N)
    xo, _ = orc.gll(N)
    bmg = W.box_mesh(ne, N, xg)
    bmo = W.box_mesh(ne, N, xo)
    kg = W.lognormal_k(bmg, kseed) if kseed is not None else None
    ko = W.lognormal_k(bmo, kseed) if kseed is not None else None
    gm = mx.Mesh(ctx, bmg.E, N, bmg.xyz, bmg.glo, bmg.bnd, kcoef=kg, helm_h=hh)
    om = orc.Mesh(bmo.E, N, bmo.xyz, bmo.glo, bmo.bnd, kcoef=ko, helm_h=hh)
    return bmg, gm, bmo, om


def _cont(bm, om, seed):
    g = np.random.default_rng(seed).standard_normal(bm.glo.max() + 1)
    return om.mask_apply(g[bm.glo.reshape(-1)])


def _cos(a, b):
    return float(np.dot(a, b) / np.linalg.norm(a) / np.linalg.norm(b))


U_BF16 = 2.0 ** -8
FWD_C = 4 * U_BF16 + 12 * U_BF16 ** 2 + 1e-4


def forward_bound(orc, om, W1, W2, r):
    """Per-node bound on |z_gpu - z_oracle| (module docstring)."""
    onn = orc.NN(np.abs(W1), np.abs(W2))
    ra = np.abs(r)
    zl_abs, _ = onn.local(om, ra)
    jac_abs = om.dinv * ra
    sY1 = np.maximum(zl_abs - jac_abs, 0.0)
    bl = FWD_C * sY1 + 1e-6 * (jac_abs + sY1)
    return om.mask_apply(om.gs(om.c * bl)) + 1e-30


def check_forward_elementwise(z, zo, bound, what):
    err = np.abs(z - zo)
    ratio = float(np.max(err / bound))
    log(f"  {what}: max |z - z_oracle| / bound = {ratio:.3f} "
        f"(max err {err.max():.2e}, max bound {bound.max():.2e})")
    assert ratio <= 1.0, f"{what}: node {int(np.argmax(err / bound))} beyond its bound"


@pytest.mark.parametrize("N", [3, 5, 7])
def test_forward_matches_oracle(orc, mx, ctx, N):
    from paper_2503_02134_amd.learned import Network
    log(f"nn forward vs oracle, N = {N}, node by node")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, N=N)
    W1, W2 = W.he_normal_weights(11)
    net = Network(gm, W1, W2)
    onn = orc.NN(W1, W2)
    r = _cont(bmo, om, 1)
    z = net.forward(torch.as_tensor(r, dtype=torch.float32, device="cuda")).cpu().numpy()
    zo = onn.apply(om, r)
    check_forward_elementwise(z, zo, forward_bound(orc, om, W1, W2, r), "He-normal weights")
    jac = om.dinv * r
    cg, co = z - jac, zo - jac
    log(f"  rel L2 z {rel_l2(z, zo):.2e}; correction cos {_cos(cg, co):.6f} "
        f"rel {rel_l2(cg, co):.2e}")
    assert rel_l2(z, zo) <= 1e-2
    assert _cos(cg, co) >= 0.999 and rel_l2(cg, co) <= 3e-2
    # zero weights: exactly the (FP32) Jacobi map
    net.set(np.zeros_like(W1), np.zeros_like(W2))
    z0 = net.forward(torch.as_tensor(r, dtype=torch.float32, device="cuda")).cpu().numpy()
    assert rel_l2(z0, jac) <= 1e-6
    net.close()


@pytest.mark.parametrize("N", [3, 7])
def test_forward_single_taps(orc, mx, ctx, N):
    """One non-zero weight per layer, swept over every offset of each
    layer, for hidden channels at both ends of the range and both input
    channels: the output is then one shifted, rectified input, so a tap
    read at the wrong offset, channel or element border is off by O(1) at
    the nodes it touches, far beyond the node-by-node bound."""
    from paper_2503_02134_amd.learned import Network
    log(f"nn forward single taps, N = {N}")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=2, N=N)
    r = _cont(bmo, om, 3)
    rt = torch.as_tensor(r, dtype=torch.float32, device="cuda")
    net = Network(gm, np.zeros((32, 2, 27)), np.zeros((32, 27)))
    onn = orc.NN(np.zeros((32, 2, 27)), np.zeros((32, 27)))
    worst = 0.0
    for c, ci in ((0, 0), (31, 1), (17, 0)):
        for layer in (1, 2):
            for o in range(27):
                W1 = np.zeros((32, 2, 27))
                W2 = np.zeros((32, 27))
                W1[c, ci, o if layer == 1 else 13] = 1.0
                W2[c, o if layer == 2 else 13] = -1.0 if (o % 2) else 1.0
                net.set(W1, W2)
                onn.set(W1, W2)
                z = net.forward(rt).cpu().numpy()
                zo = onn.apply(om, r)
                bound = forward_bound(orc, om, W1, W2, r)
                ratio = float(np.max(np.abs(z - zo) / bound))
                worst = max(worst, ratio)
                assert ratio <= 1.0, (c, ci, layer, o, ratio)
    log(f"  162 tap settings, worst |z - z_oracle| / bound = {worst:.3f}")
    net.close()


def _bf16_exact(a):
    """The nearest BF16 values (so the network's own weight rounding is exact)."""
    return torch.as_tensor(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("N", [3, 5, 7])
def test_loss_and_gradient_match_oracle(orc, mx, ctx, N):
    """Loss and gradient over two pairs against the oracle's FP64 analytic
    gradient (itself pinned to central differences).  The weights are BF16
    values, so what remains between the two is the BF16 rounding of the
    network's inputs and hidden activations and the FP32 sums; the smaller
    orders get 3^3 elements so that each gradient entry sums over about as
    many positions as at N = 7."""
    from paper_2503_02134_amd.learned import Network
    log(f"nn loss/gradient vs oracle, N = {N}")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=2 if N == 7 else 3, N=N)
    W1, W2 = W.he_normal_weights(12)
    W1, W2 = _bf16_exact(W1), _bf16_exact(W2)
    net = Network(gm, W1, W2)
    onn = orc.NN(W1, W2)
    R = np.stack([_cont(bmo, om, 20 + s) for s in range(2)])
    E = np.stack([_cont(bmo, om, 30 + s) for s in range(2)])
    lo, g1, g2 = onn.loss_grad(om, R, E)
    loss, grad = net.loss_grad(torch.as_tensor(R, dtype=torch.float32, device="cuda"),
                               torch.as_tensor(E, dtype=torch.float32, device="cuda"))
    go = np.concatenate([g1.reshape(-1), g2.reshape(-1)])
    gg = grad.cpu().numpy().astype(np.float64)
    n1 = g1.size
    log(f"  loss gpu {float(loss.item()):.6f} oracle {lo:.6f}; grad cos {_cos(gg, go):.6f} "
        f"rel {rel_l2(gg, go):.2e} (W1 part {rel_l2(gg[:n1], go[:n1]):.2e}, "
        f"W2 part {rel_l2(gg[n1:], go[n1:]):.2e})")
    assert abs(float(loss.item()) - lo) <= 1e-2 * lo
    assert _cos(gg, go) >= 0.999 and rel_l2(gg, go) <= 2e-2
    # one Adam step equals the oracle's on the same gradient
    th = np.concatenate([W1.reshape(-1), W2.reshape(-1)])
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    thc = th.copy()
    orc.adam(thc, gg.copy(), m, v, 1, lr=1e-3)
    net.adam(lr=1e-3)
    a1, a2 = net.get()
    got = np.concatenate([a1.reshape(-1), a2.reshape(-1)]).astype(np.float64)
    np.testing.assert_allclose(got, thc, rtol=1e-5, atol=1e-7)
    net.close()


def test_fcg_jacobi_matches_pcg(orc, mx, ctx):
    log("flexible CG (Jacobi) vs PCG")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=3, kseed=5)
    f = W.random_smooth_rhs(bmg, 5901)
    b = gm.mass_rhs(torch.as_tensor(f, device="cuda"))
    _, s1 = gm.solve(b, mode=mx.MODE_FP64, tol=1e-10, max_iter=5000)
    _, s2 = gm.solve(b, mode=mx.MODE_FP64, method=mx.METHOD_FCG, tol=1e-10, max_iter=5000)
    fo = W.random_smooth_rhs(bmo, 5901)
    _, so = om.fcg(om.rhs(fo), pc=orc.PC_JACOBI, tol=1e-10, maxit=5000)
    log(f"  pcg {s1.iterations} fcg {s2.iterations} oracle fcg {so.iterations}")
    assert s2.reason == mx.CONVERGED and abs(s1.iterations - s2.iterations) <= 2
    assert abs(s2.iterations - so.iterations) <= 2


def test_learned_fcg_with_zero_weights_is_jacobi(orc, mx, ctx):
    from paper_2503_02134_amd.learned import Network
    log("learned FCG with zero weights")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=3)
    net = Network(gm, np.zeros((32, 2, 27)), np.zeros((32, 27)))
    net.attach()
    b = gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 5902), device="cuda"))
    _, sj = gm.solve(b, mode=mx.MODE_MIXED_IR, tol=1e-10, max_iter=5000)
    _, sl = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                     tol=1e-10, max_iter=5000)
    log(f"  jacobi it={sj.iterations} learned(0) it={sl.iterations} outer {sl.outer}")
    assert sl.reason == mx.CONVERGED and abs(sj.iterations - sl.iterations) <= 3 * (sl.outer + 1)
    net.close()


def test_fallback_matches_oracle(orc, mx, ctx):
    """Weights set to NaN from the host: the network's z is NaN at every
    step, the first one included, so every step takes the Jacobi z.  The
    oracle's flexible CG with the same NaN network does the same: one
    fallback per preconditioner application, i.e. as many as iterations.
    The FP32 flexible CG (no refinement) to a 1e-6 residual takes the
    oracle's FP64 count of iterations within 2; inside FP64 refinement the
    solve reaches the oracle's 1e-13 solution to 1e-8."""
    from paper_2503_02134_amd.learned import Network
    log("fallback with NaN weights vs the oracle")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=2)
    Wn1, Wn2 = np.full((32, 2, 27), np.nan), np.full((32, 27), np.nan)
    net = Network(gm, Wn1, Wn2)
    net.attach()
    onn = orc.NN(Wn1, Wn2)
    b = gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 5903), device="cuda"))
    bo = om.rhs(W.random_smooth_rhs(bmo, 5903))
    _, so = om.fcg(bo, nn=onn, tol=1e-6, maxit=5000)
    _, st1 = gm.solve(b, mode=mx.MODE_MIXED, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                      tol=1e-6, max_iter=5000)
    log(f"  to 1e-6: gpu it={st1.iterations} fallback={st1.fallback_used}; "
        f"oracle it={so.iterations} fallback={so.fallback}")
    assert so.reason == orc.CONVERGED and so.fallback == so.iterations
    assert st1.reason == mx.CONVERGED and st1.fallback_used == st1.iterations
    assert abs(st1.iterations - so.iterations) <= 2
    xs, _ = om.pcg(bo, tol=1e-13, maxit=5000)
    x, st = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                     tol=1e-10, max_iter=5000)
    err = rel_l2(x.cpu().numpy(), xs, om.c)
    log(f"  refinement to 1e-10: it={st.iterations} outer={st.outer} "
        f"fallback={st.fallback_used} res={st.rel_res:.2e} err={err:.2e}")
    assert st.reason == mx.CONVERGED and st.rel_res <= 1e-10
    assert st.fallback_used == st.iterations
    assert err <= 1e-8
    net.close()


def test_training_reduces_loss_and_solves(orc, mx, ctx):
    """Pairs from the FP64 GPU solver on a small log-normal Helmholtz
    problem; 60 Adam steps lower the loss; the trained network inside
    refinement reaches the oracle solution to 1e-8."""
    from paper_2503_02134_amd.learned import Network, make_pairs, train
    log("training smoke")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=3)
    rhs = [gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 5100 + s), device="cuda"))
           for s in range(3)]
    R, E = make_pairs(gm, rhs, samples=6)
    assert torch.isfinite(R).all() and torch.isfinite(E).all()
    net = Network(gm, seed=3)
    losses = train(net, R, E, steps=60, batch=4, lr=2e-3, seed=1)
    log(f"  loss {losses[0]:.4f} -> {np.mean(losses[-10:]):.4f}")
    assert np.mean(losses[-10:]) < 0.9 * np.mean(losses[:5])
    net.attach()
    fo = W.random_smooth_rhs(bmo, 5900)
    xs, _ = om.pcg(om.rhs(fo), tol=1e-13, maxit=20000)
    b = gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 5900), device="cuda"))
    x, st = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                     tol=1e-10, max_iter=20000)
    _, sj = gm.solve(b, mode=mx.MODE_MIXED_IR, tol=1e-10, max_iter=20000)
    err = rel_l2(x.cpu().numpy(), xs, om.c)
    log(f"  learned it={st.iterations} outer={st.outer} fb={st.fallback_used} err={err:.2e}; "
        f"jacobi it={sj.iterations}")
    assert st.reason == mx.CONVERGED and err <= 1e-8
    net.close()


def test_trained_network_gains_over_jacobi(orc, mx, ctx):
    """What the learned preconditioner buys: on an 8^3-element log-normal
    Helmholtz mesh (N = 7), a network trained on pairs from the FP64 solver
    of six right-hand sides, with its correction scale calibrated on one of
    them, solves two held-out right-hand sides with flexible CG (inside FP64
    refinement) in clearly fewer iterations than Jacobi PCG in the same
    refinement, reaching the same residual."""
    from paper_2503_02134_amd.learned import Network, calibrate_scale, make_pairs, rhs_batch, train
    log("learned vs Jacobi iterations, 8^3 elements, N = 7")
    xg, _ = mx.mxsem_gll(7)
    bm = W.box_mesh(8, 7, xg)
    k = W.lognormal_k(bm, 5)
    gm = mx.Mesh(ctx, bm.E, 7, bm.xyz, bm.glo, bm.bnd, kcoef=k, helm_h=1.0)
    train_rhs = rhs_batch(bm, gm, range(5100, 5106))
    R, E = make_pairs(gm, train_rhs, samples=8, mesh_np=bm, seed=11)
    net = Network(gm, seed=3)
    losses = train(net, R, E, steps=200, batch=4, lr=2e-3, seed=1)
    del R, E
    lam, cal = calibrate_scale(net, gm, train_rhs[0])
    log(f"  loss {np.mean(losses[:5]):.3f} -> {np.mean(losses[-20:]):.3f}; scale {lam}: {cal}")
    net.attach()
    for b in rhs_batch(bm, gm, (5900, 5901)):
        _, sj = gm.solve(b, mode=mx.MODE_MIXED_IR, tol=1e-10, max_iter=20000)
        _, sl = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                         tol=1e-10, max_iter=20000)
        nj, nl = sj.iterations + sj.outer, sl.iterations + sl.outer
        log(f"  jacobi {nj} it (res {sj.rel_res:.1e}); learned {nl} it (res {sl.rel_res:.1e}, "
            f"fallback steps {sl.fallback_used})")
        assert sj.reason == mx.CONVERGED and sl.reason == mx.CONVERGED
        assert sl.rel_res <= 1e-10
        assert nl <= 0.85 * nj
    net.close()
    gm.close()


@pytest.mark.slow
def test_full_size_forward_sampled(orc, mx, ctx):
    """The network forward on the learned benchmark's mesh (24^3 elements,
    N = 7, log-normal k, Helmholtz h = 1: the persistent grid's workgroups
    take about 18 elements each, where the small meshes above give each
    workgroup at most one).  On sampled elements the oracle assembles z from
    every element within two node-sharing layers of the sample: the first
    layer holds every element whose output reaches a sampled node, the
    second completes the first layer's Jacobi diagonal, which scales the
    network's inputs.  Same node-by-node bound as the small-mesh forward,
    with the norm checks beside it."""
    from paper_2503_02134_amd.learned import Network
    wl = W.WORKLOADS["box24_N7_lognormal_helmholtz"]
    log("full-size 24^3 N7 nn forward, sampled")
    xg, _ = mx.mxsem_gll(wl.N)
    bmg = W.box_mesh(wl.ne, wl.N, xg, seed=wl.deform_seed)
    gm = mx.Mesh(ctx, bmg.E, wl.N, bmg.xyz, bmg.glo, bmg.bnd,
                 kcoef=W.lognormal_k(bmg, wl.k_seed), helm_h=wl.helm_h)
    E, n3 = bmg.E, (wl.N + 1) ** 3
    glo = np.asarray(bmg.glo, dtype=np.int64).reshape(E, n3)
    bnd = np.asarray(bmg.bnd, dtype=np.uint8).reshape(E, n3)
    g = np.random.default_rng(41).standard_normal(glo.max() + 1)
    r = np.where(bnd != 0, 0.0, g[glo])  # continuous, zero on Dirichlet nodes
    W1, W2 = W.he_normal_weights(11)
    net = Network(gm, W1, W2)
    z = net.forward(torch.as_tensor(r.reshape(-1), dtype=torch.float32,
                                    device="cuda")).cpu().numpy().reshape(E, n3)
    net.close()
    del gm, bmg

    xo, _ = orc.gll(wl.N)
    bmo = W.box_mesh(wl.ne, wl.N, xo, seed=wl.deform_seed)
    ko = np.asarray(W.lognormal_k(bmo, wl.k_seed)).reshape(E, n3)
    rng = np.random.default_rng(42)
    sample = np.unique(np.concatenate([[0, E // 2 + wl.ne // 2, E - 1],
                                       rng.choice(E, 21, replace=False)]))
    l1 = np.isin(glo, np.unique(glo[sample])).any(axis=1)
    l1[sample] = True
    l2 = np.isin(glo, np.unique(glo[l1])).any(axis=1)
    l2[l1] = True
    closure = np.nonzero(l2)[0]
    _, sub = np.unique(glo[closure], return_inverse=True)
    om = orc.Mesh(len(closure), wl.N, np.asarray(bmo.xyz).reshape(E, -1)[closure],
                  sub.reshape(len(closure), n3), bnd[closure], kcoef=ko[closure],
                  helm_h=wl.helm_h)
    onn = orc.NN(W1, W2)
    pos = np.searchsorted(closure, sample)
    zo = onn.apply(om, r[closure].reshape(-1)).reshape(-1, n3)[pos].reshape(-1)
    jac = (om.dinv.reshape(-1, n3)[pos] * r[sample]).reshape(-1)
    zs = z[sample].reshape(-1)
    bound = forward_bound(orc, om, W1, W2, r[closure].reshape(-1)).reshape(-1, n3)[pos]
    check_forward_elementwise(zs, zo, bound.reshape(-1), "sampled elements")
    cg, co = zs - jac, zo - jac
    log(f"  {len(sample)} sampled elements, closure {len(closure)}: rel L2 z "
        f"{rel_l2(zs, zo):.2e}; correction cos {_cos(cg, co):.6f} rel {rel_l2(cg, co):.2e}")
    assert rel_l2(zs, zo) <= 1e-2
    assert _cos(cg, co) >= 0.999 and rel_l2(cg, co) <= 3e-2
