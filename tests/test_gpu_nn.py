"""Learned flexible-CG preconditioner through the C ABI vs the FP64 oracle:
forward, loss and gradients, Adam, flexible CG, fallback and training.

Tolerances: the network runs with BF16-rounded inputs, weights and hidden
activations and FP32 accumulation, so its correction carries relative
errors of a few 2^-9 against the FP64 oracle; the Jacobi part is FP32."""
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


def test_forward_matches_oracle(orc, mx, ctx):
    from paper_2503_02134_amd.learned import Network
    log("nn forward vs oracle")
    bmg, gm, bmo, om = _pair(orc, mx, ctx)
    W1, W2 = W.he_normal_weights(11)
    net = Network(gm, W1, W2)
    onn = orc.NN(W1, W2)
    r = _cont(bmo, om, 1)
    z = net.forward(torch.as_tensor(r, dtype=torch.float32, device="cuda")).cpu().numpy()
    zo = onn.apply(om, r)
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


def test_loss_and_gradient_match_oracle(orc, mx, ctx):
    from paper_2503_02134_amd.learned import Network
    log("nn loss/gradient vs oracle")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=2)
    W1, W2 = W.he_normal_weights(12)
    net = Network(gm, W1, W2)
    onn = orc.NN(W1, W2)
    R = np.stack([_cont(bmo, om, 20 + s) for s in range(2)])
    E = np.stack([_cont(bmo, om, 30 + s) for s in range(2)])
    lo, g1, g2 = onn.loss_grad(om, R, E)
    loss, grad = net.loss_grad(torch.as_tensor(R, dtype=torch.float32, device="cuda"),
                               torch.as_tensor(E, dtype=torch.float32, device="cuda"))
    go = np.concatenate([g1.reshape(-1), g2.reshape(-1)])
    gg = grad.cpu().numpy().astype(np.float64)
    log(f"  loss gpu {float(loss.item()):.6f} oracle {lo:.6f}; grad cos {_cos(gg, go):.6f} "
        f"rel {rel_l2(gg, go):.2e}")
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


def test_fallback_on_non_finite_network(orc, mx, ctx):
    """Weights set to NaN from the host: every learned step falls back to
    Jacobi and the solve still converges."""
    from paper_2503_02134_amd.learned import Network
    log("fallback with NaN weights")
    bmg, gm, bmo, om = _pair(orc, mx, ctx, ne=2)
    net = Network(gm, np.full((32, 2, 27), np.nan), np.full((32, 27), np.nan))
    net.attach()
    b = gm.mass_rhs(torch.as_tensor(W.random_smooth_rhs(bmg, 5903), device="cuda"))
    x, st = gm.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                     tol=1e-10, max_iter=5000)
    log(f"  it={st.iterations} fallback={st.fallback_used} res={st.rel_res:.2e}")
    assert st.reason == mx.CONVERGED and st.fallback_used > 0 and st.rel_res <= 1e-10
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
    network's inputs.  Same tolerances as the small-mesh forward."""
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
    cg, co = zs - jac, zo - jac
    log(f"  {len(sample)} sampled elements, closure {len(closure)}: rel L2 z "
        f"{rel_l2(zs, zo):.2e}; correction cos {_cos(cg, co):.6f} rel {rel_l2(cg, co):.2e}")
    assert rel_l2(zs, zo) <= 1e-2
    assert _cos(cg, co) >= 0.999 and rel_l2(cg, co) <= 3e-2
