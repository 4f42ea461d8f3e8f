"""Learned flexible-CG preconditioner: network handle, training data from the
FP64 solver, and the training loop.  Argument marshalling only: the forward
and backward passes, the loss (with its operator applications), Adam and
the training pairs are computed by the library's kernels.

Training data: for each right-hand side b, the FP64 solver gives x* (tight
tolerance) and a trajectory of restarted FP64 PCG chunks from x = 0; every
chunk end x_k yields the pair r = (b - A x_k)/||.||, e = (x* - x_k)/||.||,
so the network learns the map from a residual to the error it hides.
"""
from __future__ import annotations

import numpy as np
import torch

from . import mxsem as mx
from . import workloads as W


class Network:
    """Per-element 2-layer 3x3x3 conv correction to Jacobi (2 -> 32 -> 1)."""

    def __init__(self, mesh: "mx.Mesh", W1=None, W2=None, seed: int = 0, max_samples: int = 16):
        self.mesh = mesh
        self.h, self.ws = mx.mxsem_nn_create(mesh.h, max_samples=max_samples)
        mesh.ctx._adopt(self)
        if W1 is None:
            W1, W2 = W.he_normal_weights(seed)
        self.set(W1, W2)
        self.step = 0

    def close(self):
        if self.h is not None:
            mx.mxsem_mesh_attach_nn(self.mesh.h, None)
            mx.mxsem_nn_destroy(self.h)
            self.h = None
            self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, W1, W2):
        mx.mxsem_nn_set_params(self.h, np.asarray(W1, np.float32).reshape(32, 2, 27),
                               np.asarray(W2, np.float32).reshape(32, 27))
        self.step = 0

    def get(self):
        return mx.mxsem_nn_get_params(self.h)

    def attach(self):
        mx.mxsem_mesh_attach_nn(self.mesh.h, self.h)

    def forward(self, r):
        z = torch.empty_like(r)
        mx.mxsem_nn_forward(self.h, r, z)
        return z

    def loss_grad(self, R, E):
        ns = R.shape[0] if R.dim() == 2 else 1
        loss = torch.zeros(1, dtype=torch.float64, device=R.device)
        grad = torch.zeros(32 * 2 * 27 + 32 * 27, dtype=torch.float32, device=R.device)
        mx.mxsem_nn_loss_grad(self.h, R.contiguous(), E.contiguous(), ns, loss, grad)
        return loss, grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        mx.mxsem_nn_adam_step(self.h, lr, beta1, beta2, eps, self.step)


def make_pairs(mesh: "mx.Mesh", rhs: list, samples: int = 8, mesh_np=None, seed: int = 0,
               tol_star: float = 1e-12):
    """(R, E) device FP32 tensors [len(rhs) * samples, nloc] of training pairs.

    For each right-hand side: x* from a tight FP64 solve; then, from a rough
    seeded initial guess x0 (when mesh_np is given, else x0 = 0), restarted
    FP64 PCG chunks of 0, 1, 1, 2, 4, 8, ... iterations; each chunk end gives
    one pair, so the errors range from rough to smooth."""
    R, E = [], []
    for q, b in enumerate(rhs):
        xs = torch.zeros_like(b)
        mesh.solve(b, xs, mode=mx.MODE_FP64, tol=tol_star, max_iter=50000)
        if mesh_np is not None:
            x = torch.as_tensor(W.random_nodal_field(mesh_np, seed + 7919 * q), device=b.device)
        else:
            x = torch.zeros_like(b)
        step = 0
        for k in range(samples):
            if step > 0:
                mesh.solve(b, x, mode=mx.MODE_FP64, tol=0.0, max_iter=step, x0_given=1)
            r = torch.empty(mesh.nloc, dtype=torch.float32, device=b.device)
            e = torch.empty_like(r)
            mx.mxsem_nn_make_pair(mesh.h, b, x, xs, r, e)
            R.append(r)
            E.append(e)
            step = 1 if step == 0 else (step if k == 1 else 2 * step)
    return torch.stack(R), torch.stack(E)


def train(net: Network, R, E, steps: int, batch: int = 4, lr: float = 1e-3, seed: int = 0,
          log=None):
    """Adam on minibatches drawn (seeded) from the pairs; returns the losses."""
    rng = np.random.default_rng(seed)
    n = R.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.as_tensor(np.sort(rng.choice(n, size=min(batch, n), replace=False)),
                              device=R.device)
        loss, _ = net.loss_grad(R.index_select(0, idx), E.index_select(0, idx))
        net.adam(lr=lr)
        losses.append(float(loss.item()))
        if log and (it % 25 == 0 or it == steps - 1):
            log(f"train step {it}: loss {losses[-1]:.4f}")
    return losses


def rhs_batch(mesh_np, mesh: "mx.Mesh", seeds):
    """Device right-hand sides b = M QQ^T (B f) for seeded random smooth f."""
    out = []
    for s in seeds:
        f = W.random_smooth_rhs(mesh_np, s)
        out.append(mesh.mass_rhs(torch.as_tensor(f, device=mesh.dev)))
    return out


def compare_on(mesh: "mx.Mesh", rhs: list, net: Network, tol: float = 1e-10,
               max_iter: int = 50000):
    """Learned flexible CG vs Jacobi PCG (both inside FP64 refinement with the
    FP32 inner loop) and FP64 Jacobi PCG on the same right-hand sides."""
    net.attach()
    rows = []
    for b in rhs:
        x64 = torch.zeros_like(b)
        _, s64 = mesh.solve(b, x64, mode=mx.MODE_FP64, tol=tol, max_iter=max_iter)
        xj = torch.zeros_like(b)
        _, sj = mesh.solve(b, xj, mode=mx.MODE_MIXED_IR, tol=tol, max_iter=max_iter)
        xl = torch.zeros_like(b)
        _, sl = mesh.solve(b, xl, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED,
                           method=mx.METHOD_FCG, tol=tol, max_iter=max_iter)
        dn = float(torch.linalg.vector_norm(x64))
        rows.append({
            "fp64": (s64.iterations, s64.ms, s64.rel_res),
            "jacobi": (sj.iterations + sj.outer, sj.ms, sj.rel_res),
            "learned": (sl.iterations + sl.outer, sl.ms, sl.rel_res, sl.fallback_used),
            "learned_vs_fp64": float(torch.linalg.vector_norm(xl - x64)) / dn,
            "jacobi_vs_fp64": float(torch.linalg.vector_norm(xj - x64)) / dn,
        })
    return rows


def calibrate_scale(net: Network, mesh: "mx.Mesh", b, scales=(1.0, 0.5, 0.35, 0.25, 0.18, 0.125),
                    tol: float = 1e-8, max_iter: int = 50000, log=None):
    """Choose the factor applied to the learned correction (W2 scaled, so
    z_L = dinv r + lambda s_e y) by the flexible-CG iteration count on a
    training right-hand side: the A-norm loss fits one application, while CG
    prefers a damped correction.  Leaves the best scale in the network and
    returns (scale, {scale: iterations})."""
    W1, W2 = net.get()
    net.attach()
    its = {}
    for lam in scales:
        net.set(W1, W2 * lam)
        _, st = mesh.solve(b, mode=mx.MODE_MIXED_IR, pc=mx.PC_LEARNED, method=mx.METHOD_FCG,
                           tol=tol, max_iter=max_iter)
        its[lam] = st.iterations + st.outer if st.reason == mx.CONVERGED else 10 ** 9
        if log:
            log(f"calibrate lambda {lam}: {its[lam]} iterations")
    best = min(its, key=its.get)
    net.set(W1, W2 * best)
    return best, its
