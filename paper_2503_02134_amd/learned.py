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

    def __init__(self, mesh: "mx.Mesh", W1=None, W2=None, seed: int = 0):
        self.mesh = mesh
        self.h = mx.mxsem_nn_create(mesh.h)
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


def make_pairs(mesh: "mx.Mesh", rhs: list, samples: int, chunk: int | None = None,
               tol_star: float = 1e-12):
    """(R, E) device FP32 tensors [len(rhs) * samples, nloc] of training pairs."""
    R, E = [], []
    for b in rhs:
        xs = torch.zeros_like(b)
        _, st = mesh.solve(b, xs, mode=mx.MODE_FP64, tol=tol_star, max_iter=50000)
        step = chunk or max(1, st.iterations // (samples + 1))
        x = torch.zeros_like(b)
        for _ in range(samples):
            mesh.solve(b, x, mode=mx.MODE_FP64, tol=0.0, max_iter=step, x0_given=1)
            r = torch.empty(mesh.nloc, dtype=torch.float32, device=b.device)
            e = torch.empty_like(r)
            mx.mxsem_nn_make_pair(mesh.h, b, x, xs, r, e)
            R.append(r)
            E.append(e)
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
