"""Independent numpy/scipy routes used to pin the oracle.

Nothing here is shared with the oracle or with the HIP library: GLL weights
come from a moment system, the derivative matrix from barycentric Lagrange
weights, element matrices from the weak form evaluated by quadrature with
numpy.linalg for the Jacobian, and convolutions from scipy.ndimage.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gll_numpy(N: int):
    """GLL nodes: +-1 and the roots of L_N' (numpy's Legendre class);
    weights: the unique rule exact for x^0..x^N on those nodes (moment
    system), which for GLL is exact up to degree 2N-1."""
    inner = npleg.Legendre.basis(N).deriv().roots() if N > 1 else np.array([])
    x = np.sort(np.concatenate([[-1.0], np.real(inner), [1.0]]))
    V = np.vander(x, N + 1, increasing=True).T  # V[k, i] = x_i^k
    mom = np.array([(1 - (-1) ** (k + 1)) / (k + 1) for k in range(N + 1)])
    w = np.linalg.solve(V, mom)
    return x, w


def lagrange_deriv(x: np.ndarray) -> np.ndarray:
    """D[i, j] = l_j'(x_i) from barycentric weights."""
    n = len(x)
    bw = np.array([1.0 / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (bw[j] / bw[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def ref_grads(N: int):
    """Reference gradients of the n^3 nodal basis functions at the n^3 GLL
    nodes: dphi[a][q, p] = d phi_p / d r_a at node q (Kronecker products)."""
    x, w = gll_numpy(N)
    D = lagrange_deriv(x)
    I = np.eye(N + 1)
    # node index p = i + n (j + n k)  ->  kron order (k, j, i)
    Dr = np.kron(I, np.kron(I, D))
    Ds = np.kron(I, np.kron(D, I))
    Dt = np.kron(D, np.kron(I, I))
    W = np.kron(w, np.kron(w, w))
    return (Dr, Ds, Dt), W


def element_matrix(xyz_e: np.ndarray, N: int, k_e=None, helm_h: float = 0.0):
    """Weak-form element matrix  int k grad(phi_p).grad(phi_q) + h phi_p phi_q
    by GLL quadrature on the isoparametric element (xyz_e [3][n^3])."""
    (Dr, Ds, Dt), W = ref_grads(N)
    n3 = (N + 1) ** 3
    # Jacobian at every node: J[q, c, d] = d x_c / d r_d
    J = np.zeros((n3, 3, 3))
    for d, Dd in enumerate((Dr, Ds, Dt)):
        J[:, :, d] = (Dd @ xyz_e.T)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)  # Jinv[q, d, c] = d r_d / d x_c
    gref = np.stack([Dr, Ds, Dt], axis=0)  # [d, q, p]
    # physical gradient of phi_p at q: g[q, c, p] = sum_d Jinv[q, d, c] gref[d, q, p]
    g = np.einsum("qdc,dqp->qcp", Jinv, gref)
    wq = W * det * (np.ones(n3) if k_e is None else k_e)
    A = np.einsum("q,qcp,qcr->pr", wq, g, g)
    if helm_h:
        A += np.diag(helm_h * W * det)
    return A


def assemble_dense(xyz, glo, N, kcoef=None, helm_h=0.0):
    """Dense assembled matrix over unique global ids (ascending)."""
    E = xyz.shape[0]
    gids, inv = np.unique(glo.reshape(-1), return_inverse=True)
    inv = inv.reshape(E, -1)
    A = np.zeros((len(gids), len(gids)))
    for e in range(E):
        ke = None if kcoef is None else kcoef.reshape(E, -1)[e]
        Ae = element_matrix(xyz[e], N, ke, helm_h)
        idx = inv[e]
        A[np.ix_(idx, idx)] += Ae
    return A, gids, inv


def conv3_same(x: np.ndarray, w27: np.ndarray) -> np.ndarray:
    """3x3x3 cross-correlation with zero padding of a field x[k, j, i]; the
    kernel index o = (di+1) + 3 (dj+1) + 9 (dk+1)."""
    from scipy import ndimage
    K = w27.reshape(3, 3, 3)  # [dk][dj][di]
    return ndimage.correlate(x, K, mode="constant", cval=0.0)
