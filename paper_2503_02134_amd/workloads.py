"""Seeded synthetic inputs: box meshes, deformations, coefficient fields, RHS.

This module is the problem statement shared by the HIP path and by the CPU
oracle.  It holds none of the solver's arithmetic: no quadrature, no
derivative matrix, no operator, no gather-scatter.  The one piece of the
discretisation a nodal mesh needs, the 1-D reference node positions, is a
parameter (``xi``) that each caller supplies from its own GLL routine.

Mesh conventions (unit cube [0,1]^3, ne elements per direction, order N,
n = N+1 nodes per direction):
  element e = ex + ne*(ey + ne*ez); local node (i,j,k) -> entry
  ((e*n + k)*n + j)*n + i; global lattice index gx = ex*N + i (likewise y, z);
  global id = gx + G1*(gy + G1*gz) with G1 = ne*N + 1.
Coordinates and every field are evaluated once per global node and then
scattered to the local copies, so the copies of a shared node agree bitwise.

The workloads stand in for the paper's Nekbone box meshes and Neko's cube
Poisson case (Sec. 6.1.2 and Sec. 6.2; no public dataset is involved).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class BoxMesh:
    ne: int
    N: int
    xyz: np.ndarray  # [E][3][n^3] float64
    glo: np.ndarray  # [E][n^3] int64
    bnd: np.ndarray  # [E][n^3] uint8, 1 on the boundary of the cube
    h: float         # element size 1/ne
    gxyz: np.ndarray = field(repr=False)  # [G1^3][3] coordinates per global node
    l2g: np.ndarray = field(repr=False)   # [E*n^3] global id per local entry

    @property
    def E(self) -> int:
        return self.ne ** 3

    @property
    def n(self) -> int:
        return self.N + 1

    @property
    def nloc(self) -> int:
        return self.E * self.n ** 3

    def to_local(self, g: np.ndarray) -> np.ndarray:
        """Scatter a per-global-node field to the local layout [E*n^3]."""
        return np.ascontiguousarray(g[self.l2g])


def _lattice_1d(ne: int, N: int, xi: np.ndarray) -> np.ndarray:
    """Undeformed 1-D node positions of the global lattice (ne*N+1 points)."""
    xi = np.asarray(xi, dtype=np.float64)
    assert xi.shape == (N + 1,)
    g = np.arange(ne * N + 1)
    e = np.minimum(g // N, ne - 1)
    loc = g - e * N
    return (e + 0.5 * (xi[loc] + 1.0)) / ne


def _local_to_global(ne: int, N: int) -> np.ndarray:
    n = N + 1
    G1 = ne * N + 1
    ez, ey, ex = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    gx = (ex.reshape(-1, 1) * N + i.reshape(1, -1))
    gy = (ey.reshape(-1, 1) * N + j.reshape(1, -1))
    gz = (ez.reshape(-1, 1) * N + k.reshape(1, -1))
    return (gx + G1 * (gy + G1 * gz)).astype(np.int64).reshape(-1)


def smooth_field(seed: int, pts: np.ndarray, modes: int = 16, kmax: int = 4) -> np.ndarray:
    """Seeded smooth scalar field vanishing on the cube boundary, max |.| = 1.

    phi(x) = S(x) * sum_m a_m cos(2 pi k_m . x + theta_m) / max|sum|, with
    S = sin(pi x) sin(pi y) sin(pi z), integer k_m in [-kmax, kmax]^3,
    a_m ~ N(0,1), theta_m ~ U(0, 2 pi).  Returns one value per point.
    """
    rng = np.random.default_rng(seed)
    kv = rng.integers(-kmax, kmax + 1, size=(modes, 3))
    a = rng.standard_normal(modes)
    th = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    s = np.zeros(len(pts))
    for m in range(modes):
        s += a[m] * np.cos(2.0 * np.pi * (pts @ kv[m].astype(np.float64)) + th[m])
    s /= np.max(np.abs(s))
    S = np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1]) * np.sin(np.pi * pts[:, 2])
    return S * s


def box_mesh(ne: int, N: int, xi, seed: int | None = None, amp: float = 0.05) -> BoxMesh:
    """Box mesh of ne^3 hexahedra of order N on the unit cube.

    With a seed, every node (interior and element-face nodes alike, so the
    mesh stays conforming) moves by amp*h*phi_c(x) in each direction c, phi_c
    a seeded smooth field that vanishes on the cube boundary.
    """
    n = N + 1
    G1 = ne * N + 1
    x1 = _lattice_1d(ne, N, xi)
    gz, gy, gx = np.meshgrid(np.arange(G1), np.arange(G1), np.arange(G1), indexing="ij")
    gxyz = np.stack([x1[gx.reshape(-1)], x1[gy.reshape(-1)], x1[gz.reshape(-1)]], axis=1)
    h = 1.0 / ne
    if seed is not None:
        disp = np.stack([smooth_field(seed * 3 + c, gxyz) for c in range(3)], axis=1)
        gxyz = gxyz + amp * h * disp
    onb = ((gx == 0) | (gx == G1 - 1) | (gy == 0) | (gy == G1 - 1) | (gz == 0)
           | (gz == G1 - 1)).reshape(-1)
    l2g = _local_to_global(ne, N)
    E = ne ** 3
    xyz = np.ascontiguousarray(
        gxyz[l2g].reshape(E, n ** 3, 3).transpose(0, 2, 1))
    glo = l2g.reshape(E, n ** 3).copy()
    bnd = onb[l2g].astype(np.uint8).reshape(E, n ** 3)
    return BoxMesh(ne=ne, N=N, xyz=xyz, glo=glo, bnd=bnd, h=h, gxyz=gxyz, l2g=l2g)


def block_ranks(ne: int, px: int, py: int, pz: int) -> np.ndarray:
    """Rank of every element when the ne^3 box is cut into px x py x pz blocks
    of elements (integer division), ranks numbered x fastest; element
    e = ex + ne (ey + ne ez), as in box_mesh."""
    ez, ey, ex = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    rx, ry, rz = ex * px // ne, ey * py // ne, ez * pz // ne
    return (rx + px * (ry + py * rz)).astype(np.int32).reshape(-1)


def sin3(pts: np.ndarray, scale: float = 1.0) -> np.ndarray:
    """scale * sin(pi x) sin(pi y) sin(pi z) per point."""
    return scale * (np.sin(np.pi * pts[:, 0]) * np.sin(np.pi * pts[:, 1])
                    * np.sin(np.pi * pts[:, 2]))


def manufactured(mesh: BoxMesh):
    """Manufactured Poisson problem: u = sin sin sin, f = 3 pi^2 sin sin sin.

    Returns (f_local, u_exact_local).
    """
    u = sin3(mesh.gxyz)
    f = 3.0 * np.pi ** 2 * u
    return mesh.to_local(f), mesh.to_local(u)


def neumann_cosine_rhs(mesh: BoxMesh, offset: float = 1e-6) -> np.ndarray:
    """f = cos(pi x) cos(pi y) cos(pi z) + offset (local layout).

    The cosine product has zero mean on the unit cube, so with no Dirichlet
    node (pure Neumann Poisson, whose operator annihilates constants) the
    offset is the part of the source outside the operator's range: the
    problem has no solution and the CG residual cannot fall below that
    part.  Used to exercise the stagnation rule."""
    pts = mesh.gxyz
    f = (np.cos(np.pi * pts[:, 0]) * np.cos(np.pi * pts[:, 1]) * np.cos(np.pi * pts[:, 2])
         + offset)
    return mesh.to_local(f)


def random_smooth_rhs(mesh: BoxMesh, seed: int, kmax: int = 4) -> np.ndarray:
    """f = sum_{k in [1,kmax]^3} a_k sin(k1 pi x) sin(k2 pi y) sin(k3 pi z),
    a_k ~ N(0,1)/|k|^2 (seeded), sampled at the nodes (local layout)."""
    rng = np.random.default_rng(seed)
    ks = np.arange(1, kmax + 1)
    a = rng.standard_normal((kmax, kmax, kmax))
    P = mesh.gxyz
    sx = np.sin(np.pi * np.outer(P[:, 0], ks))
    sy = np.sin(np.pi * np.outer(P[:, 1], ks))
    sz = np.sin(np.pi * np.outer(P[:, 2], ks))
    f = np.zeros(len(P))
    for a1 in range(kmax):
        for a2 in range(kmax):
            for a3 in range(kmax):
                k2 = (a1 + 1) ** 2 + (a2 + 1) ** 2 + (a3 + 1) ** 2
                f += (a[a1, a2, a3] / k2) * sx[:, a1] * sy[:, a2] * sz[:, a3]
    return mesh.to_local(f)


def lognormal_k(mesh: BoxMesh, seed: int, corr: float = 0.2, sigma: float = 1.0,
                features: int = 256, chunk: int = 1 << 18) -> np.ndarray:
    """Log-normal coefficient k = exp(g), g a random-Fourier-feature Gaussian
    field with unit-variance squared-exponential-like spectrum:
    g = sigma sqrt(2/M) sum_m cos(w_m . x + b_m), w_m ~ N(0, I/corr^2),
    b_m ~ U(0, 2 pi).  Evaluated per global node, returned in local layout."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((features, 3)) / corr
    b = rng.uniform(0.0, 2.0 * np.pi, size=features)
    P = mesh.gxyz
    g = np.empty(len(P))
    for s in range(0, len(P), chunk):
        ph = P[s:s + chunk] @ w.T + b
        g[s:s + chunk] = np.cos(ph).sum(axis=1)
    g *= sigma * np.sqrt(2.0 / features)
    return mesh.to_local(np.exp(g))


def random_nodal_field(mesh: BoxMesh, seed: int) -> np.ndarray:
    """Seeded N(0,1) value per global node, 0 on the cube boundary, in local
    layout (a rough, continuous field: initial guesses for training data)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(len(mesh.gxyz))
    loc = mesh.to_local(g)
    loc[mesh.bnd.reshape(-1) > 0] = 0.0
    return loc


def he_normal_weights(seed: int, ch: int = 32, cin: int = 2):
    """He-normal initial weights for the two 3x3x3 convolutions (no bias):
    W1 [ch][cin][27] ~ N(0, 2/(27 cin)), W2 [ch][27] ~ N(0, 2/(27 ch))."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((ch, cin, 27)) * np.sqrt(2.0 / (27 * cin))
    W2 = rng.standard_normal((ch, 27)) * np.sqrt(2.0 / (27 * ch))
    return W1, W2


# --------------------------------------------------------------------------
# The workloads (unit cube, homogeneous Dirichlet on the whole boundary)
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    ne: int
    N: int
    deform_seed: int | None
    tol: float
    maxit: int
    rhs: str = "manufactured"   # or "random"
    rhs_seed: int = 0
    k_seed: int | None = None
    helm_h: float = 0.0

    @property
    def E(self) -> int:
        return self.ne ** 3

    @property
    def nloc(self) -> int:
        return self.E * (self.N + 1) ** 3


WORKLOADS = {
    "box4_N7": Workload("box4_N7", 4, 7, None, 1e-10, 100),
    "box16_N9_deformed": Workload("box16_N9_deformed", 16, 9, 2, 1e-10, 5000),
    "box32_N7_deformed": Workload("box32_N7_deformed", 32, 7, 3, 1e-10, 5000),
    "box24_N7_lognormal_helmholtz": Workload("box24_N7_lognormal_helmholtz", 24, 7, None,
                                             1e-10, 10000, rhs="random", rhs_seed=5900,
                                             k_seed=5, helm_h=1.0),
    # undeformed cube Poisson problem of 8000 elements, N = 7, to 1e-9: the
    # size and tolerance of the cube Poisson runs of the Neko evaluation
    # (8192 elements there), for the mixed-precision strategy table; a
    # random smooth source, so that CG has many modes to resolve in FP64 too
    "box20_N7": Workload("box20_N7", 20, 7, None, 1e-9, 10000, rhs="random", rhs_seed=20),
}


def batch_draws(seed: int = 4, count: int = 64):
    """Element counts per direction and orders of the uneven batch:
    ne uniform in {8, 12, 16, 24}, N uniform in {5, 7, 9}; RHS seed 4000+p."""
    rng = np.random.default_rng(seed)
    ne = rng.choice(np.array([8, 12, 16, 24]), size=count)
    N = rng.choice(np.array([5, 7, 9]), size=count)
    return [(int(ne[p]), int(N[p]), 4000 + p) for p in range(count)]
